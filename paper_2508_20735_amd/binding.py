"""ctypes binding of libdfamin (include/dfamin.h).

Argument marshalling only: every step of minimisation, equivalence and
inclusion runs in the library's HIP kernels.  Importing this module does not
load the library; the first call does, and it raises DfaError if the library
is missing (it never falls back to another implementation).

Host variants take numpy arrays; ``*_device`` variants take torch tensors on
the GPU (torch provides device memory and the stream only).
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import numpy as np

from . import build as _build

DFA_OK = 0
DFA_EINVAL = -1
DFA_ENOMEM = -2
DFA_EDEVICE = -3
DFA_EAGAIN = -4
DFA_ELIMIT = -5
DFA_ECANCELED = -6
REQ_MINIMISE = 0
REQ_EQUIVALENT = 1

TC = {"off": 0, "on": 1, "auto": 2}
LOOP = {"host": 0, "chunk": 1, "graph": 2, "persistent": 3}
# block id of a state removed by reachability pruning
UNREACHABLE = 0xFFFFFFFF
# signature rounds (sortPR semantics, hashed) or leader rounds (naivePR)
ALGO = {"signature": 0, "leader": 1, "sort": 2}
# equivalence by refining the disjoint union, or by exploring the product
EQ = {"union": 0, "product": 1}


class DfaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libdfamin status {status}: {message}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("tc_mode", ctypes.c_int32), ("loop_mode", ctypes.c_int32),
                ("start", ctypes.c_uint32), ("max_rounds", ctypes.c_uint32),
                ("chunk", ctypes.c_uint32), ("lds_stage", ctypes.c_int32),
                ("algorithm", ctypes.c_int32), ("prune", ctypes.c_int32),
                ("equiv_method", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_uint32), ("changing_rounds", ctypes.c_uint32),
                ("num_blocks", ctypes.c_uint32), ("k_eff", ctypes.c_uint32),
                ("tc_used", ctypes.c_uint32), ("tc_levels", ctypes.c_uint32),
                ("plain_rounds", ctypes.c_uint32), ("reachable", ctypes.c_uint32),
                ("h2d_ms", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("d2h_ms", ctypes.c_double), ("transitions_refined", ctypes.c_uint64),
                ("algorithmic_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved0"}


class Tuning(ctypes.Structure):
    _fields_ = [("round_grid_cap", ctypes.c_uint32), ("label_grid_cap", ctypes.c_uint32),
                ("label_rounds", ctypes.c_uint32), ("cached_probe", ctypes.c_uint32),
                ("chunk", ctypes.c_uint32), ("hash_bits", ctypes.c_uint32),
                ("batch_lds_states", ctypes.c_uint32), ("insert_pair", ctypes.c_uint32),
                ("slice_min_states", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 7)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double), ("algorithmic_bytes", ctypes.c_uint64),
                ("states", ctypes.c_uint64), ("state_letters", ctypes.c_uint64)]


class BatchStats(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint32), ("rounds", ctypes.c_uint32),
                ("k_eff", ctypes.c_uint32), ("reserved0", ctypes.c_uint32),
                ("h2d_ms", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("d2h_ms", ctypes.c_double), ("states", ctypes.c_uint64),
                ("transitions_refined", ctypes.c_uint64), ("algorithmic_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved0"}


class Quotient(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_void_p), ("accepting", ctypes.c_void_p),
                ("num_blocks", ctypes.c_uint32), ("start", ctypes.c_uint32)]


class View(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("k", ctypes.c_uint32), ("start", ctypes.c_uint32),
                ("delta", ctypes.c_void_p), ("accepting", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("lanes", ctypes.c_uint32),
                ("max_group", ctypes.c_uint32), ("batch_max_states", ctypes.c_uint32),
                ("batch_round_budget", ctypes.c_uint32), ("tc_mode", ctypes.c_int32),
                ("paused", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 8)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_uint32), ("a", View),
                ("b", View)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("verdict", ctypes.c_int32),
                ("num_blocks", ctypes.c_uint32), ("rounds", ctypes.c_uint32),
                ("blocks", ctypes.POINTER(ctypes.c_uint32)), ("n", ctypes.c_uint32),
                ("batched", ctypes.c_uint32), ("queue_ms", ctypes.c_double),
                ("service_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("h2d_ms", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("d2h_ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("pending", ctypes.c_uint64),
                ("batched_groups", ctypes.c_uint64), ("solo_runs", ctypes.c_uint64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("uptime_s", ctypes.c_double),
                ("requests_per_s", ctypes.c_double), ("hbm_in_use", ctypes.c_uint64),
                ("hbm_budget", ctypes.c_uint64), ("waiting_threads", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


EXPORTS = sorted(["dfa_options_default", "dfa_minimise", "dfa_minimise_device",
                  "dfa_minimise_device_fixed",
                  "dfa_equivalent", "dfa_equivalent_device", "dfa_included",
                  "dfa_included_device", "dfa_last_error", "dfa_device_info",
                  "dfa_tuning_default", "dfa_get_tuning", "dfa_set_tuning",
                  "dfa_profile_enable", "dfa_profile_read", "dfa_profile_only",
                  "dfa_minimise_batch", "dfa_minimise_batch_device", "dfa_equivalent_batch",
                  "dfa_equivalent_batch_device", "dfa_server_config_default",
                  "dfa_server_create", "dfa_server_submit", "dfa_server_poll",
                  "dfa_server_wait", "dfa_result_release", "dfa_server_get_stats",
                  "dfa_server_destroy", "dfa_server_footprint", "dfa_server_resume"])

_lock = threading.Lock()
_lib = None


def library_path() -> str:
    return _build.LIB


def load(build_if_missing: bool = True):
    """Load libdfamin.so (building it first only if it does not exist)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_build.LIB):
            if not build_if_missing:
                raise DfaError(DFA_EDEVICE, f"{_build.LIB} is not built")
            _build.build()
        # torch ships its own HIP runtime with the same soname as ROCm's; load
        # it first so that libdfamin binds to it and the process keeps one
        # HIP runtime (two runtimes in one process do not share the device)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(_build.LIB)
        vp, u32, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int
        P = ctypes.POINTER
        lib.dfa_options_default.argtypes = [P(Options)]
        lib.dfa_options_default.restype = None
        lib.dfa_minimise.argtypes = [u32, u32, vp, vp, vp, P(Quotient), P(Options), P(Stats)]
        lib.dfa_minimise_device.argtypes = [u32, u32, vp, vp, vp, P(Quotient), P(Options),
                                            P(Stats), vp]
        lib.dfa_minimise_device_fixed.argtypes = [u32, u32, vp, vp, vp, P(Quotient),
                                                  P(Options), P(Stats), vp]
        lib.dfa_equivalent.argtypes = [P(View), P(View), P(i32), P(Options), P(Stats)]
        lib.dfa_equivalent_device.argtypes = [P(View), P(View), P(i32), P(Options), P(Stats), vp]
        lib.dfa_included.argtypes = [P(View), P(View), P(i32), P(ctypes.c_uint64), P(Options),
                                     P(Stats)]
        lib.dfa_included_device.argtypes = [P(View), P(View), P(i32), P(ctypes.c_uint64),
                                            P(Options), P(Stats), vp]
        lib.dfa_last_error.argtypes = []
        lib.dfa_last_error.restype = ctypes.c_char_p
        lib.dfa_device_info.argtypes = [ctypes.c_char_p, ctypes.c_size_t, P(i32),
                                        P(ctypes.c_size_t)]
        lib.dfa_tuning_default.argtypes = [P(Tuning)]
        lib.dfa_tuning_default.restype = None
        lib.dfa_get_tuning.argtypes = [P(Tuning)]
        lib.dfa_set_tuning.argtypes = [P(Tuning)]
        lib.dfa_minimise_batch.argtypes = [u32, P(View), vp, vp, vp, vp, P(Options),
                                           P(BatchStats)]
        lib.dfa_minimise_batch_device.argtypes = [u32, P(View), vp, vp, vp, vp, P(Options),
                                                  P(BatchStats), vp]
        lib.dfa_equivalent_batch.argtypes = [u32, P(View), P(View), vp, P(Options),
                                             P(BatchStats)]
        lib.dfa_equivalent_batch_device.argtypes = [u32, P(View), P(View), vp, P(Options),
                                                    P(BatchStats), vp]
        lib.dfa_server_config_default.argtypes = [P(ServerConfig)]
        lib.dfa_server_config_default.restype = None
        lib.dfa_server_create.argtypes = [P(ServerConfig)]
        lib.dfa_server_create.restype = vp
        lib.dfa_server_submit.argtypes = [vp, P(Request), P(ctypes.c_uint64)]
        lib.dfa_server_footprint.argtypes = [vp, P(Request), P(ctypes.c_size_t)]
        lib.dfa_server_footprint.restype = i32
        lib.dfa_server_poll.argtypes = [vp, ctypes.c_uint64, P(Result)]
        lib.dfa_server_wait.argtypes = [vp, ctypes.c_uint64, P(Result)]
        lib.dfa_result_release.argtypes = [vp, ctypes.c_uint64]
        lib.dfa_server_get_stats.argtypes = [vp, P(ServerStats)]
        lib.dfa_server_resume.argtypes = [vp]
        lib.dfa_server_destroy.argtypes = [vp]
        lib.dfa_server_destroy.restype = None
        lib.dfa_profile_enable.argtypes = [i32]
        lib.dfa_profile_read.argtypes = [P(KernelTime), i32, P(i32)]
        lib.dfa_profile_only.argtypes = [ctypes.c_char_p]
        for fn in ("dfa_minimise", "dfa_minimise_device", "dfa_minimise_device_fixed",
                   "dfa_equivalent",
                   "dfa_equivalent_device", "dfa_included", "dfa_included_device",
                   "dfa_device_info", "dfa_get_tuning", "dfa_set_tuning",
                   "dfa_profile_enable", "dfa_profile_read", "dfa_minimise_batch",
                   "dfa_minimise_batch_device", "dfa_equivalent_batch",
                   "dfa_equivalent_batch_device", "dfa_server_submit", "dfa_server_poll",
                   "dfa_server_wait", "dfa_result_release", "dfa_server_get_stats",
                   "dfa_server_resume"):
            getattr(lib, fn).restype = i32
        _lib = lib
        return lib


def _check(rc: int, allow=()) -> int:
    if rc != DFA_OK and rc not in allow:
        msg = load().dfa_last_error().decode(errors="replace")
        raise DfaError(rc, msg)
    return rc


def options(tc: str = "auto", loop: str = "graph", start: int = 0, max_rounds: int = 0,
            chunk: int = 0, lds_stage=2, algorithm: str = "signature",
            prune: bool = False, method: str = "union") -> Options:
    o = Options()
    load().dfa_options_default(ctypes.byref(o))
    o.tc_mode = TC[tc]
    o.loop_mode = LOOP[loop]
    o.start = start
    o.max_rounds = max_rounds
    o.chunk = chunk
    # True/False select always/never; 2 (the default) lets each round decide
    o.lds_stage = int(lds_stage) if not isinstance(lds_stage, bool) else (1 if lds_stage else 0)
    o.algorithm = ALGO[algorithm]
    o.prune = 1 if prune else 0
    o.equiv_method = EQ[method]
    return o


def default_tuning() -> dict:
    t = Tuning()
    load().dfa_tuning_default(ctypes.byref(t))
    return t.as_dict()


def get_tuning() -> dict:
    t = Tuning()
    _check(load().dfa_get_tuning(ctypes.byref(t)))
    return t.as_dict()


def set_tuning(**values) -> dict:
    """Update fields of the current device's tuning; returns the new tuning."""
    t = Tuning()
    _check(load().dfa_get_tuning(ctypes.byref(t)))
    for key, value in values.items():
        if key not in t.as_dict():
            raise KeyError(key)
        setattr(t, key, int(value))
    _check(load().dfa_set_tuning(ctypes.byref(t)))
    return t.as_dict()


def profile_enable(on: bool = True) -> None:
    """Start (and clear) or stop per-kernel event timing in the library."""
    _check(load().dfa_profile_enable(1 if on else 0))


def profile_only(name: str | None) -> None:
    """Time only the round kernel `name` (e.g. "k_signature"); None: all."""
    _check(load().dfa_profile_only(name.encode() if name else None))


def profile_read() -> dict:
    """{kernel name: {launches, total_ms, algorithmic_bytes, states, state_letters}}
    since profile_enable(True)."""
    lib = load()
    count = ctypes.c_int()
    _check(lib.dfa_profile_read(None, 0, ctypes.byref(count)))
    buf = (KernelTime * max(count.value, 1))()
    _check(lib.dfa_profile_read(buf, count.value, ctypes.byref(count)))
    return {buf[i].name.decode(): {"launches": int(buf[i].launches),
                                   "total_ms": float(buf[i].total_ms),
                                   "algorithmic_bytes": int(buf[i].algorithmic_bytes),
                                   "states": int(buf[i].states),
                                   "state_letters": int(buf[i].state_letters)}
            for i in range(count.value)}


def device_info() -> dict:
    name = ctypes.create_string_buffer(256)
    cu = ctypes.c_int()
    mem = ctypes.c_size_t()
    _check(load().dfa_device_info(name, 256, ctypes.byref(cu), ctypes.byref(mem)))
    return {"name": name.value.decode(), "compute_units": cu.value, "hbm_bytes": mem.value}


def _host_arrays(delta, accepting):
    d = np.ascontiguousarray(delta, dtype=np.uint32)
    if d.ndim != 2:
        raise ValueError("delta must be [n, k]")
    a = np.ascontiguousarray(np.asarray(accepting) != 0, dtype=np.uint8)
    if a.shape != (d.shape[0],):
        raise ValueError("accepting must have n entries")
    return d, a


@dataclass
class MinimiseResult:
    block: object          # numpy array (host call) or torch tensor (device call)
    stats: dict
    quotient: tuple | None = None  # (num_blocks, qdelta [B,k], qacc [B], qstart)


def minimise(delta, accepting, *, tc: str = "auto", loop: str = "graph", start: int = 0,
             max_rounds: int = 0, chunk: int = 0, lds_stage=2,
             quotient: bool = False, algorithm: str = "signature",
             prune: bool = False) -> MinimiseResult:
    """dfa_minimise on host arrays.  With ``prune``, only the states reachable
    from ``start`` are partitioned (the others get UNREACHABLE)."""
    d, a = _host_arrays(delta, accepting)
    n, k = d.shape
    block = np.empty(n, dtype=np.uint32)
    o = options(tc, loop, start, max_rounds, chunk, lds_stage, algorithm, prune)
    st = Stats()
    q = None
    if quotient:
        qd = np.empty((n, k), dtype=np.uint32)
        qa = np.empty(n, dtype=np.uint8)
        q = Quotient(qd.ctypes.data, qa.ctypes.data, 0, 0)
    rc = load().dfa_minimise(n, k, d.ctypes.data, a.ctypes.data, block.ctypes.data,
                             ctypes.byref(q) if q is not None else None, ctypes.byref(o),
                             ctypes.byref(st))
    _check(rc)
    res = MinimiseResult(block, st.as_dict())
    if q is not None:
        B = q.num_blocks
        res.quotient = (B, qd[:B], qa[:B], q.start)
    return res


def _stream_ptr(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(getattr(stream, "cuda_stream", stream))


def _check_device_tensor(t, dtype_name: str, numel: int, what: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{what} must be a torch tensor on the GPU")
    if str(t.dtype) != dtype_name or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{what} must be a contiguous {dtype_name} tensor of {numel} elements")


def minimise_device(delta, accepting, block_out=None, *, tc: str = "auto", loop: str = "graph",
                    start: int = 0, max_rounds: int = 0, chunk: int = 0, lds_stage=2,
                    quotient: bool = False, stream=None,
                    algorithm: str = "signature", prune: bool = False) -> MinimiseResult:
    """dfa_minimise_device on torch GPU tensors: delta int32/uint32 [n, k]
    (row-major), accepting uint8 [n]; block_out int32 [n] (allocated if None)."""
    return _minimise_device("dfa_minimise_device", delta, accepting, block_out, tc, loop, start,
                            max_rounds, chunk, lds_stage, quotient, stream, algorithm, prune)


def minimise_device_fixed(delta, accepting, block_out=None, *, tc: str = "auto",
                          loop: str = "graph", start: int = 0, max_rounds: int = 0,
                          chunk: int = 0, lds_stage=2, quotient: bool = False, stream=None,
                          algorithm: str = "signature", prune: bool = False) -> MinimiseResult:
    """dfa_minimise_device_fixed (no device allocation inside the library: its
    workspace is a fixed device array) on torch GPU tensors; arguments as
    minimise_device.  The tensors it is given, and block_out / the quotient
    when they are allocated here, come from the caller's side."""
    return _minimise_device("dfa_minimise_device_fixed", delta, accepting, block_out, tc, loop,
                            start, max_rounds, chunk, lds_stage, quotient, stream, algorithm,
                            prune)


def _minimise_device(entry, delta, accepting, block_out, tc, loop, start, max_rounds, chunk,
                     lds_stage, quotient, stream, algorithm, prune) -> MinimiseResult:
    import torch
    n, k = delta.shape
    if delta.dtype not in (torch.int32, torch.uint32):
        raise ValueError("delta must be int32 or uint32")
    _check_device_tensor(delta, str(delta.dtype), n * k, "delta")
    _check_device_tensor(accepting, "torch.uint8", n, "accepting")
    if block_out is None:
        block_out = torch.empty(n, dtype=torch.int32, device=delta.device)
    _check_device_tensor(block_out, str(block_out.dtype), n, "block_out")
    o = options(tc, loop, start, max_rounds, chunk, lds_stage, algorithm, prune)
    st = Stats()
    q = None
    if quotient:
        qd = torch.empty((n, k), dtype=torch.int32, device=delta.device)
        qa = torch.empty(n, dtype=torch.uint8, device=delta.device)
        q = Quotient(qd.data_ptr(), qa.data_ptr(), 0, 0)
    rc = getattr(load(), entry)(n, k, delta.data_ptr(), accepting.data_ptr(),
                                block_out.data_ptr(),
                                ctypes.byref(q) if q is not None else None, ctypes.byref(o),
                                ctypes.byref(st), _stream_ptr(stream))
    _check(rc)
    res = MinimiseResult(block_out, st.as_dict())
    if q is not None:
        B = q.num_blocks
        res.quotient = (B, qd[:B], qa[:B], q.start)
    return res


def _view_host(dfa) -> tuple[View, tuple]:
    d, a = _host_arrays(dfa.delta, dfa.accepting)
    v = View(d.shape[0], d.shape[1], int(dfa.start), d.ctypes.data, a.ctypes.data)
    return v, (d, a)


def _view_device(delta, accepting, start) -> View:
    n, k = delta.shape
    _check_device_tensor(delta, str(delta.dtype), n * k, "delta")
    _check_device_tensor(accepting, "torch.uint8", n, "accepting")
    return View(n, k, int(start), delta.data_ptr(), accepting.data_ptr())


def equivalent(A, B, *, tc: str = "auto", loop: str = "graph", max_rounds: int = 0,
               chunk: int = 0, lds_stage=2, algorithm: str = "signature",
               method: str = "union") -> tuple[bool, dict]:
    """dfa_equivalent on two host DFAs (objects with delta, accepting, start).
    method "union" refines the disjoint union; "product" explores the product
    (stats: rounds = levels, reachable = pairs visited)."""
    va, keep_a = _view_host(A)
    vb, keep_b = _view_host(B)
    o = options(tc, loop, 0, max_rounds, chunk, lds_stage, algorithm, method=method)
    v = ctypes.c_int()
    st = Stats()
    _check(load().dfa_equivalent(ctypes.byref(va), ctypes.byref(vb), ctypes.byref(v),
                                 ctypes.byref(o), ctypes.byref(st)))
    return bool(v.value), st.as_dict()


def equivalent_device(dA, accA, sA, dB, accB, sB, *, tc: str = "auto", loop: str = "graph",
                      max_rounds: int = 0, chunk: int = 0, lds_stage=2,
                      stream=None, algorithm: str = "signature",
                      method: str = "union") -> tuple[bool, dict]:
    va = _view_device(dA, accA, sA)
    vb = _view_device(dB, accB, sB)
    o = options(tc, loop, 0, max_rounds, chunk, lds_stage, algorithm, method=method)
    v = ctypes.c_int()
    st = Stats()
    _check(load().dfa_equivalent_device(ctypes.byref(va), ctypes.byref(vb), ctypes.byref(v),
                                        ctypes.byref(o), ctypes.byref(st), _stream_ptr(stream)))
    return bool(v.value), st.as_dict()


def included(A, B) -> tuple[bool, int, dict]:
    """dfa_included on two host DFAs: (verdict, pairs visited, stats)."""
    va, keep_a = _view_host(A)
    vb, keep_b = _view_host(B)
    v = ctypes.c_int()
    cnt = ctypes.c_uint64()
    st = Stats()
    _check(load().dfa_included(ctypes.byref(va), ctypes.byref(vb), ctypes.byref(v),
                               ctypes.byref(cnt), None, ctypes.byref(st)))
    return bool(v.value), int(cnt.value), st.as_dict()


def included_device(dA, accA, sA, dB, accB, sB, stream=None) -> tuple[bool, int, dict]:
    va = _view_device(dA, accA, sA)
    vb = _view_device(dB, accB, sB)
    v = ctypes.c_int()
    cnt = ctypes.c_uint64()
    st = Stats()
    _check(load().dfa_included_device(ctypes.byref(va), ctypes.byref(vb), ctypes.byref(v),
                                      ctypes.byref(cnt), None, ctypes.byref(st),
                                      _stream_ptr(stream)))
    return bool(v.value), int(cnt.value), st.as_dict()


# --------------------------------------------------------------------------- batches

def _views_host(dfas):
    keep, views = [], (View * len(dfas))()
    for i, d in enumerate(dfas):
        v, arrays = _view_host(d)
        views[i] = v
        keep.append(arrays)
    return views, keep


def minimise_batch(dfas, *, tc: str = "auto", loop: str = "graph", max_rounds: int = 0,
                   chunk: int = 0, lds_stage=2, offsets=None, algorithm: str = "signature"):
    """dfa_minimise_batch on host DFAs.  Returns (list of block arrays,
    num_blocks array, rounds array, stats)."""
    count = len(dfas)
    views, keep = _views_host(dfas)
    sizes = np.array([int(v.n) for v in views], dtype=np.uint64)
    if offsets is None:
        offs = None
        total = int(sizes.sum())
    else:
        offs = np.ascontiguousarray(offsets, dtype=np.uint64)
        total = int((offs + sizes).max())
    out = np.zeros(total, dtype=np.uint32)
    nb = np.empty(count, dtype=np.uint32)
    rounds = np.empty(count, dtype=np.uint32)
    o = options(tc, loop, 0, max_rounds, chunk, lds_stage, algorithm)
    st = BatchStats()
    _check(load().dfa_minimise_batch(count, views, out.ctypes.data,
                                     None if offs is None else offs.ctypes.data, nb.ctypes.data,
                                     rounds.ctypes.data, ctypes.byref(o), ctypes.byref(st)))
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.uint64) if offs is None \
        else offs
    blocks = [out[int(starts[i]):int(starts[i]) + int(sizes[i])] for i in range(count)]
    return blocks, nb, rounds, st.as_dict()


_VIEW_NP = np.dtype({"names": ["n", "k", "start", "delta", "accepting"],
                     "formats": [np.uint32, np.uint32, np.uint32, np.uint64, np.uint64],
                     "offsets": [View.n.offset, View.k.offset, View.start.offset,
                                 View.delta.offset, View.accepting.offset],
                     "itemsize": ctypes.sizeof(View)})


class PackedBatch:
    """A batch of DFAs held in two flat GPU tensors: delta_flat (int32, the
    row-major transition tables one after another, n_i * k_i entries each)
    and acc_flat (uint8, the acceptance arrays one after another).  The
    dfa_view array of the batched calls is computed in bulk from the sizes
    (no per-DFA Python work), so a call on thousands of DFAs costs the
    library's time, not the binding's."""

    def __init__(self, delta_flat, acc_flat, ns, ks, starts=None):
        ns = np.asarray(ns, dtype=np.uint64)
        ks = np.asarray(ks, dtype=np.uint64)
        count = len(ns)
        if len(ks) != count or count == 0:
            raise ValueError("ns and ks must be non-empty and of the same length")
        if (ns == 0).any() or (ks == 0).any():
            raise ValueError("every DFA needs at least one state and one letter")
        cells = ns * ks
        _check_device_tensor(delta_flat, str(delta_flat.dtype), int(cells.sum()), "delta_flat")
        if str(delta_flat.dtype) not in ("torch.int32", "torch.uint32"):
            raise ValueError("delta_flat must be an int32 tensor")
        _check_device_tensor(acc_flat, "torch.uint8", int(ns.sum()), "acc_flat")
        arr = np.zeros(count, dtype=_VIEW_NP)
        arr["n"] = ns
        arr["k"] = ks
        arr["start"] = 0 if starts is None else np.asarray(starts, dtype=np.uint32)
        arr["delta"] = delta_flat.data_ptr() + 4 * (np.cumsum(cells) - cells)
        arr["accepting"] = acc_flat.data_ptr() + (np.cumsum(ns) - ns)
        self._arr = arr
        self._keep = (delta_flat, acc_flat)
        self.views = (View * count).from_buffer(arr)
        self.count = count
        self.states = int(ns.sum())

    @classmethod
    def from_dfas(cls, dfas, device="cuda:0"):
        """Packs host DFAs (objects with delta, accepting, start) onto the GPU."""
        import torch
        delta = np.concatenate([np.ascontiguousarray(d.delta, dtype=np.uint32).ravel()
                                for d in dfas])
        acc = np.concatenate([np.ascontiguousarray(d.accepting, dtype=np.uint8).ravel()
                              for d in dfas])
        dev = torch.device(device)
        return cls(torch.from_numpy(delta.view(np.int32)).to(dev), torch.from_numpy(acc).to(dev),
                   [d.delta.shape[0] for d in dfas], [d.delta.shape[1] for d in dfas],
                   [d.start for d in dfas])


def _batch_views(deltas, accs=None, starts=None):
    if isinstance(deltas, PackedBatch):
        return deltas.views, deltas.count
    count = len(deltas)
    views = (View * count)()
    for i, (d, a) in enumerate(zip(deltas, accs)):
        views[i] = _view_device(d, a, 0 if starts is None else starts[i])
    return views, count


def minimise_batch_device(deltas, accs, out, *, tc: str = "auto", loop: str = "graph",
                          lds_stage=2, stream=None):
    """dfa_minimise_batch_device: deltas / accs are lists of GPU tensors (or
    deltas a PackedBatch and accs None), out a GPU int32 tensor with room for
    all states (packed in order)."""
    views, count = _batch_views(deltas, accs)
    nb = np.empty(count, dtype=np.uint32)
    rounds = np.empty(count, dtype=np.uint32)
    o = options(tc, loop, 0, 0, 0, lds_stage)
    st = BatchStats()
    _check(load().dfa_minimise_batch_device(count, views, out.data_ptr(), None, nb.ctypes.data,
                                            rounds.ctypes.data, ctypes.byref(o),
                                            ctypes.byref(st), _stream_ptr(stream)))
    return nb, rounds, st.as_dict()


def equivalent_batch(pairs, *, tc: str = "auto", loop: str = "graph", max_rounds: int = 0,
                     lds_stage=2):
    """dfa_equivalent_batch on host DFA pairs: (verdict array, stats)."""
    count = len(pairs)
    va, keep_a = _views_host([p[0] for p in pairs])
    vb, keep_b = _views_host([p[1] for p in pairs])
    verdicts = np.empty(count, dtype=np.int32)
    o = options(tc, loop, 0, max_rounds, 0, lds_stage)
    st = BatchStats()
    _check(load().dfa_equivalent_batch(count, va, vb, verdicts.ctypes.data, ctypes.byref(o),
                                       ctypes.byref(st)))
    return verdicts.astype(bool), st.as_dict()


def equivalent_batch_device(a_list, b_list, *, loop: str = "graph", lds_stage=2, stream=None):
    """a_list / b_list: lists of (delta tensor, accepting tensor, start), or
    two PackedBatch of the same count."""
    if isinstance(a_list, PackedBatch) != isinstance(b_list, PackedBatch):
        raise ValueError("both operand lists must be PackedBatch, or neither")
    if isinstance(a_list, PackedBatch):
        if a_list.count != b_list.count:
            raise ValueError("the two PackedBatch must hold the same number of DFAs")
        va, vb, count = a_list.views, b_list.views, a_list.count
    else:
        count = len(a_list)
        va, vb = (View * count)(), (View * count)()
        for i in range(count):
            va[i] = _view_device(*a_list[i])
            vb[i] = _view_device(*b_list[i])
    verdicts = np.empty(count, dtype=np.int32)
    o = options("auto", loop, 0, 0, 0, lds_stage)
    st = BatchStats()
    _check(load().dfa_equivalent_batch_device(count, va, vb, verdicts.ctypes.data,
                                              ctypes.byref(o), ctypes.byref(st),
                                              _stream_ptr(stream)))
    return verdicts.astype(bool), st.as_dict()


# --------------------------------------------------------------------------- serving

class Server:
    """dfa_server_*: continuous batching of minimise / equivalence requests."""

    def __init__(self, hbm_budget: int = 0, lanes: int = 4, max_group: int = 512,
                 batch_max_states: int = 1 << 18, batch_round_budget: int = 12,
                 tc: str = "auto", paused: bool = False):
        lib = load()
        cfg = ServerConfig()
        lib.dfa_server_config_default(ctypes.byref(cfg))
        cfg.hbm_budget = hbm_budget
        cfg.lanes = lanes
        cfg.max_group = max_group
        cfg.batch_max_states = batch_max_states
        cfg.batch_round_budget = batch_round_budget
        cfg.tc_mode = TC[tc]
        cfg.paused = 1 if paused else 0
        h = lib.dfa_server_create(ctypes.byref(cfg))
        if not h:
            raise DfaError(DFA_EINVAL, lib.dfa_last_error().decode(errors="replace"))
        self._h = h
        self._lib = lib

    def submit_minimise(self, dfa) -> int:
        return self._submit(REQ_MINIMISE, dfa, None)

    def submit_equivalent(self, a, b) -> int:
        return self._submit(REQ_EQUIVALENT, a, b)

    def _request(self, kind, a, b):
        req = Request()
        req.kind = kind
        va, keep_a = _view_host(a)
        req.a = va
        keep = [keep_a]
        if b is not None:
            vb, keep_b = _view_host(b)
            req.b = vb
            keep.append(keep_b)
        return req, keep

    def _submit(self, kind, a, b) -> int:
        req, keep = self._request(kind, a, b)
        t = ctypes.c_uint64()
        _check(self._lib.dfa_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        return int(t.value)

    def footprint(self, a, b=None) -> int:
        """Device bytes the server charges for running this minimise (b None)
        or equivalence request alone (dfa_server_footprint)."""
        req, keep = self._request(REQ_MINIMISE if b is None else REQ_EQUIVALENT, a, b)
        out = ctypes.c_size_t()
        _check(self._lib.dfa_server_footprint(self._h, ctypes.byref(req), ctypes.byref(out)))
        return int(out.value)

    def _convert(self, r: Result) -> dict:
        out = {"status": r.status, "verdict": bool(r.verdict), "num_blocks": r.num_blocks,
               "rounds": r.rounds, "batched": bool(r.batched), "queue_ms": r.queue_ms,
               "service_ms": r.service_ms, "latency_ms": r.latency_ms, "h2d_ms": r.h2d_ms,
               "device_ms": r.device_ms, "d2h_ms": r.d2h_ms, "blocks": None}
        if r.blocks:
            out["blocks"] = np.ctypeslib.as_array(r.blocks, shape=(r.n,)).copy()
        return out

    def poll(self, ticket: int):
        """Result dict, or None while the request is not finished."""
        r = Result()
        rc = self._lib.dfa_server_poll(self._h, ticket, ctypes.byref(r))
        if rc == DFA_EAGAIN:
            return None
        _check(rc)
        return self._convert(r)

    def wait(self, ticket: int, release: bool = True) -> dict:
        r = Result()
        _check(self._lib.dfa_server_wait(self._h, ticket, ctypes.byref(r)))
        out = self._convert(r)
        if release:
            self.release(ticket)
        return out

    def release(self, ticket: int) -> None:
        _check(self._lib.dfa_result_release(self._h, ticket))

    def resume(self) -> None:
        """Lets the lanes of a server created paused take requests."""
        _check(self._lib.dfa_server_resume(self._h))

    def stats(self) -> dict:
        st = ServerStats()
        _check(self._lib.dfa_server_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self) -> None:
        if self._h:
            self._lib.dfa_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
