"""Sequential CPU oracle for DFA minimisation, equivalence and inclusion.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  The product library never imports, links or calls
anything in this package, and this package imports nothing from the product.

The arithmetic lives in ``oracle.c`` (plain C, compiled with gcc) and in
``words.py`` (brute-force word enumeration, numpy).  This module only
marshals numpy arrays into the C functions.

Every function follows a passage of Heemstra, Martens and Wijs, "Evaluating
Massively Parallel Algorithms for DFA Minimisation, Equivalence Checking and
Inclusion Checking":

* ``moore``          -- signature refinement with the semantics of sortPR
                        (Section 3.3, Algorithm 4), with round counts;
* ``naive_pr``       -- leader-based refinement naivePR (Section 3.2,
                        Algorithm 2), with iteration counts; ``naive_pr_tc`` is
                        transPR (Algorithm 5 followed by naivePR);
* ``hopcroft``       -- Hopcroft's n log n algorithm (cited in Section 1);
* ``table_fill``     -- the Apart fixpoint computed by trans (Section 3.1,
                        Algorithm 1), sequentially;
* ``pointer_jump``   -- the partial transitive closure of transPR
                        (Section 3.4, Algorithm 5);
* ``equiv_hk``       -- Hopcroft-Karp with union-find (Section 4, Algorithm 6);
* ``product_bfs``    -- the naive pair-set Hopcroft-Karp of Section 4, for
                        equivalence and for inclusion (changed acceptance test);
* ``quotient``       -- the quotient DFA of a canonical partition (Section 2);
* ``reachable``, ``minimise_reachable`` -- breadth-first reachability and the
                        minimisation of the reachable part (Section 2 assumes
                        every state reachable; this is the usual definition).

Parity is pinned for every function (see tests/test_oracle_*.py): nothing here
is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "liboracle.so")

_lock = threading.Lock()
_lib = None

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = False) -> str:
    """Compile oracle.c into oracle/_build/liboracle.so with gcc -O3."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-shared",
                           "-fPIC", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        lib = ctypes.CDLL(_LIB)
        lib.orc_canonicalise.argtypes = [ctypes.c_uint32, _u32p, _u32p]
        lib.orc_moore_round.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u32p, _u32p, _u32p]
        lib.orc_moore_round.restype = ctypes.c_uint32
        lib.orc_moore.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u32p, _u8p, _u32p,
                                  _u32p, _u32p, _u32p, ctypes.c_uint32]
        lib.orc_naive_pr.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u32p, _u8p, _u32p,
                                     _u32p, _u32p, _u32p, ctypes.c_uint32]
        lib.orc_hopcroft.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u32p, _u8p, _u32p, _u32p]
        lib.orc_table_fill.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u32p, _u8p, _u8p, _u32p]
        lib.orc_pointer_jump.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u32p,
                                         ctypes.c_uint32, _u32p]
        lib.orc_floor_log2.argtypes = [ctypes.c_uint32]
        lib.orc_floor_log2.restype = ctypes.c_uint32
        lib.orc_quotient.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u32p, _u8p, _u32p,
                                     ctypes.c_uint32, _u32p, _u32p, _u8p, _u32p]
        dfa_args = [ctypes.c_uint32, ctypes.c_uint32, _u32p, _u8p, ctypes.c_uint32]
        lib.orc_equiv_hk.argtypes = dfa_args + dfa_args + [ctypes.POINTER(ctypes.c_int)]
        lib.orc_product_bfs.argtypes = dfa_args + dfa_args + [
            ctypes.c_int, ctypes.POINTER(ctypes.c_int), _u64p]
        lib.orc_reachable.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u32p, ctypes.c_uint32,
                                      _u8p, _u32p]
        lib.orc_minimise_reachable.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u32p, _u8p,
                                               ctypes.c_uint32, _u32p, _u32p, _u32p]
        lib.orc_minimise_many.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint32, _u32p, _u8p, _u32p]
        for fn in ("orc_canonicalise", "orc_moore", "orc_naive_pr", "orc_hopcroft", "orc_table_fill",
                   "orc_pointer_jump", "orc_quotient", "orc_equiv_hk", "orc_product_bfs",
                   "orc_minimise_many", "orc_reachable", "orc_minimise_reachable"):
            getattr(lib, fn).restype = ctypes.c_int
        _lib = lib
        return lib


_ELIMIT = -3


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def _as_delta(delta) -> np.ndarray:
    d = np.ascontiguousarray(delta, dtype=np.uint32)
    if d.ndim != 2:
        raise ValueError("delta must be a 2-D array [n, k]")
    return d


def _as_acc(acc) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(acc) != 0, dtype=np.uint8)


def _p32(a: np.ndarray):
    return a.ctypes.data_as(_u32p)


def _p8(a: np.ndarray):
    return a.ctypes.data_as(_u8p)


def canonicalise(ids) -> np.ndarray:
    """out[q] = smallest state carrying the same label as q."""
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    out = np.empty_like(ids)
    _check(_load().orc_canonicalise(len(ids), _p32(ids), _p32(out)), "canonicalise")
    return out


def moore_round(delta, block) -> tuple[np.ndarray, int]:
    """One signature round from canonical partition ``block``."""
    d = _as_delta(delta)
    b = np.ascontiguousarray(block, dtype=np.uint32)
    out = np.empty_like(b)
    c = _load().orc_moore_round(d.shape[0], d.shape[1], _p32(d), _p32(b), _p32(out))
    if c == 0:
        raise OracleError("moore_round: out of memory")
    return out, int(c)


def moore(delta, acc, max_rounds: int = 0):
    """Signature refinement.  Returns (block, num_blocks, rounds, changing_rounds)."""
    d = _as_delta(delta)
    a = _as_acc(acc)
    n, k = d.shape
    block = np.empty(n, dtype=np.uint32)
    nb, rounds, changing = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    rc = _load().orc_moore(n, k, _p32(d), _p8(a), _p32(block), ctypes.byref(nb),
                           ctypes.byref(rounds), ctypes.byref(changing), max_rounds)
    _check(rc, "moore")
    return block, nb.value, rounds.value, changing.value


def naive_pr(delta, acc, max_rounds: int = 0, partial: bool = False):
    """Leader-based refinement (naivePR).  Returns (block, num_blocks, rounds,
    changing_rounds); the leaders are the smallest members, so ``block`` is
    canonical.  With ``partial``, reaching ``max_rounds`` returns the
    partition after that many rounds instead of raising."""
    d = _as_delta(delta)
    a = _as_acc(acc)
    n, k = d.shape
    block = np.empty(n, dtype=np.uint32)
    nb, rounds, changing = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    rc = _load().orc_naive_pr(n, k, _p32(d), _p8(a), _p32(block), ctypes.byref(nb),
                              ctypes.byref(rounds), ctypes.byref(changing), max_rounds)
    if not (partial and rc == _ELIMIT):
        _check(rc, "naive_pr")
    return block, nb.value, rounds.value, changing.value


def naive_pr_tc(delta, acc, levels: int | None = None):
    """The paper's transPR: naivePR over the closure letters."""
    ext = pointer_jump(delta, levels)
    return naive_pr(ext, acc)


def hopcroft(delta, acc) -> tuple[np.ndarray, int]:
    """Hopcroft minimisation.  Returns (canonical block, num_blocks)."""
    d = _as_delta(delta)
    a = _as_acc(acc)
    n, k = d.shape
    block = np.empty(n, dtype=np.uint32)
    nb = ctypes.c_uint32()
    _check(_load().orc_hopcroft(n, k, _p32(d), _p8(a), _p32(block), ctypes.byref(nb)),
           "hopcroft")
    return block, nb.value


def table_fill(delta, acc) -> tuple[np.ndarray, int]:
    """Apart relation (n x n bool) and the number of marking sweeps."""
    d = _as_delta(delta)
    a = _as_acc(acc)
    n, k = d.shape
    apart = np.empty((n, n), dtype=np.uint8)
    sweeps = ctypes.c_uint32()
    _check(_load().orc_table_fill(n, k, _p32(d), _p8(a), _p8(apart), ctypes.byref(sweeps)),
           "table_fill")
    return apart.astype(bool), sweeps.value


def floor_log2(n: int) -> int:
    return int(_load().orc_floor_log2(n))


def pointer_jump(delta, levels: int | None = None) -> np.ndarray:
    """Extended table [n, k*(L+1)]; column i*k+a is the letter a^(2^i).

    ``levels`` is L; by default floor(log2 n) as in Algorithm 5."""
    d = _as_delta(delta)
    n, k = d.shape
    L = floor_log2(n) if levels is None else int(levels)
    out = np.empty((n, k * (L + 1)), dtype=np.uint32)
    _check(_load().orc_pointer_jump(n, k, _p32(d), L, _p32(out)), "pointer_jump")
    return out


def quotient(delta, acc, block, start: int = 0):
    """Quotient of a canonical partition: (num_blocks, qdelta [B,k], qacc [B], qstart)."""
    d = _as_delta(delta)
    a = _as_acc(acc)
    b = np.ascontiguousarray(block, dtype=np.uint32)
    n, k = d.shape
    qdelta = np.empty((n, k), dtype=np.uint32)
    qacc = np.empty(n, dtype=np.uint8)
    qn, qs = ctypes.c_uint32(), ctypes.c_uint32()
    _check(_load().orc_quotient(n, k, _p32(d), _p8(a), _p32(b), start, ctypes.byref(qn),
                                _p32(qdelta), _p8(qacc), ctypes.byref(qs)), "quotient")
    B = qn.value
    return B, qdelta[:B].copy(), qacc[:B].copy(), qs.value


def _dfa_args(delta, acc, start):
    d = _as_delta(delta)
    a = _as_acc(acc)
    return (d, a), [d.shape[0], d.shape[1], _p32(d), _p8(a), int(start)]


def equiv_hk(dA, accA, sA, dB, accB, sB) -> bool:
    """Union-find Hopcroft-Karp: True iff L(A) == L(B)."""
    keepA, argsA = _dfa_args(dA, accA, sA)
    keepB, argsB = _dfa_args(dB, accB, sB)
    v = ctypes.c_int()
    _check(_load().orc_equiv_hk(*argsA, *argsB, ctypes.byref(v)), "equiv_hk")
    return bool(v.value)


def product_bfs(dA, accA, sA, dB, accB, sB, mode: str = "inclusion") -> tuple[bool, int]:
    """Naive pair-set exploration.  mode 'inclusion' decides L(A) <= L(B),
    'equivalence' decides L(A) == L(B).  Returns (verdict, pairs visited)."""
    keepA, argsA = _dfa_args(dA, accA, sA)
    keepB, argsB = _dfa_args(dB, accB, sB)
    m = {"inclusion": 0, "equivalence": 1}[mode]
    v = ctypes.c_int()
    cnt = ctypes.c_uint64()
    _check(_load().orc_product_bfs(*argsA, *argsB, m, ctypes.byref(v), ctypes.byref(cnt)),
           "product_bfs")
    return bool(v.value), int(cnt.value)


def included(dA, accA, sA, dB, accB, sB) -> bool:
    return product_bfs(dA, accA, sA, dB, accB, sB, "inclusion")[0]


def minimise_many(deltas, accs, algo: str = "hopcroft") -> np.ndarray:
    """Minimise ``count`` DFAs of one shape: deltas [count, n, k], accs [count, n]."""
    d = np.ascontiguousarray(deltas, dtype=np.uint32)
    a = np.ascontiguousarray(np.asarray(accs) != 0, dtype=np.uint8)
    count, n, k = d.shape
    out = np.empty((count, n), dtype=np.uint32)
    code = {"hopcroft": 0, "moore": 1, "naive_pr": 2}[algo]
    _check(_load().orc_minimise_many(code, count, n, k, _p32(d), _p8(a), _p32(out)),
           "minimise_many")
    return out


def reachable(delta, start: int = 0) -> np.ndarray:
    """Boolean mask of the states reachable from ``start`` (breadth-first)."""
    d = _as_delta(delta)
    n, k = d.shape
    out = np.empty(n, dtype=np.uint8)
    cnt = ctypes.c_uint32()
    _check(_load().orc_reachable(n, k, _p32(d), start, _p8(out), ctypes.byref(cnt)), "reachable")
    return out.astype(bool)


UNREACHABLE = 0xFFFFFFFF


def minimise_reachable(delta, acc, start: int = 0):
    """Minimisation of the part reachable from ``start``.  Returns (block,
    num_blocks, num_reachable); block[q] = UNREACHABLE for unreachable q."""
    d = _as_delta(delta)
    a = _as_acc(acc)
    n, k = d.shape
    block = np.empty(n, dtype=np.uint32)
    nb, nr = ctypes.c_uint32(), ctypes.c_uint32()
    _check(_load().orc_minimise_reachable(n, k, _p32(d), _p8(a), start, _p32(block),
                                          ctypes.byref(nb), ctypes.byref(nr)),
           "minimise_reachable")
    return block, nb.value, nr.value


def union(dA, accA, dB, accB) -> tuple[np.ndarray, np.ndarray]:
    """Disjoint union of two DFAs (B's states follow A's)."""
    dA = _as_delta(dA)
    dB = _as_delta(dB)
    nA = dA.shape[0]
    return (np.concatenate([dA, dB.astype(np.uint64) + nA]).astype(np.uint32),
            np.concatenate([_as_acc(accA), _as_acc(accB)]))


def minimise_tc(delta, acc, levels: int | None = None):
    """Moore refinement on the DFA extended by pointer jumping (Algorithm 5
    followed by signature rounds).  Returns (block, num_blocks, rounds, changing)."""
    ext = pointer_jump(delta, levels)
    return moore(ext, acc)
