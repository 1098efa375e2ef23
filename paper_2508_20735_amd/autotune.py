"""Autotuner for the batched calls' kernel tuning.

The library's tuning (``dfa_tuning``: launch caps of the round kernels, the
first chunk length, and the largest DFA that the batched calls refine inside
one workgroup) changes speed, never results.  The autotuner measures
candidate tunings on the caller's own batch (device time reported by the
library, median of a few runs), one field at a time starting from the current
tuning (coordinate descent), keeps the fastest, and stores it in a JSON cache
keyed by the device (name and compute units) and a coarse shape of the
workload.  ``apply`` looks the shape up at call time and sets the cached
tuning; ``tuned`` does the same for the length of a ``with`` block.

    import paper_2508_20735_amd.autotune as T
    best = T.autotune_batch(deltas, accs)          # search, cache, leave it set
    with T.tuned(T.batch_shape(ns, ks)):           # later calls on the same shape
        B.minimise_batch_device(deltas, accs, out)

The cache file is ``$DFAMIN_TUNING_CACHE``, else
``~/.cache/dfamin/tuning.json``.
"""
from __future__ import annotations

import contextlib
import json
import math
import os
import statistics
import threading

from . import binding as B

# Candidate values per field, searched in this order.
SEARCH_SPACE = {
    "batch_lds_states": [0, 1024, 2048, 4096, 8192, 16384],
    "round_grid_cap": [2048, 4096, 8192, 16384],
    "chunk": [2, 4, 8, 16],
    "label_grid_cap": [1024, 2048, 4096],
}

_lock = threading.Lock()


def cache_path() -> str:
    return os.environ.get("DFAMIN_TUNING_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "dfamin", "tuning.json")


def device_key() -> str:
    info = B.device_info()
    return f"{info['name']}|{info['compute_units']}cu"


def _bucket(x: float) -> int:
    """log2 bucket (0 for x <= 1)."""
    return int(math.floor(math.log2(x))) if x > 1 else 0


def batch_shape(ns, ks, kind: str = "minimise") -> str:
    """Coarse shape of a batch: kind, log2 buckets of the DFA count, of the
    total states and of the median DFA size, and the largest alphabet."""
    ns = list(ns)
    ks = list(ks)
    return (f"batch-{kind}|count2^{_bucket(len(ns))}|states2^{_bucket(sum(ns))}"
            f"|median2^{_bucket(statistics.median(ns))}|kmax{max(ks)}")


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_entry(shape: str, tuning: dict, ms: float, path: str | None = None,
               device: str | None = None) -> None:
    """Adds (or replaces) the entry of this device and shape in the cache."""
    path = path or cache_path()
    with _lock:
        data = load_cache(path)
        data.setdefault(device or device_key(), {})[shape] = {"tuning": tuning, "device_ms": ms}
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        tmp = f"{path}.tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)


def lookup(shape: str, path: str | None = None, device: str | None = None) -> dict | None:
    entry = load_cache(path).get(device or device_key(), {}).get(shape)
    return dict(entry["tuning"]) if entry else None


def apply(shape: str, path: str | None = None) -> dict | None:
    """Sets the cached tuning of this device and shape (if any); returns it."""
    t = lookup(shape, path)
    if t is not None:
        B.set_tuning(**t)
    return t


@contextlib.contextmanager
def tuned(shape: str, path: str | None = None):
    """The cached tuning of `shape` for the block's calls, the previous one
    afterwards (no change when the shape is not cached)."""
    before = B.get_tuning()
    try:
        apply(shape, path)
        yield
    finally:
        B.set_tuning(**before)


def search(run, space: dict | None = None, reps: int = 3, start: dict | None = None,
           log=None) -> tuple[dict, float]:
    """Coordinate descent over `space` from `start` (default: the current
    tuning).  run() executes the workload once and returns its device time in
    ms; each candidate is timed `reps` times after one warm-up run, and the
    median counts.  Returns (best tuning, its median ms); the best tuning is
    left set."""
    space = space or SEARCH_SPACE
    best = dict(start or B.get_tuning())

    def measure(t: dict) -> float:
        B.set_tuning(**t)
        run()
        return statistics.median(run() for _ in range(reps))

    best_ms = measure(best)
    for field, values in space.items():
        for v in values:
            if best.get(field) == v:
                continue
            cand = dict(best)
            cand[field] = v
            ms = measure(cand)
            if log:
                log(f"{field}={v}: {ms:.3f} ms (best {best_ms:.3f})")
            if ms < best_ms:
                best, best_ms = cand, ms
    B.set_tuning(**best)
    return best, best_ms


def autotune_batch(deltas, accs, out=None, pairs=None, space: dict | None = None,
                   reps: int = 3, path: str | None = None, log=None) -> dict:
    """Tunes the batched calls on this workload and caches the result.

    deltas / accs: lists of device tensors (as minimise_batch_device takes);
    out: the output tensor (allocated if None).  pairs: optional
    (a_list, b_list) of (delta, accepting, start) tuples for
    equivalent_batch_device, tuned as a second shape.  Returns
    {shape: {"tuning": ..., "device_ms": ...}} for what was tuned."""
    import torch

    ns = [int(d.shape[0]) for d in deltas]
    ks = [int(d.shape[1]) for d in deltas]
    if out is None:
        out = torch.empty(sum(ns), dtype=torch.int32, device=deltas[0].device)
    result = {}

    def run_min():
        return B.minimise_batch_device(deltas, accs, out)[2]["device_ms"]

    shape = batch_shape(ns, ks, "minimise")
    best, ms = search(run_min, space, reps, log=log)
    save_entry(shape, best, ms, path)
    result[shape] = {"tuning": best, "device_ms": ms}
    if pairs is not None:
        a_list, b_list = pairs
        pn = [int(a[0].shape[0]) + int(b[0].shape[0]) for a, b in zip(a_list, b_list)]
        pk = [int(a[0].shape[1]) for a in a_list]

        def run_eq():
            return B.equivalent_batch_device(a_list, b_list)[1]["device_ms"]

        pshape = batch_shape(pn, pk, "equivalent")
        pbest, pms = search(run_eq, space, reps, start=best, log=log)
        save_entry(pshape, pbest, pms, path)
        result[pshape] = {"tuning": pbest, "device_ms": pms}
    return result
