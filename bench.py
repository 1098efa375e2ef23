#!/usr/bin/env python3
"""Benchmark of the partition-refinement hot path on one MI355X.

One step = the whole path over one synthetic workload already resident in HBM:
  * minimise a random complete DFA with n = 2^22 states, |Sigma| = 4,
    acceptance p = 0.1 (seed 2): ingest, initial partition, signature rounds
    (closure on demand), canonical block ids and the quotient DFA;
  * decide its equivalence with a state-permuted copy (seed 20) and with a
    copy where one transition is redirected (seed 21), by refining the
    disjoint unions.
The metric is transitions refined per second: the sum over the step's
refinements of n * k_eff * rounds, divided by the step time.

Prints one JSON line.  Kernel timing (HIP events inside the library, on the
stream the kernels run on) gives the dominant kernel's average launch time
for the roofline entry; the CPU baseline runs the sequential oracle on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "transitions refined/sec (n·|Σ|·rounds/s) and achieved HBM GB/s; batched vs plain"
UNIT = "transitions/s"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_digest() -> str:
    """Digest of the round-kernel sources the counter summary was taken with
    (the same files the summary tool hashes)."""
    from paper_2508_20735_amd.profiling import kernel_source_digest as digest
    return digest(ROOT)


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--loop", default="graph", choices=["host", "chunk", "graph"])
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timing on the host cores")
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="steps with every round kernel timed, before the timed region")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="time the steps without per-kernel events (roofline omitted)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-vs-plain comparison on the 4,096-DFA workload")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served request stream")
    ap.add_argument("--serve-requests", type=int, default=96)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the comparison of grouping / refinement variants")
    ap.add_argument("--no-table2", action="store_true",
                    help="skip the runs on the paper's Table 2 families")
    ap.add_argument("--no-host-path", action="store_true",
                    help="skip the same step through the host-pointer calls (copies included)")
    ap.add_argument("--no-products", action="store_true",
                    help="skip the product explorations (Tables 4 and 5 families)")
    ap.add_argument("--no-chain", action="store_true",
                    help="skip the chain-structured workload (plain vs closure)")
    ap.add_argument("--no-chain-plain", action="store_true",
                    help="in the chain leg, skip the plain refinement (about 2^20 rounds)")
    ap.add_argument("--only", choices=["batch", "served", "chain"],
                    help="run only this leg (no timed step) and print its object: for "
                         "profiling one leg under rocprofv3")
    return ap.parse_args()


def note(msg: str) -> None:
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def traffic_for(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when it is missing or the kernels changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha1") != kernel_source_digest():
        return None
    entry = t.get("library_kernels", {}).get(kernel)
    if not entry:
        return None
    return entry.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads for the all-cores oracle runs: the cores this process may use,
    at most 16 (the share of one GPU on a shared host)."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return max(1, min(16, usable))


def cpu_baseline(W, d, perm) -> dict:
    """The oracle (plain C, gcc -O3) on the machine's host cores, on bounded
    samples of the same workloads.  value: sequential Moore signature
    refinement (one thread) of the 2^22-state DFA and of its union with the
    permuted copy, in transitions refined per second (n * k * rounds / s).
    Beside it: sequential Hopcroft on the same DFA and union-find
    Hopcroft-Karp on the permuted pair; and, with one DFA per thread over all
    usable cores, the 4,096-DFA batch workload (Moore) and the 96 served
    requests (Hopcroft, or Hopcroft-Karp for equivalence requests)."""
    import concurrent.futures

    import oracle
    t0 = time.perf_counter()
    _, _, rounds_a, _ = oracle.moore(d.delta, d.accepting)
    t1 = time.perf_counter()
    ud, ua = oracle.union(d.delta, d.accepting, perm.delta, perm.accepting)
    t2 = time.perf_counter()
    _, _, rounds_u, _ = oracle.moore(ud, ua)
    t3 = time.perf_counter()
    work = d.n * d.k * rounds_a + 2 * d.n * d.k * rounds_u
    secs = (t1 - t0) + (t3 - t2)
    t4 = time.perf_counter()
    oracle.hopcroft(d.delta, d.accepting)
    t5 = time.perf_counter()
    oracle.equiv_hk(d.delta, d.accepting, d.start, perm.delta, perm.accepting, perm.start)
    t6 = time.perf_counter()
    threads = host_threads()

    def pool_map(fn, xs):
        with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
            return list(ex.map(fn, xs))

    items = W.batch_workload(count=4096, paired_from=2048)
    t7 = time.perf_counter()
    res = pool_map(lambda it: oracle.moore(it.dfa.delta, it.dfa.accepting), items)
    t8 = time.perf_counter()
    batch_work = sum(it.dfa.n * it.dfa.k * r[2] for it, r in zip(items, res))
    reqs = W.serving_workload(96, rate=1.0)

    def serve_one(r):
        if r.kind == "minimise":
            return oracle.hopcroft(r.dfa.delta, r.dfa.accepting)[1]
        return oracle.equiv_hk(r.dfa.delta, r.dfa.accepting, r.dfa.start, r.other.delta,
                               r.other.accepting, r.other.start)
    t9 = time.perf_counter()
    pool_map(serve_one, reqs)
    t10 = time.perf_counter()
    return {"value": work / secs, "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": (f"Moore rounds on the n=2^22 DFA ({rounds_a} rounds) and on its union "
                       f"with the permuted copy ({rounds_u} rounds), {secs:.1f} s, one thread"),
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "usable_cores": threads,
            "compiler": "gcc -O3 -std=c11",
            "hopcroft_2e22_s": t5 - t4,
            "hopcroft_2e22_transitions_per_s": d.n * d.k / (t5 - t4),
            "hk_equivalence_2e22_permuted_s": t6 - t5,
            "batch_all_cores": {"threads": threads, "dfas": len(items), "seconds": t8 - t7,
                                "transitions_per_s": batch_work / (t8 - t7),
                                "what": "Moore on each of the 4,096 batch DFAs, one per thread"},
            "served_all_cores": {"threads": threads, "requests": len(reqs),
                                 "seconds": t10 - t9, "requests_per_s": len(reqs) / (t10 - t9),
                                 "what": "Hopcroft (minimise) or union-find Hopcroft-Karp "
                                         "(equivalence) per request, one per thread"}}


def chain_leg(B, W, torch, np, dev, plain: bool) -> dict:
    """The chain-structured workload: a 2^20-state chain (letter a steps, b is
    the identity, only the last state accepts) followed by a 2^20-state random
    tail.  Plain refinement (about 2^20 rounds, run once) against the closure
    built first (tc on) and on demand (tc auto), median device time of 3 runs
    after one warm-up, with the input resident.  rate = the library's
    transitions refined (n * k_eff * rounds) over the time;
    plain_equivalent_rate = n * k * (rounds of the plain run) over the time."""
    d = W.cfg_chain()
    delta = torch.from_numpy(d.delta.view(np.int32)).to(dev)
    acc = torch.from_numpy(d.accepting).to(dev)
    blk = torch.empty(d.n, dtype=torch.int32, device=dev)
    plain_rounds = (1 << 20) - 1  # the closed form, replaced by the plain run's count
    out = {"workload": "chain 2^20 (a: i -> i+1, b: identity, last state accepting) + "
                       "2^20-state random tail (k = 2, p = 0.5), seed 3",
           "n": d.n, "k": d.k}
    if plain:
        print("chain leg: plain refinement", file=sys.stderr, flush=True)
        st = B.minimise_device(delta, acc, blk, tc="off", loop="graph").stats
        plain_rounds = st["rounds"]
        out["off"] = {"ms": st["device_ms"], "rounds": st["rounds"],
                      "changing_rounds": st["changing_rounds"], "k_eff": st["k_eff"],
                      "rate": st["transitions_refined"] / (st["device_ms"] * 1e-3),
                      "algorithmic_GBps": st["algorithmic_bytes"] / (st["device_ms"] * 1e-3) / 1e9}
    for tc in ("on", "auto"):
        def once():
            return B.minimise_device(delta, acc, blk, tc=tc, loop="graph").stats
        once()
        sts = [once() for _ in range(3)]
        ms = float(np.median([s_["device_ms"] for s_ in sts]))
        st = sts[-1]
        out[tc] = {"ms": ms, "rounds": st["rounds"], "changing_rounds": st["changing_rounds"],
                   "k_eff": st["k_eff"], "plain_rounds_before_closure": st["plain_rounds"],
                   "rate": st["transitions_refined"] / (ms * 1e-3),
                   "plain_equivalent_rate": d.n * d.k * plain_rounds / (ms * 1e-3)}
    out["plain_rounds_used"] = plain_rounds
    if plain:
        out["closure_speedup"] = {tc: out["off"]["ms"] / out[tc]["ms"] for tc in ("on", "auto")}
    del delta, acc, blk
    return out


def batch_leg(B, W, torch, np, count: int) -> dict:
    """Batched vs plain on the same GPU: `count` random DFAs (n log-uniform in
    [64, 65536], k in 2..8, p in [0.05, 0.5]); the upper half also checked for
    equivalence (even: permuted copy, odd: one-transition mutation).  Batched =
    one dfa_minimise_batch_device + one dfa_equivalent_batch_device call, the
    operands packed in flat GPU tensors (PackedBatch); plain = one
    dfa_minimise_device / dfa_equivalent_device call per DFA/pair."""
    dev = torch.device("cuda:0")
    items = W.batch_workload(count=count, paired_from=count // 2)

    def up(d):
        return (torch.from_numpy(d.delta.view(np.int32)).to(dev),
                torch.from_numpy(d.accepting).to(dev), d.start)

    A = [up(it.dfa) for it in items]
    pairs = [(i, up(it.pair)) for i, it in enumerate(items) if it.pair is not None]
    total = sum(it.dfa.n for it in items)
    out = torch.empty(total, dtype=torch.int32, device=dev)
    blocks = [torch.empty(it.dfa.n, dtype=torch.int32, device=dev) for it in items]
    # the batched calls take each operand list packed in two flat tensors
    pack_all = B.PackedBatch.from_dfas([it.dfa for it in items])
    pack_l = B.PackedBatch.from_dfas([items[i].dfa for i, _ in pairs])
    pack_r = B.PackedBatch.from_dfas([it.pair for it in items if it.pair is not None])
    torch.cuda.synchronize()

    def batched():
        nb, rounds, st = B.minimise_batch_device(pack_all, None, out)
        v, st2 = B.equivalent_batch_device(pack_l, pack_r)
        return st["transitions_refined"] + st2["transitions_refined"], v

    def plain():
        work = 0
        for a, blk in zip(A, blocks):
            r = B.minimise_device(a[0], a[1], blk, tc="off")
            work += r.stats["transitions_refined"]
        verdicts = []
        for i, p in pairs:
            v, s2 = B.equivalent_device(A[i][0], A[i][1], A[i][2], p[0], p[1], p[2], tc="off")
            verdicts.append(v)
            work += s2["transitions_refined"]
        return work, verdicts

    batched()
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        work_b, vb = batched()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    work_p, vp = plain()
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    if list(vb) != list(vp):
        raise RuntimeError("batched and plain equivalence verdicts differ")
    leg = {"workload": f"{count} random DFAs, n log-uniform [64, 65536], k in 2..8, "
                       f"{len(pairs)} equivalence pairs",
           "states": total, "batched_ms": tb * 1e3, "plain_ms": tp * 1e3,
           "speedup": tp / tb,
           "batched_transitions_per_s": work_b / tb,
           "plain_transitions_per_s": work_p / tp}
    leg["autotuned"] = autotuned_batch(B, torch, A, pairs, batched=batched, plain_s=tp)
    return leg


def autotuned_batch(B, torch, A, pairs, batched, plain_s) -> dict:
    """The same batch under the tuning the package's autotuner picks for it
    (coordinate descent over the batch tuning on this workload, a scratch
    cache file), timed like the default one; the default tuning is restored
    afterwards."""
    import tempfile

    from paper_2508_20735_amd import autotune as T
    before = B.get_tuning()
    space = {"batch_lds_states": [0, 2048, 4096, 8192], "round_grid_cap": [4096, 8192, 16384],
             "chunk": [4, 8, 16]}
    try:
        with tempfile.TemporaryDirectory() as tmp:
            res = T.autotune_batch([a[0] for a in A], [a[1] for a in A],
                                   pairs=([A[i] for i, _ in pairs], [p for _, p in pairs]),
                                   space=space, reps=2, path=os.path.join(tmp, "tuning.json"))
        tunings = list(res.values())
        # the minimisation's tuning for the whole step (the equivalence search
        # starts from it and may move further)
        B.set_tuning(**tunings[0]["tuning"])
        batched()
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            work, _v = batched()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        return {"tuning": tunings[0]["tuning"], "searched": space,
                "per_shape_device_ms": {k: v["device_ms"] for k, v in res.items()},
                "batched_ms": t * 1e3, "speedup": plain_s / t,
                "batched_transitions_per_s": work / t}
    finally:
        B.set_tuning(**before)


def variants_leg(B, W, torch, np, dev, A_d, A_a, n, pairs) -> dict:
    """The same GPU on the same inputs with the other refinement options:
    sort-based grouping (sortPR's grouping) vs the hash table on the 2^22
    minimisation; leader rounds (naivePR) vs signature rounds on the
    bit-splitter B_20 of Table 2; reachability pruning on the 2^22 workload;
    the step's two equivalences decided by product exploration instead of
    refining the union.  Median device time of 3 runs after one warm-up."""

    def med(fn, runs=3):
        fn()
        ts = []
        st = None
        for _ in range(runs):
            st = fn()
            ts.append(st["device_ms"])
        return float(np.median(ts)), st

    block = torch.empty(n, dtype=torch.int32, device=dev)
    out = {}
    for alg in ("signature", "sort"):
        ms, st = med(lambda: B.minimise_device(A_d, A_a, block, tc="off", loop="graph",
                                               algorithm=alg).stats)
        out[f"minimise_2e22_{alg}_ms"] = ms
        out[f"minimise_2e22_{alg}_rounds"] = st["rounds"]
    ms, st = med(lambda: B.minimise_device(A_d, A_a, block, tc="off", loop="graph",
                                           prune=True).stats)
    out["minimise_2e22_pruned_ms"] = ms
    out["minimise_2e22_reachable"] = st["reachable"]
    bs = W.bitsplitter(20)
    bd = torch.from_numpy(bs.delta.view(np.int32)).to(dev)
    ba = torch.from_numpy(bs.accepting).to(dev)
    bb = torch.empty(bs.n, dtype=torch.int32, device=dev)
    for alg in ("signature", "leader"):
        ms, st = med(lambda: B.minimise_device(bd, ba, bb, tc="off", loop="graph",
                                               algorithm=alg).stats)
        out[f"b20_{alg}_ms"] = ms
        out[f"b20_{alg}_rounds"] = st["rounds"]
    out["b20_transitions"] = bs.n * bs.k
    for name, (start, P_d, P_a, p_start) in pairs.items():
        for method in ("union", "product"):
            ms, st = med(lambda: B.equivalent_device(A_d, A_a, start, P_d, P_a, p_start,
                                                     method=method)[1])
            out[f"equiv_2e22_{name}_{method}_ms"] = ms
        out[f"equiv_2e22_{name}_product_pairs"] = st["reachable"]
    return out


def host_path_leg(B, np, d, perm, mut, steps: int = 5) -> dict:
    """The timed step through the host-pointer calls: the DFAs start in host
    memory (pageable numpy arrays) and the block ids and quotient come back to
    it, so the rate includes the PCIe copies each way.  Not the headline
    value, which is measured with the inputs resident in HBM."""

    def step():
        r = B.minimise(d.delta, d.accepting, quotient=True)
        _, s1 = B.equivalent(d, perm)
        _, s2 = B.equivalent(d, mut)
        stats = (r.stats, s1, s2)
        return (sum(s["transitions_refined"] for s in stats),
                sum(s["h2d_ms"] for s in stats), sum(s["d2h_ms"] for s in stats),
                sum(s["device_ms"] for s in stats))

    step()
    work = h2d = d2h = device = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        w, a, b, c = step()
        work, h2d, d2h, device = work + w, h2d + a, d2h + b, device + c
    wall = time.perf_counter() - t0
    return {"steps": steps, "ms_per_step": wall / steps * 1e3,
            "transitions_per_s": work / wall, "h2d_ms_per_step": h2d / steps,
            "d2h_ms_per_step": d2h / steps, "device_ms_per_step": device / steps,
            "bytes_in_per_step": int(3 * d.delta.nbytes + 3 * d.accepting.nbytes
                                     + perm.delta.nbytes + mut.delta.nbytes
                                     + perm.accepting.nbytes + mut.accepting.nbytes),
            "bytes_out_per_step": int(4 * d.n + d.delta.nbytes + d.n)}


# Table 2 of the paper (TITAN RTX, times include the host-to-device copy):
# context for the runs below, not a target.
PAPER_TABLE2_MS = {
    "Fib20": {"naivePR": 308.8, "sortPR": 3909.2, "transPR": 1.7},
    "B20": {"naivePR": 19.3, "sortPR": 520.2, "transPR": 139.8},
    "B22": {"naivePR": 82.6, "sortPR": 2538.5, "transPR": 728.7},
}


def table2_leg(B, W, torch, np, dev) -> dict:
    """The paper's Table 2 families on this GPU: leader rounds (naivePR),
    signature rounds grouped by hashing and by sorting (sortPR's semantics),
    transPR (closure + naivePR), signature rounds over the closure letters,
    and the closure on demand.  Device time with the input resident, median
    of 3 runs after one warm-up."""
    runs = {
        "Fib20": (lambda: W.fibonacci(21),
                  [("naivePR", "leader", "off"), ("signature", "signature", "off"),
                   ("transPR", "leader", "on"), ("signature_tc_on", "signature", "on"),
                   ("signature_tc_auto", "signature", "auto")]),
        "B20": (lambda: W.bitsplitter(20),
                [("naivePR", "leader", "off"), ("signature", "signature", "off"),
                 ("sort", "sort", "off"), ("transPR", "leader", "on")]),
        "B22": (lambda: W.bitsplitter(22),
                [("naivePR", "leader", "off"), ("signature", "signature", "off"),
                 ("sort", "sort", "off")]),
    }
    out = {}
    for name, (make, variants) in runs.items():
        d = make()
        delta = torch.from_numpy(d.delta.view(np.int32)).to(dev)
        acc = torch.from_numpy(d.accepting).to(dev)
        blk = torch.empty(d.n, dtype=torch.int32, device=dev)
        row = {"n": d.n, "k": d.k, "paper_ms": PAPER_TABLE2_MS[name]}
        for label, alg, tc in variants:
            def once():
                return B.minimise_device(delta, acc, blk, tc=tc, loop="graph",
                                         algorithm=alg).stats
            once()
            sts = [once() for _ in range(3)]
            ms = float(np.median([st["device_ms"] for st in sts]))
            row[label] = {"ms": ms, "rounds": sts[-1]["rounds"],
                          "num_blocks": sts[-1]["num_blocks"],
                          "algorithmic_GBps": sts[-1]["algorithmic_bytes"] / (ms * 1e-3) / 1e9}
        out[name] = row
        del delta, acc, blk
    return out


# Tables 4 and 5 of the paper: exploration time (ms) of the product on an
# RTX 3090 and a Titan RTX (initialisation excluded): context only.
PAPER_PRODUCT_MS = {
    "memory20_incl": (117, 173), "memory22_incl": (309, 420), "memory24_incl": (1269, 1481),
    "Bext20_self": (130, 302), "C30_self": (239, 271), "C32_self": (556, 553),
}


def product_leg(B, W, torch, np, dev) -> dict:
    """Product exploration (Section 4): inclusion of forgetful memory_n in
    perfect memory_n (Table 5) and equivalence of B'_n and C_n with
    themselves by product exploration (Table 4).  Device time with the inputs
    resident, median of 3 runs after one warm-up; pairs = reached pairs."""
    def t(x):
        x = np.ascontiguousarray(x)
        return torch.from_numpy(x.view(np.int32) if x.dtype == np.uint32 else x).to(dev)

    runs = [("memory20_incl", lambda: (W.memory(20, True), W.memory(20, False)), "incl"),
            ("memory22_incl", lambda: (W.memory(22, True), W.memory(22, False)), "incl"),
            ("memory24_incl", lambda: (W.memory(24, True), W.memory(24, False)), "incl"),
            ("Bext20_self", lambda: (W.extended_bitsplitter(20),) * 2, "equiv"),
            ("C30_self", lambda: (W.cycle(30),) * 2, "equiv"),
            ("C32_self", lambda: (W.cycle(32),) * 2, "equiv")]
    out = {}
    for name, make, kind in runs:
        a, b = make()
        args = (t(a.delta), t(a.accepting), a.start, t(b.delta), t(b.accepting), b.start)

        def once():
            if kind == "incl":
                ok, pairs, st = B.included_device(*args)
            else:
                ok, st = B.equivalent_device(*args, method="product")
                pairs = st["reachable"]
            return ok, pairs, st
        once()
        res = [once() for _ in range(3)]
        ms = float(np.median([r[2]["device_ms"] for r in res]))
        ok, pairs, st = res[-1]
        out[name] = {"verdict": ok, "pairs": pairs, "levels": st["rounds"], "ms": ms,
                     "pairs_per_s": pairs / (ms * 1e-3),
                     "paper_exploration_ms_rtx3090_titanrtx": PAPER_PRODUCT_MS[name]}
        del args
    return out


def gather_reference(torch, dev, sizes) -> dict:
    """Random-gather rate of the device as a plain framework gather reaches
    it (torch indexing: 4 * size random int32 gathers from a size-element
    array, int64 indices), median of 10 timed repetitions: the ceiling of a
    kernel whose successor-id gathers hit random lines."""
    out = {}
    for size in sizes:
        x = torch.randint(0, size, (size,), dtype=torch.int32, device=dev)
        idx = torch.randint(0, size, (4 * size,), dtype=torch.int64, device=dev)
        for _ in range(3):
            x[idx]
        times = []
        for _ in range(10):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            x[idx]
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = sorted(times)[len(times) // 2]
        out[str(size)] = 4 * size / (ms * 1e-3)
        del x, idx
    return out


def probe_reference(torch, dev, slots: int, probes: int) -> float:
    """Random 8-byte loads per second from a table of `slots` int64 words (the
    size of the grouping kernel's hash table), as torch indexing reaches
    them: `probes` random indices, median of 10 timed repetitions."""
    table = torch.randint(0, 1 << 62, (slots,), dtype=torch.int64, device=dev)
    idx = torch.randint(0, slots, (probes,), dtype=torch.int64, device=dev)
    for _ in range(3):
        table[idx]
    times = []
    for _ in range(10):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        table[idx]
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = sorted(times)[len(times) // 2]
    del table, idx
    return probes / (ms * 1e-3)


def serve_leg(B, W, count: int) -> dict:
    """Served requests: n log-uniform in [1,000, 4,194,304], k in {2,4,8,16},
    80% minimise / 20% equivalence, 10% chain DFAs, host arrays.  First a
    burst (all requests submitted at once, after one untimed burst on the same
    server) gives the capacity; then a Poisson stream at 0.7x that rate gives
    p50/p99 latency; plain = the same requests one by one through the
    single-request host calls."""
    reqs = W.serving_workload(count, rate=1.0)

    def submit(srv, r):
        return srv.submit_minimise(r.dfa) if r.kind == "minimise" else \
            srv.submit_equivalent(r.dfa, r.other)

    def plain_one(r):
        """One request through the single-request host calls; returns the
        call's device time (copies excluded)."""
        if r.kind == "minimise":
            return B.minimise(r.dfa.delta, r.dfa.accepting).stats["device_ms"]
        return B.equivalent(r.dfa, r.other)[1]["device_ms"]

    def burst(srv, results=None):
        t0 = time.perf_counter()
        tickets = [submit(srv, r) for r in reqs]
        for t in tickets:
            res = srv.wait(t)
            if results is not None:
                results.append(res)
        return time.perf_counter() - t0

    burst_res = []
    with B.Server() as srv:
        # a long-running server: one untimed pass warms its page-locked
        # input pool and the lanes' device workspaces
        burst(srv)
        burst_s = burst(srv, burst_res)
    capacity = count / burst_s
    rate = 0.7 * capacity
    gaps = W._rng(55).exponential(1.0 / rate, size=count)
    with B.Server() as srv:
        burst(srv)
        t0 = time.perf_counter()
        tickets = []
        due = t0
        for r, g in zip(reqs, gaps):
            due += g
            delay = due - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets.append(submit(srv, r))
        stream_res = [srv.wait(t) for t in tickets]
        lat = [r_["latency_ms"] for r_ in stream_res]
        stream_s = time.perf_counter() - t0
    for r in reqs[:2]:
        plain_one(r)
    t0 = time.perf_counter()
    plain_device_ms = sum(plain_one(r) for r in reqs)
    plain_s = time.perf_counter() - t0
    lat_sorted = sorted(lat)
    pick = lambda q: lat_sorted[min(len(lat_sorted) - 1, int(q * (len(lat_sorted) - 1) + 0.5))]
    return {"workload": (f"{count} requests, n log-uniform [1000, 4194304], k in {{2,4,8,16}}, "
                         "80% minimise / 20% equivalence, 10% chain"),
            "burst_requests_per_s": capacity,
            "plain_requests_per_s": count / plain_s,
            "speedup": (count / burst_s) / (count / plain_s),
            "poisson_rate": rate, "p50_ms": pick(0.5), "p99_ms": pick(0.99),
            "stream_requests_per_s": count / stream_s, "lanes": 4,
            "plain_ms": plain_s * 1e3, "plain_device_ms_sum": plain_device_ms,
            # the served form overlaps requests but runs the same device work:
            # plain time over its device time bounds the speed-up of any
            # server on this mix while each request's kernels fill the GPU
            "speedup_ceiling_device_bound": plain_s * 1e3 / plain_device_ms,
            "breakdown": {"stream": _served_breakdown(stream_res),
                          "burst": _served_breakdown(burst_res)}}


def _served_breakdown(results) -> dict:
    """Where served requests spend their time: medians and means over the
    requests of queue (submit -> start), input copies, device work and result
    copy (a batched request reports its group's copies and device work), and
    the device time of the distinct groups summed (each group counted once)."""
    import statistics
    parts = ("queue_ms", "h2d_ms", "device_ms", "d2h_ms", "service_ms", "latency_ms")
    out = {}
    for p in parts:
        vals = [r[p] for r in results]
        out[p] = {"median": statistics.median(vals), "mean": statistics.fmean(vals)}
    groups = {(r["h2d_ms"], r["device_ms"], r["d2h_ms"]) for r in results}
    out["distinct_groups"] = len(groups)
    out["device_ms_sum_over_groups"] = sum(g[1] for g in groups)
    out["h2d_ms_sum_over_groups"] = sum(g[0] for g in groups)
    out["d2h_ms_sum_over_groups"] = sum(g[2] for g in groups)
    return out


def main() -> int:
    args = parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent DFAs would shard one queue per GPU)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2508_20735_amd import binding as B
    from paper_2508_20735_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    B.load(build_if_missing=True)
    dev = torch.device("cuda:0")

    if args.only:
        if args.only == "batch":
            leg = batch_leg(B, W, torch, np, args.batch_count)
        elif args.only == "served":
            leg = serve_leg(B, W, args.serve_requests)
        else:
            leg = chain_leg(B, W, torch, np, dev, plain=not args.no_chain_plain)
        print(json.dumps({args.only: leg}), flush=True)
        return 0

    d = W.cfg_large()
    perm, _ = W.permuted_copy(d, W.CFG_LARGE_PERM_SEED)
    mut, _ = W.mutate_one(d, W.CFG_LARGE_MUT_SEED)

    def to_dev(x):
        return (torch.from_numpy(x.delta.view(np.int32)).to(dev),
                torch.from_numpy(x.accepting).to(dev))

    A_d, A_a = to_dev(d)
    P_d, P_a = to_dev(perm)
    M_d, M_a = to_dev(mut)
    block = torch.empty(d.n, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    loop = "chunk" if not args.no_kernel_timing and args.loop == "graph" else args.loop

    def step():
        r = B.minimise_device(A_d, A_a, block, quotient=True, loop=loop)
        e1, s1 = B.equivalent_device(A_d, A_a, d.start, P_d, P_a, perm.start, loop=loop)
        e2, s2 = B.equivalent_device(A_d, A_a, d.start, M_d, M_a, mut.start, loop=loop)
        if not e1:
            raise RuntimeError("permuted copy reported inequivalent")
        work = (r.stats["transitions_refined"] + s1["transitions_refined"]
                + s2["transitions_refined"])
        return work, (r.stats, s1, s2, e2)

    note("timed step")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kernels, dom = {}, None
    if not args.no_kernel_timing:
        # every round kernel timed over extra steps before the timed region
        # (the per-kernel table, and which kernel dominates) ...
        B.profile_only(None)
        B.profile_enable(True)
        for _ in range(args.profile_steps):
            step()
        torch.cuda.synchronize()
        kernels = B.profile_read()
        B.profile_enable(False)
        dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
        # ... and only the dominant kernel inside the timed region, so that
        # the events hardly disturb the measured step
        B.profile_only(dom)
        B.profile_enable(True)
    total = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        work, last = step()
        total += work
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    timed = {}
    if dom is not None:
        timed = B.profile_read()
        B.profile_enable(False)
        B.profile_only(None)

    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    stats_min, stats_perm, stats_mut, verdict_mut = last
    out = {
        "metric": METRIC,
        "value": total / elapsed,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": ("random complete DFA n=2^22 |Sigma|=4 p=0.1 seed 2: minimise "
                         "(+quotient) and equivalence vs permuted copy (seed 20) and vs "
                         "one-transition mutation (seed 21)"),
            "n": d.n, "k": d.k, "tc": "auto", "loop": loop,
            "rounds": [stats_min["rounds"], stats_perm["rounds"], stats_mut["rounds"]],
            "mutation_equivalent": bool(verdict_mut),
            "device_ms": [round(stats_min["device_ms"], 3), round(stats_perm["device_ms"], 3),
                          round(stats_mut["device_ms"], 3)],
            "tuning": B.get_tuning(),
        },
    }
    if dom is not None and dom in timed:
        kd = timed[dom]
        avg_s = kd["total_ms"] / kd["launches"] / 1e3
        bytes_per_launch = kd["algorithmic_bytes"] / kd["launches"]
        achieved = bytes_per_launch / avg_s / 1e9
        out["roofline"] = {
            "bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(dom),
            "avg_launch_us": avg_s * 1e6, "launches": kd["launches"],
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "refined_states_per_s": kd["states"] / (kd["total_ms"] / 1e3),
        }
        if dom == "k_signature":
            # the kernel gathers k block ids per refined state: its rate of
            # random gathers against the device's, measured the same way on
            # the union's size (most launches refine the 2n-state unions)
            gathers = kd["state_letters"]
            ref = gather_reference(torch, dev, [d.n, 2 * d.n])
            achieved_g = gathers / (kd["total_ms"] / 1e3)
            out["gather_roofline"] = {
                "kernel": dom, "achieved": achieved_g / 1e9, "peak": ref[str(2 * d.n)] / 1e9,
                "unit": "G gathers/s", "frac": achieved_g / ref[str(2 * d.n)],
                "reference": ("torch index gather: 4 * size random int32 gathers from a "
                              "size-element array (size = 2n), median of 10"),
                "reference_by_size": {s_: v / 1e9 for s_, v in ref.items()},
                "note": ("achieved = the timed region's gathers over all k_signature launches, "
                         "incremental rounds included (their fixed per-state work has no "
                         "gathers); full-round launches in the kernel trace run at the "
                         "reference rate"),
            }
        if dom == "k_insert":
            # every refined state that groups through the table probes it at
            # a random slot at least once: the kernel's refined states per
            # second against the device's random 8-byte load rate on a table
            # of the unions' size (2^ceil(log2(2 * 2n)) slots) is a lower
            # bound on the fraction of that rate it reaches
            slots = 1 << (4 * d.n - 1).bit_length()
            ref_probes = probe_reference(torch, dev, slots, 2 * d.n)
            achieved_p = kd["states"] / (kd["total_ms"] / 1e3)
            out["probe_roofline"] = {
                "kernel": dom, "achieved": achieved_p / 1e9, "peak": ref_probes / 1e9,
                "unit": "G random table probes/s (lower bound: one per refined state)",
                "frac": achieved_p / ref_probes,
                "reference": (f"torch index gather: {2 * d.n} random int64 loads from a "
                              f"{slots}-slot table, median of 10"),
            }
        pbg = kernels.get("k_pb_gather")
        if pbg and pbg["total_ms"] > 0 and pbg["state_letters"]:
            # the dense rounds' successor-id gathers, served from slices of
            # the id array held in LDS (edges bucketed by target slice)
            out["slice_gather"] = {
                "kernel": "k_pb_gather", "launches": pbg["launches"],
                "achieved": pbg["state_letters"] / (pbg["total_ms"] / 1e3) / 1e9,
                "unit": "G gathers/s",
                "note": ("gathers of the rounds that took the slice path over the pass's "
                         "time in the profiled steps (its no-op launches in other rounds "
                         "included)"),
            }
        out["kernels_profiled_steps"] = args.profile_steps
        out["kernels"] = {
            k: {"launches": v["launches"], "avg_us": v["total_ms"] / v["launches"] * 1e3,
                "share": v["total_ms"] / sum(x["total_ms"] for x in kernels.values()),
                "algorithmic_GBps": (v["algorithmic_bytes"] / (v["total_ms"] / 1e3) / 1e9
                                     if v["total_ms"] else 0.0)}
            for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["total_ms"])}
    if not args.no_batch:
        note("batched leg")
        out["batched"] = batch_leg(B, W, torch, np, args.batch_count)
    if not args.no_serve:
        note("served leg")
        out["served"] = serve_leg(B, W, args.serve_requests)
    if not args.no_variants:
        note("variants leg")
        out["variants"] = variants_leg(B, W, torch, np, dev, A_d, A_a, d.n,
                                       {"permuted": (d.start, P_d, P_a, perm.start),
                                        "mutated": (d.start, M_d, M_a, mut.start)})
    if not args.no_host_path:
        note("host-path leg")
        out["host_path"] = host_path_leg(B, np, d, perm, mut)
    if not args.no_table2:
        note("Table 2 leg")
        out["table2"] = table2_leg(B, W, torch, np, dev)
    if not args.no_products:
        note("products leg")
        out["products"] = product_leg(B, W, torch, np, dev)
    if not args.no_chain:
        note("chain leg")
        out["chain"] = chain_leg(B, W, torch, np, dev, plain=not args.no_chain_plain)
    if not args.no_cpu_baseline:
        note("CPU baseline")
        out["cpu_baseline"] = cpu_baseline(W, d, perm)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
