"""Calls from several host threads at once.

Calls on one device are serialised inside the library (one workspace per
device), so concurrent callers must each get exactly the result a lone call
gives.  Each thread mixes host calls, device calls on a stream of its own,
batch calls and requests to one shared server.  Every result is checked
against the oracle.
"""
import threading

import numpy as np
import pytest

import oracle
from paper_2508_20735_amd import binding as B
from paper_2508_20735_amd import workloads as W

pytestmark = pytest.mark.gpu

THREADS = 6


def _jobs(t):
    rng = np.random.default_rng(100 + t)
    jobs = []
    for i in range(8):
        n = int(rng.integers(1, 30000))
        k = int(rng.integers(1, 6))
        d = W.random_dfa(n, k, float(rng.uniform(0.05, 0.6)), 1000 * t + i)
        kind = ("minimise", "device", "equivalent", "product", "included", "batch",
                "server", "server_eq")[(t + i) % 8]
        jobs.append((kind, d))
    return jobs


def _run(kind, d, srv, stream):
    import torch
    if kind == "minimise":
        res = B.minimise(d.delta, d.accepting, tc=("off", "auto", "on")[d.n % 3],
                         loop=("host", "chunk", "graph", "graph")[d.k % 4])
        return res.block
    if kind == "device":
        with torch.cuda.stream(stream):
            delta = torch.from_numpy(d.delta.astype(np.int32)).cuda()
            acc = torch.from_numpy(d.accepting).cuda()
            res = B.minimise_device(delta, acc, stream=stream)
            stream.synchronize()
            return res.block.cpu().numpy().astype(np.uint32)
    if kind in ("equivalent", "product", "included", "server_eq"):
        other, _ = (W.permuted_copy(d, d.n + 7) if d.n % 2 else W.mutate_one(d, d.n + 7)) \
            if d.n > 1 else (d, None)
        if kind == "included":
            return B.included(d, other)[0]
        if kind == "server_eq":
            return srv.wait(srv.submit_equivalent(d, other))["verdict"]
        return B.equivalent(d, other, method="product" if kind == "product" else "union")[0]
    if kind == "batch":
        blocks, nb, _, _ = B.minimise_batch([d, d])
        assert np.array_equal(blocks[0], blocks[1])
        return blocks[0]
    got = srv.wait(srv.submit_minimise(d))
    assert got["status"] == 0
    return got["blocks"]


def _expected(kind, d):
    if kind in ("minimise", "device", "batch", "server"):
        return oracle.hopcroft(d.delta, d.accepting)[0]
    other, _ = (W.permuted_copy(d, d.n + 7) if d.n % 2 else W.mutate_one(d, d.n + 7)) \
        if d.n > 1 else (d, None)
    args = (d.delta, d.accepting, d.start, other.delta, other.accepting, other.start)
    return oracle.included(*args) if kind == "included" else oracle.equiv_hk(*args)


def test_concurrent_callers():
    import torch
    jobs = [_jobs(t) for t in range(THREADS)]
    want = [[_expected(kind, d) for kind, d in js] for js in jobs]
    got = [[None] * len(js) for js in jobs]
    errors = []
    start = threading.Barrier(THREADS)

    with B.Server(lanes=2) as srv:
        def worker(t):
            try:
                stream = torch.cuda.Stream()
                start.wait()
                for i, (kind, d) in enumerate(jobs[t]):
                    got[t][i] = _run(kind, d, srv, stream)
            except BaseException as e:  # reported below, with the thread
                errors.append((t, repr(e)))

        threads = [threading.Thread(target=worker, args=(t,)) for t in range(THREADS)]
        for th in threads:
            th.start()
        for th in threads:
            th.join(timeout=100)
        assert not any(th.is_alive() for th in threads), "a caller did not finish"
    assert not errors, errors
    for t in range(THREADS):
        for i, (kind, d) in enumerate(jobs[t]):
            if isinstance(want[t][i], np.ndarray):
                np.testing.assert_array_equal(got[t][i], want[t][i], err_msg=f"{t} {i} {kind}")
            else:
                assert got[t][i] == want[t][i], (t, i, kind)



def test_graph_capture_beside_allocating_thread():
    """Graph-loop minimisations (a new round graph built for each size) while
    another thread allocates, fills and frees device memory through torch
    without pause: every call succeeds and every partition equals the oracle's."""
    import torch
    stop = threading.Event()
    churn = {"iterations": 0, "errors": []}

    def allocate():
        stream = torch.cuda.Stream()
        size = 1 << 20
        while not stop.is_set():
            try:
                with torch.cuda.stream(stream):
                    x = torch.empty(size, dtype=torch.uint8, device="cuda")
                    x.fill_(1)
                    del x
                torch.cuda.empty_cache()
            except RuntimeError as e:
                churn["errors"].append(repr(e))
            churn["iterations"] += 1
            size = (size * 3) % (64 << 20) + (1 << 20)

    th = threading.Thread(target=allocate)
    th.start()
    try:
        for i in range(40):
            d = W.random_dfa(3000 + 257 * i, 2 + i % 3, 0.3, 500 + i)
            res = B.minimise(d.delta, d.accepting, tc="off", loop="graph", chunk=1 + i % 5)
            hb, _ = oracle.hopcroft(d.delta, d.accepting)
            np.testing.assert_array_equal(res.block, hb, err_msg=str(i))
    finally:
        stop.set()
        th.join(timeout=60)
    assert not th.is_alive()
    assert churn["iterations"] > 0 and not churn["errors"], churn["errors"][:2]
