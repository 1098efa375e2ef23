"""The allocation-free entry point (dfa_minimise_device_fixed) against the
ordinary device entry point (dfa_minimise_device) and the oracle.

Both are called through the C ABI on the same device tensors; block ids,
quotients and round counts must be identical (integer work: exact).  Two
calls in a row, the second on a smaller DFA, check that nothing left in the
shared fixed workspace by one call leaks into the next.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_20735_amd import binding as B
from paper_2508_20735_amd import workloads as W

pytestmark = pytest.mark.gpu


def _device(d):
    dev = torch.device("cuda:0")
    delta = torch.from_numpy(np.ascontiguousarray(d.delta).view(np.int32)).to(dev)
    acc = torch.from_numpy(np.ascontiguousarray(d.accepting)).to(dev)
    return delta, acc


def _compare(d, tc="auto", loop="graph"):
    print(f"fixed vs device: n={d.n} k={d.k} tc={tc} loop={loop}", flush=True)
    delta, acc = _device(d)
    fixed = B.minimise_device_fixed(delta, acc, tc=tc, loop=loop, quotient=True, start=d.start)
    plain = B.minimise_device(delta, acc, tc=tc, loop=loop, quotient=True, start=d.start)
    torch.cuda.synchronize()
    got = fixed.block.cpu().numpy().view(np.uint32)
    want = plain.block.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got, want)
    ref, nb = oracle.hopcroft(d.delta, d.accepting)
    np.testing.assert_array_equal(got, ref)
    for key in ("num_blocks", "rounds", "changing_rounds", "k_eff", "tc_used"):
        assert fixed.stats[key] == plain.stats[key], key
    assert fixed.stats["num_blocks"] == nb
    fb, fd, fa, fs = fixed.quotient
    pb, pd, pa, ps = plain.quotient
    assert fb == pb == nb and fs == ps
    np.testing.assert_array_equal(fd.cpu().numpy(), pd.cpu().numpy())
    np.testing.assert_array_equal(fa.cpu().numpy(), pa.cpu().numpy())


def test_fixed_matches_device_entry_twice_shrinking():
    B.load(build_if_missing=False)
    torch.cuda.set_device(0)
    # several tiles and a ragged tail, then a much smaller DFA in the same
    # workspace
    _compare(W.random_dfa(300_001, 4, 0.1, 31))
    _compare(W.random_dfa(1_003, 2, 0.5, 32))


def test_fixed_chain_with_closure_and_loops():
    B.load(build_if_missing=False)
    # a chain-like DFA: the closure is built on demand inside the fixed
    # workspace; every loop driver (graph runs as chunk there)
    d = W.fibonacci(14)
    for loop in ("host", "chunk", "graph", "persistent"):
        _compare(d, tc="auto", loop=loop)
    _compare(d, tc="on")
    _compare(W.random_dfa(5_000, 3, 0.3, 33), tc="off")


def test_fixed_rejects_oversize_before_any_work():
    B.load(build_if_missing=False)
    n, k = 1 << 23, 8  # about 1 GB of workspace: beyond the fixed 256 MiB
    dev = torch.device("cuda:0")
    delta = torch.zeros((n, k), dtype=torch.int32, device=dev)
    acc = torch.zeros(n, dtype=torch.uint8, device=dev)
    with pytest.raises(B.DfaError) as e:
        B.minimise_device_fixed(delta, acc)
    assert e.value.status == B.DFA_ENOMEM
    assert "fixed workspace" in str(e.value)
    del delta, acc
    # still usable afterwards
    _compare(W.random_dfa(20_000, 3, 0.2, 34))


def test_fixed_reads_the_device_tuning():
    """The device's tuning (dfa_set_tuning) applies to the allocation-free
    entry point as to every other call: without label rounds the chain's
    closure is switched on at another round, and both entry points agree."""
    B.load(build_if_missing=False)
    before = B.get_tuning()
    try:
        B.set_tuning(label_rounds=0)
        d = W.chain_with_tail(400, 210, 7)
        for loop in ("host", "chunk"):
            _compare(d, tc="auto", loop=loop)
    finally:
        B.set_tuning(**before)
