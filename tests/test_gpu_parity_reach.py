"""GPU parity of reachability pruning (minimisation of the part reachable from
the start) against the oracle's breadth-first search + Hopcroft.

Block ids are exact integers: element-by-element equality, including the
UNREACHABLE marks; the quotient is compared with one built from the oracle's
ids.
"""
import numpy as np
import pytest

import oracle
from paper_2508_20735_amd import binding as B
from paper_2508_20735_amd import workloads as W

pytestmark = pytest.mark.gpu


def expected_quotient(d, block, start):
    mask = block != oracle.UNREACHABLE
    leaders = np.flatnonzero(mask & (block == np.arange(d.n, dtype=np.uint32)))
    dense = np.full(d.n, -1, dtype=np.int64)
    dense[leaders] = np.arange(len(leaders))
    qd = dense[block[d.delta[leaders]]].astype(np.uint32)
    qa = (d.accepting[leaders] != 0).astype(np.uint8)
    return len(leaders), qd, qa, int(dense[block[start]])


def check_pruned(d, start=None, tc="auto", quotient=True):
    start = d.start if start is None else start
    res = B.minimise(d.delta, d.accepting, tc=tc, start=start, prune=True, quotient=quotient)
    block, nb, nr = oracle.minimise_reachable(d.delta, d.accepting, start)
    np.testing.assert_array_equal(res.block, block)
    assert res.stats["num_blocks"] == nb and res.stats["reachable"] == nr
    if quotient:
        qn, qd, qa, qs = expected_quotient(d, block, start)
        gn, gd, ga, gs = res.quotient
        assert gn == qn and gs == qs
        np.testing.assert_array_equal(gd, qd)
        np.testing.assert_array_equal(ga, qa)
    return res


@pytest.mark.parametrize("n,k,p,seed,start", [
    (1, 1, 0.5, 1, 0), (2, 1, 0.5, 2, 1), (3, 2, 0.5, 3, 2), (65, 2, 0.3, 4, 7),
    (1000, 2, 0.5, 5, 0), (4097, 3, 0.2, 6, 4000), (20000, 2, 0.5, 7, 123),
    (30000, 8, 0.4, 8, 29999), (100000, 4, 0.1, 9, 0),
])
def test_pruned_random(n, k, p, seed, start):
    check_pruned(W.random_dfa(n, k, p, seed), start=start)


def test_pruned_small_config_all_loops():
    d = W.cfg_small()  # ~20% of its states are unreachable from 0
    for loop in ("host", "chunk", "graph"):
        res = B.minimise(d.delta, d.accepting, loop=loop, prune=True)
        block, nb, nr = oracle.minimise_reachable(d.delta, d.accepting, 0)
        np.testing.assert_array_equal(res.block, block)
        assert nr < d.n and res.stats["reachable"] == nr


def test_pruned_chain_with_tail():
    """The tail (targets inside the tail) is unreachable from 0; the chain is
    a search of depth N, done inside one workgroup."""
    d = W.chain_with_tail(1 << 14, 1 << 14, 11)
    res = check_pruned(d, start=0, quotient=False)
    assert res.stats["reachable"] == 1 << 14
    assert (res.block[1 << 14:] == B.UNREACHABLE).all()


def test_pruned_wide_and_narrow_frontiers():
    """Many letters (narrow search capacity 4096 / k) and a large random
    frontier (grid-wide levels)."""
    check_pruned(W.random_dfa(50000, 16, 0.3, 12), start=5, quotient=False)
    check_pruned(W.random_dfa(300000, 2, 0.5, 13), start=0, quotient=False)


def test_pruned_degenerate():
    # identity letters: only the start is reachable
    ident = W.DFA(np.tile(np.arange(9, dtype=np.uint32)[:, None], (1, 2)),
                  np.array([1, 0, 1, 0, 1, 0, 1, 0, 1], dtype=np.uint8), 4)
    res = check_pruned(ident)
    assert res.stats["reachable"] == 1 and res.stats["num_blocks"] == 1
    # every state reachable: same ids as without pruning
    f = W.fibonacci(11)
    res = check_pruned(f, tc="on")
    np.testing.assert_array_equal(res.block, oracle.hopcroft(f.delta, f.accepting)[0])


def test_pruned_device_api_and_errors():
    import torch
    d = W.random_dfa(5000, 3, 0.3, 21)
    dev = torch.device("cuda:0")
    delta = torch.from_numpy(d.delta.view(np.int32)).to(dev)
    acc = torch.from_numpy(d.accepting).to(dev)
    res = B.minimise_device(delta, acc, prune=True, start=17)
    block, nb, _ = oracle.minimise_reachable(d.delta, d.accepting, 17)
    np.testing.assert_array_equal(res.block.cpu().numpy().view(np.uint32), block)
    with pytest.raises(B.DfaError) as e:
        B.minimise(d.delta, d.accepting, prune=True, start=d.n)
    assert e.value.status == B.DFA_EINVAL
    bad = d.delta.copy()
    bad[3, 1] = d.n
    with pytest.raises(B.DfaError) as e:
        B.minimise(bad, d.accepting, prune=True)
    assert e.value.status == B.DFA_EINVAL


@pytest.mark.parametrize("algorithm", ["leader", "sort"])
def test_pruned_with_other_algorithms(algorithm):
    """Pruning composes with the other refinement algorithms: the same ids."""
    d = W.random_dfa(20000, 3, 0.3, 61)
    res = B.minimise(d.delta, d.accepting, tc="off", prune=True, start=3, algorithm=algorithm)
    block, nb, nr = oracle.minimise_reachable(d.delta, d.accepting, 3)
    np.testing.assert_array_equal(res.block, block)
    assert res.stats["num_blocks"] == nb and res.stats["reachable"] == nr
