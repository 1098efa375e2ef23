"""GPU parity of sort-based grouping (the grouping of sortPR, Section 3.3,
Algorithm 4: a stable radix sort of the key hashes, runs split by comparing
keys) against the oracle's Moore rounds, and of both groupings under forced
hash collisions.

Sort grouping computes the same partition after every round as the table, so
partitions, rounds and separating rounds match the oracle exactly.
"""
import numpy as np
import pytest

import oracle
from paper_2508_20735_amd import binding as B
from paper_2508_20735_amd import workloads as W

pytestmark = pytest.mark.gpu


def check_sort(d, tc="off", loop="graph", quotient=False, algorithm="sort"):
    res = B.minimise(d.delta, d.accepting, tc=tc, loop=loop, quotient=quotient, start=d.start,
                     algorithm=algorithm)
    block, nb, rounds, changing = oracle.moore(d.delta, d.accepting)
    np.testing.assert_array_equal(res.block, block)
    assert res.stats["num_blocks"] == nb
    if tc == "off":
        assert (res.stats["rounds"], res.stats["changing_rounds"]) == (rounds, changing)
    if quotient:
        qn, qd, qa, qs = oracle.quotient(d.delta, d.accepting, block, d.start)
        gn, gd, ga, gs = res.quotient
        assert gn == qn and gs == qs
        np.testing.assert_array_equal(gd, qd)
        np.testing.assert_array_equal(ga, qa)
    return res


@pytest.mark.parametrize("n,k,p,seed", [
    (1, 1, 0.5, 1), (2, 1, 0.5, 2), (3, 2, 0.5, 3), (63, 2, 0.3, 4), (64, 3, 0.5, 5),
    (257, 5, 0.5, 9), (4095, 2, 0.5, 14), (4097, 8, 0.4, 11), (12345, 9, 0.3, 12),
    (70000, 4, 0.2, 15),
])
@pytest.mark.parametrize("loop", ["host", "graph"])
def test_sort_random(n, k, p, seed, loop):
    check_sort(W.random_dfa(n, k, p, seed), loop=loop, quotient=True)


def test_sort_shared_rows_long_runs():
    """Many equal keys: long runs in the sorted order (sort tiles of 4,096
    elements and several radix tiles per digit)."""
    d = W.random_dfa(60000, 3, 0.3, 99)
    rng = np.random.default_rng(5)
    src = rng.integers(0, 50, 55000)
    dst = rng.integers(50, d.n, 55000)
    d.delta[dst] = d.delta[src]
    d.accepting[dst] = d.accepting[src]
    check_sort(d, quotient=True)


def test_sort_families_and_closure():
    check_sort(W.fibonacci(12), tc="off")
    check_sort(W.fibonacci(12), tc="on")
    check_sort(W.bitsplitter(12), tc="off")
    check_sort(W.chain_with_tail(1 << 10, 1 << 10, 7), tc="auto")


def test_sort_equivalence():
    a = W.random_dfa(20000, 4, 0.1, 31)
    perm, _ = W.permuted_copy(a, 32)
    mut, _ = W.mutate_one(a, 33)
    for other in (perm, mut):
        expect = oracle.equiv_hk(a.delta, a.accepting, a.start, other.delta, other.accepting,
                                 other.start)
        got, _ = B.equivalent(a, other, tc="off", algorithm="sort")
        assert got == expect


def test_sort_large_config_minimise():
    """The 2^22-state, 4-letter workload (seed 2) with sort grouping: the
    same partition as Hopcroft and Moore's round count."""
    d = W.cfg_large()
    res = B.minimise(d.delta, d.accepting, tc="off", algorithm="sort")
    hb, hnb = oracle.hopcroft(d.delta, d.accepting)
    np.testing.assert_array_equal(res.block, hb)
    assert res.stats["num_blocks"] == hnb


@pytest.fixture
def restore_tuning():
    saved = B.get_tuning()
    yield
    B.set_tuning(**saved)


@pytest.mark.parametrize("algorithm", ["signature", "sort"])
@pytest.mark.parametrize("bits", [3, 12])
def test_forced_hash_collisions(restore_tuning, algorithm, bits):
    """Only the low `bits` bits of every key hash are kept, so thousands of
    distinct keys share a hash: table probes compare rows after every tag
    match, sorted runs hold interleaved keys.  Results stay exact."""
    B.set_tuning(hash_bits=bits)
    for lds in (True, False):
        d = W.random_dfa(3000, 3, 0.3, 50 + bits)
        res = B.minimise(d.delta, d.accepting, tc="off", algorithm=algorithm, lds_stage=lds)
        block, nb, rounds, changing = oracle.moore(d.delta, d.accepting)
        np.testing.assert_array_equal(res.block, block)
        assert (res.stats["rounds"], res.stats["changing_rounds"]) == (rounds, changing)


def test_sort_transpr_and_leader_equivalence_agree():
    """Equivalence verdicts agree across the three algorithms and the closure
    modes on the paper's families."""
    cases = [(W.fibonacci(11), W.permuted_copy(W.fibonacci(11), 2)[0]),
             (W.bitsplitter(9), W.mutate_one(W.bitsplitter(9), 4)[0]),
             (W.random_dfa(5000, 4, 0.2, 70), W.mutate_one(W.random_dfa(5000, 4, 0.2, 70), 71)[0])]
    for a, b in cases:
        expect = oracle.equiv_hk(a.delta, a.accepting, a.start, b.delta, b.accepting, b.start)
        for alg in ("signature", "sort", "leader"):
            for tc in ("off", "on"):
                got, _ = B.equivalent(a, b, tc=tc, algorithm=alg)
                assert got == expect, (alg, tc)
