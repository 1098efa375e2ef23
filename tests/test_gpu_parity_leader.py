"""GPU parity of the leader rounds (naivePR, Section 3.2, Algorithm 2) and of
transPR (Algorithm 5 followed by naivePR) against the CPU oracle.

Both sides elect the smallest separated state as the new leader, so the
partition after every round, and with it the round counts, are deterministic:
partitions are compared element by element, rounds and separating rounds
exactly.  Families whose oracle run would take too long are checked against
Table 2's closed forms instead.
"""
import numpy as np
import pytest

import oracle
from paper_2508_20735_amd import binding as B
from paper_2508_20735_amd import workloads as W

pytestmark = pytest.mark.gpu

LOOPS = ["host", "chunk", "graph"]


def check_leader(d, tc="off", loop="graph", quotient=False, ref=None):
    res = B.minimise(d.delta, d.accepting, tc=tc, loop=loop, quotient=quotient, start=d.start,
                     algorithm="leader")
    if ref is None:
        ref = (oracle.naive_pr_tc(d.delta, d.accepting) if tc == "on"
               else oracle.naive_pr(d.delta, d.accepting))
    block, nb, rounds, changing = ref
    np.testing.assert_array_equal(res.block, block)
    st = res.stats
    assert st["num_blocks"] == nb
    if tc in ("off", "on"):
        assert (st["rounds"], st["changing_rounds"]) == (rounds, changing)
        assert st["tc_used"] == (1 if tc == "on" else 0)
    if quotient:
        qn, qd, qa, qs = oracle.quotient(d.delta, d.accepting, block, d.start)
        gn, gd, ga, gs = res.quotient
        assert gn == qn and gs == qs
        np.testing.assert_array_equal(gd, qd)
        np.testing.assert_array_equal(ga, qa)
    return res


@pytest.mark.parametrize("n,k,p,seed", [
    (1, 1, 0.5, 1), (2, 1, 0.5, 2), (3, 2, 0.5, 3), (63, 2, 0.3, 4), (64, 3, 0.5, 5),
    (65, 2, 0.5, 6), (257, 5, 0.5, 9), (1000, 3, 0.2, 10), (4097, 8, 0.4, 11),
])
@pytest.mark.parametrize("loop", LOOPS)
def test_leader_random_small(n, k, p, seed, loop):
    d = W.random_dfa(n, k, p, seed)
    check_leader(d, loop=loop, quotient=True)


@pytest.mark.parametrize("loop", LOOPS)
def test_leader_shared_rows(loop):
    """Many states with equal rows: large blocks whose separated states go
    through the workgroup election tables and the global slots together."""
    d = W.random_dfa(20000, 3, 0.3, 99)
    rng = np.random.default_rng(5)
    src = rng.integers(0, 200, 19000)
    dst = rng.integers(200, d.n, 19000)
    d.delta[dst] = d.delta[src]
    d.accepting[dst] = d.accepting[src]
    check_leader(d, loop=loop, quotient=True)


def test_leader_degenerate():
    # one state; all accepting; all rejecting; only identity letters
    for n, acc in ((1, [1]), (5, [1] * 5), (5, [0] * 5)):
        d = W.DFA(np.array([[(q + 1) % n] for q in range(n)], dtype=np.uint32),
                  np.array(acc, dtype=np.uint8), 0)
        check_leader(d)
    ident = W.DFA(np.tile(np.arange(6, dtype=np.uint32)[:, None], (1, 3)),
                  np.array([0, 1, 0, 1, 1, 0], dtype=np.uint8), 0)
    res = check_leader(ident)
    assert res.stats["k_eff"] == 0 and res.stats["rounds"] == 1


def test_leader_max_rounds():
    d = W.fibonacci(10)  # 89 states, 88 rounds
    with pytest.raises(B.DfaError) as e:
        B.minimise(d.delta, d.accepting, tc="off", max_rounds=5, algorithm="leader")
    assert e.value.status == B.DFA_ELIMIT


@pytest.mark.parametrize("i", [5, 8, 12])
@pytest.mark.parametrize("tc", ["off", "on"])
def test_leader_fibonacci(i, tc):
    check_leader(W.fibonacci(i), tc=tc, quotient=True)


def test_leader_table2_fib18():
    """Table 2 row Fib_18: 6,765 states, all distinct, 6,764 naivePR
    iterations (the oracle agrees; here the GPU is compared with both)."""
    d = W.fibonacci(19)
    res = check_leader(d, loop="graph")
    assert res.stats["rounds"] == 6764 and res.stats["num_blocks"] == 6765


@pytest.mark.parametrize("n", [3, 8, 15])
@pytest.mark.parametrize("tc", ["off", "on"])
def test_leader_bitsplitter(n, tc):
    check_leader(W.bitsplitter(n), tc=tc)


def test_leader_table2_b20_closed_form():
    """Table 2, B_20: 2^20 states, 19 letters, minimal, naivePR separates in
    n - 1 = 19 rounds (the 20th finds nothing)."""
    d = W.bitsplitter(20)
    res = B.minimise(d.delta, d.accepting, tc="off", algorithm="leader")
    assert res.stats["num_blocks"] == 2 ** 20
    assert res.stats["changing_rounds"] == 19 and res.stats["rounds"] == 20
    np.testing.assert_array_equal(res.block, np.arange(2 ** 20, dtype=np.uint32))


def test_leader_fig1_and_chain_with_tail():
    check_leader(W.fig1_chain(), tc="on")
    check_leader(W.fig1_chain(), tc="off")
    d = W.chain_with_tail(2 ** 10, 2 ** 10, 7)
    check_leader(d, tc="off")
    check_leader(d, tc="on")
    # AUTO switches to the closure when splitting stalls: same partition
    res = B.minimise(d.delta, d.accepting, tc="auto", algorithm="leader")
    np.testing.assert_array_equal(res.block, oracle.hopcroft(d.delta, d.accepting)[0])


@pytest.mark.parametrize("seed", range(3))
def test_leader_equivalence(seed):
    a = W.random_dfa(3000, 3, 0.3, 200 + seed)
    perm, _ = W.permuted_copy(a, 300 + seed)
    mut, _ = W.mutate_one(a, 400 + seed)
    for other in (perm, mut):
        expect = oracle.equiv_hk(a.delta, a.accepting, a.start,
                                 other.delta, other.accepting, other.start)
        got, st = B.equivalent(a, other, tc="off", algorithm="leader")
        assert got == expect
        sig, _ = B.equivalent(a, other, tc="off")
        assert sig == expect


def test_leader_equivalence_families():
    f = W.fibonacci(10)
    got, _ = B.equivalent(f, W.permuted_copy(f, 1)[0], tc="on", algorithm="leader")
    assert got
    bs = W.bitsplitter(8)
    mut, _ = W.mutate_one(bs, 3)
    got, _ = B.equivalent(bs, mut, tc="off", algorithm="leader")
    assert got == oracle.equiv_hk(bs.delta, bs.accepting, bs.start,
                                  mut.delta, mut.accepting, mut.start)


def test_leader_rejected_by_batch_calls():
    d = W.random_dfa(100, 2, 0.5, 1)
    o = B.options(algorithm="leader")
    assert o.algorithm == 1
    with pytest.raises(B.DfaError) as e:
        B.minimise_batch([d, d], algorithm="leader")
    assert e.value.status == B.DFA_EINVAL
