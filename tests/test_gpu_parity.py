"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Partitions are compared element by element after canonical renumbering (block
id = smallest state of the block), which both sides produce; round counts are
compared with the oracle's Moore rounds (plain letters, or the closure letters
built by Algorithm 5); verdicts with union-find Hopcroft-Karp and the oracle's
product exploration.  Integer work: every comparison is exact.
"""
import concurrent.futures
import ctypes
import os

import numpy as np
import pytest

import oracle
from paper_2508_20735_amd import binding as B
from paper_2508_20735_amd import workloads as W

pytestmark = pytest.mark.gpu

LOOPS = ["host", "chunk", "graph"]


def _ref(d):
    block, nb, rounds, changing = oracle.moore(d.delta, d.accepting)
    return block, nb, rounds, changing


def _ref_tc(d):
    return oracle.minimise_tc(d.delta, d.accepting)


def check_minimise(d, tc="off", loop="graph", lds=2, quotient=False, ref=None):
    res = B.minimise(d.delta, d.accepting, tc=tc, loop=loop, lds_stage=lds, quotient=quotient,
                     start=d.start)
    block, nb, rounds, changing = ref if ref is not None else _ref(d)
    np.testing.assert_array_equal(res.block, block)
    st = res.stats
    assert st["num_blocks"] == nb
    if tc == "off":
        assert st["changing_rounds"] == changing and st["rounds"] == rounds
        assert st["tc_used"] == 0
    if quotient:
        qn, qd, qa, qs = oracle.quotient(d.delta, d.accepting, block, d.start)
        gn, gd, ga, gs = res.quotient
        assert gn == qn and gs == qs
        np.testing.assert_array_equal(gd, qd)
        np.testing.assert_array_equal(ga, qa)
    return res


# ---------------------------------------------------------------- small / ragged

@pytest.mark.parametrize("n,k,p,seed", [
    (1, 1, 0.5, 1), (2, 1, 0.5, 2), (3, 2, 0.5, 3), (63, 2, 0.3, 4), (64, 3, 0.5, 5),
    (65, 2, 0.5, 6), (255, 4, 0.1, 7), (256, 2, 0.5, 8), (257, 5, 0.5, 9),
    (1000, 3, 0.2, 10), (4097, 8, 0.4, 11), (12345, 9, 0.3, 12), (5000, 17, 0.5, 13),
    (20000, 16, 0.3, 21), (3000, 15, 0.4, 22),
])
@pytest.mark.parametrize("loop", LOOPS)
def test_random_small(n, k, p, seed, loop):
    d = W.random_dfa(n, k, p, seed)
    check_minimise(d, tc="off", loop=loop, quotient=True)


@pytest.mark.parametrize("lds", [True, False, 2])
def test_lds_and_global_grouping_agree(lds):
    d = W.random_dfa(30000, 3, 0.3, 99)
    # duplicate rows: many states share signatures, stressing the grouping
    rng = np.random.default_rng(5)
    src = rng.integers(0, d.n, 20000)
    dst = rng.integers(0, d.n, 20000)
    d.delta[dst] = d.delta[src]
    d.accepting[dst] = d.accepting[src]
    check_minimise(d, tc="off", loop="chunk", lds=lds, quotient=True)


def test_config_small_all_modes():
    """n = 10,000, k = 2, p = 0.5, seed 1."""
    d = W.cfg_small()
    ref = _ref(d)
    for loop in LOOPS:
        for tc in ("off", "auto"):
            for lds in (True, False, 2):
                check_minimise(d, tc=tc, loop=loop, lds=lds, ref=ref)
    res = check_minimise(d, tc="on", loop="graph", ref=ref)
    block, nb, rounds, changing = _ref_tc(d)
    assert res.stats["changing_rounds"] == changing and res.stats["tc_used"] == 1


def test_degenerate_inputs():
    # all accepting / none accepting: one block, one confirming round
    for v in (0, 1):
        d = W.random_dfa(777, 3, 0.5, 3)
        d.accepting[:] = v
        res = check_minimise(d, tc="off", quotient=True)
        assert (res.block == 0).all() and res.stats["rounds"] == 1
    # every letter the identity: the signature is the block id alone
    n = 300
    d = W.DFA(np.tile(np.arange(n, dtype=np.uint32)[:, None], (1, 3)),
              (np.arange(n) % 3 == 0).astype(np.uint8), 0)
    for tc in ("off", "on", "auto"):
        res = check_minimise(d, tc=tc)
        assert res.stats["k_eff"] == 0
    # a single state
    d = W.DFA(np.zeros((1, 4), dtype=np.uint32), np.ones(1, dtype=np.uint8), 0)
    for tc in ("off", "on"):
        check_minimise(d, tc=tc, quotient=True)


def test_invalid_arguments():
    d = W.random_dfa(100, 2, 0.5, 1)
    bad = d.delta.copy()
    bad[57, 1] = 100
    with pytest.raises(B.DfaError) as e:
        B.minimise(bad, d.accepting)
    assert e.value.status == B.DFA_EINVAL
    with pytest.raises(B.DfaError) as e:
        B.minimise(d.delta, d.accepting, start=100)
    assert e.value.status == B.DFA_EINVAL
    other = W.random_dfa(50, 3, 0.5, 2)
    with pytest.raises(B.DfaError) as e:
        B.equivalent(d, other)
    assert e.value.status == B.DFA_EINVAL
    # the library is still usable afterwards
    check_minimise(d)


def test_max_rounds_limit():
    d = W.fibonacci(12)  # 233 states, 231 refining rounds
    with pytest.raises(B.DfaError) as e:
        B.minimise(d.delta, d.accepting, tc="off", max_rounds=10)
    assert e.value.status == B.DFA_ELIMIT


def test_deterministic_repeats():
    d = W.random_dfa(50000, 4, 0.1, 8)
    first = B.minimise(d.delta, d.accepting, tc="off").block
    for loop in LOOPS:
        np.testing.assert_array_equal(B.minimise(d.delta, d.accepting, tc="off",
                                                 loop=loop).block, first)


# ---------------------------------------------------------------- the paper's families

@pytest.mark.parametrize("i", [5, 8, 12, 16])
def test_fibonacci(i):
    d = W.fibonacci(i)
    ref = _ref(d)
    check_minimise(d, tc="off", loop="chunk", ref=ref)
    res = check_minimise(d, tc="on", ref=ref)
    _, _, _, changing_tc = _ref_tc(d)
    assert res.stats["changing_rounds"] == changing_tc
    check_minimise(d, tc="auto", ref=ref)


@pytest.mark.parametrize("n", [2, 3, 8, 14])
def test_bitsplitter(n):
    d = W.bitsplitter(n)
    res = check_minimise(d, tc="off", loop="graph")
    assert res.stats["changing_rounds"] == n - 1
    check_minimise(d, tc="on")


def test_fig1_chain_closure():
    d = W.fig1_chain()
    res = check_minimise(d, tc="off", loop="host")
    assert res.stats["changing_rounds"] == 8
    res = check_minimise(d, tc="on")
    _, _, _, changing_tc = _ref_tc(d)
    assert res.stats["changing_rounds"] == changing_tc


@pytest.mark.parametrize("M", [6, 10, 14])
def test_chain_round_counts(M):
    N = 2 ** M
    d = W.chain_with_tail(N, 0, seed=0)
    hb, nb = oracle.hopcroft(d.delta, d.accepting)
    # closed forms (derived in the oracle tests): N - 2 plain rounds, M - 1 with the closure
    ref = (hb, nb, N - 1, N - 2)
    res = check_minimise(d, tc="off", loop="chunk", ref=ref)
    assert res.stats["changing_rounds"] == N - 2
    res = check_minimise(d, tc="on", ref=ref)
    assert res.stats["changing_rounds"] == M - 1


def test_chain_with_tail_medium_auto():
    d = W.chain_with_tail(1 << 14, 1 << 14, seed=3)
    hb, nb = oracle.hopcroft(d.delta, d.accepting)
    for tc in ("on", "auto"):
        res = B.minimise(d.delta, d.accepting, tc=tc)
        np.testing.assert_array_equal(res.block, hb)
        assert res.stats["tc_used"] == 1
    tb, _, _, changing_tc = _ref_tc(d)
    res = B.minimise(d.delta, d.accepting, tc="on")
    assert res.stats["changing_rounds"] == changing_tc


@pytest.mark.parametrize("i", [5, 12])
def test_cycle_and_extended_bitsplitter(i):
    for d in (W.cycle(i + 10), W.extended_bitsplitter(i)):
        check_minimise(d, tc="off", quotient=True)
        check_minimise(d, tc="auto")


def test_column_lists_across_calls():
    """Consecutive calls whose signatures use different column lists (all
    letters, a dropped identity letter, the closure levels, then all letters
    again): the device's list is replaced whenever it differs."""
    d = W.random_dfa(30000, 3, 0.3, 88)
    ident = W.DFA(d.delta.copy(), d.accepting.copy(), 0)
    ident.delta[:, 1] = np.arange(d.n, dtype=np.uint32)
    for case, tc in ((d, "off"), (ident, "off"), (d, "off"), (d, "on"), (ident, "on"),
                     (d, "off"), (ident, "off")):
        res = B.minimise(case.delta, case.accepting, tc=tc)
        hb, hnb = oracle.hopcroft(case.delta, case.accepting)
        np.testing.assert_array_equal(res.block, hb)
        assert res.stats["num_blocks"] == hnb


# ---------------------------------------------------------------- equivalence

def test_equivalence_tiny_random_pairs():
    rng = np.random.default_rng(7)
    seen = {True: 0, False: 0}
    for _ in range(300):
        nA, nB, k = int(rng.integers(1, 6)), int(rng.integers(1, 6)), int(rng.integers(1, 3))
        A = W.DFA(rng.integers(0, nA, (nA, k)).astype(np.uint32),
                  rng.integers(0, 2, nA).astype(np.uint8), int(rng.integers(0, nA)))
        Bd = W.DFA(rng.integers(0, nB, (nB, k)).astype(np.uint32),
                   rng.integers(0, 2, nB).astype(np.uint8), int(rng.integers(0, nB)))
        ref = oracle.equiv_hk(A.delta, A.accepting, A.start, Bd.delta, Bd.accepting, Bd.start)
        got, _ = B.equivalent(A, Bd, loop="chunk")
        assert got == ref
        seen[ref] += 1
    assert seen[True] > 10 and seen[False] > 10


@pytest.mark.parametrize("seed", range(4))
def test_equivalence_permuted_and_mutated(seed):
    d = W.random_dfa(20000 + 1111 * seed, 2 + seed, 0.2, seed)
    perm, _ = W.permuted_copy(d, seed + 10)
    mut, _ = W.mutate_one(d, seed + 20)
    for loop in LOOPS:
        got, st = B.equivalent(d, perm, loop=loop)
        assert got
        got, _ = B.equivalent(d, mut, loop=loop)
        assert got == oracle.equiv_hk(d.delta, d.accepting, d.start, mut.delta, mut.accepting,
                                      mut.start)


def test_equivalence_families():
    for d in (W.cycle(15), W.extended_bitsplitter(6), W.fibonacci(10)):
        perm, _ = W.permuted_copy(d, 3)
        assert B.equivalent(d, perm)[0]
        assert B.equivalent(d, perm, tc="on")[0]
    F, P = W.memory(8, True), W.memory(8, False)
    assert not B.equivalent(F, P)[0]


# ------------------------------------------- equivalence by product exploration

def test_product_equivalence_tiny_random_pairs():
    """method="product": the breadth-first pair exploration of Section 4 with
    the equivalence test (exactly one accepting side).  Verdicts match the
    oracle's exploration; when equivalent, so does the number of pairs."""
    rng = np.random.default_rng(17)
    seen = {True: 0, False: 0}
    for _ in range(300):
        nA, nB, k = int(rng.integers(1, 6)), int(rng.integers(1, 6)), int(rng.integers(1, 3))
        A = W.DFA(rng.integers(0, nA, (nA, k)).astype(np.uint32),
                  rng.integers(0, 2, nA).astype(np.uint8), int(rng.integers(0, nA)))
        Bd = W.DFA(rng.integers(0, nB, (nB, k)).astype(np.uint32),
                   rng.integers(0, 2, nB).astype(np.uint8), int(rng.integers(0, nB)))
        ref, ref_pairs = oracle.product_bfs(A.delta, A.accepting, A.start, Bd.delta,
                                            Bd.accepting, Bd.start, "equivalence")
        got, st = B.equivalent(A, Bd, method="product")
        assert got == ref
        assert got == oracle.equiv_hk(A.delta, A.accepting, A.start, Bd.delta, Bd.accepting,
                                      Bd.start)
        if ref:
            assert st["reachable"] == ref_pairs
        seen[ref] += 1
    assert seen[True] > 10 and seen[False] > 10


@pytest.mark.parametrize("seed", range(3))
def test_product_equivalence_permuted_and_mutated(seed):
    d = W.random_dfa(20000 + 1111 * seed, 2 + seed, 0.2, seed)
    perm, _ = W.permuted_copy(d, seed + 10)
    mut, _ = W.mutate_one(d, seed + 20)
    got, st = B.equivalent(d, perm, method="product")
    ok, pairs = oracle.product_bfs(d.delta, d.accepting, d.start, perm.delta, perm.accepting,
                                   perm.start, "equivalence")
    assert got and ok and st["reachable"] == pairs and st["rounds"] >= 1
    expect = oracle.equiv_hk(d.delta, d.accepting, d.start, mut.delta, mut.accepting, mut.start)
    assert B.equivalent(d, mut, method="product")[0] == expect
    assert B.equivalent(d, mut, method="union")[0] == expect


def test_product_equivalence_families():
    """Table 4: a DFA against itself explores 2^(n+1) pairs for B'_n and
    fib(n) pairs for C_n; memory_n forgetful and perfect differ."""
    d = W.extended_bitsplitter(10)
    ok, st = B.equivalent(d, d, method="product")
    assert ok and st["reachable"] == 2 ** 11
    c = W.cycle(20)
    ok, st = B.equivalent(c, c, method="product")
    assert ok and st["reachable"] == W.fib_numbers(20)
    F, P = W.memory(9, True), W.memory(9, False)
    assert not B.equivalent(F, P, method="product")[0]
    assert not B.equivalent(P, F, method="product")[0]


def _bfs_dist(delta, start):
    """Breadth-first distance of every state from start (-1: unreachable),
    by a plain level-by-level search."""
    dist = np.full(delta.shape[0], -1, dtype=np.int64)
    dist[start] = 0
    front, depth = np.array([start]), 0
    while front.size:
        nxt = np.unique(delta[front].ravel())
        nxt = nxt[dist[nxt] < 0]
        depth += 1
        dist[nxt] = depth
        front = nxt
    return dist


def test_product_deep_thin_search():
    """C_25 against itself: 121,393 pairs over more levels than one
    workgroup-local launch expands (256), a few hundred pairs per level.  The
    levels expanded are the search depth + 1 (the last level adds nothing)."""
    c = W.cycle(25)
    dist = _bfs_dist(c.delta, c.start)
    depth = int(dist.max())
    assert depth > 256
    ok, st = B.equivalent(c, c, method="product")
    assert ok and st["reachable"] == W.fib_numbers(25) and st["rounds"] == depth + 1
    ok, pairs, st = B.included(c, c)
    assert ok and pairs == W.fib_numbers(25) and st["rounds"] == depth + 1
    # a refuting pair deep in the search: accept, in the copy, one more state
    # among the farthest from the start
    other = W.DFA(c.delta, c.accepting.copy(), c.start)
    far = int(np.flatnonzero((dist == depth) & (c.accepting == 0))[0])
    other.accepting[far] = 1
    expect = oracle.equiv_hk(c.delta, c.accepting, c.start, other.delta, other.accepting,
                             other.start)
    assert B.equivalent(c, other, method="product")[0] == expect
    assert B.included(c, other)[0] == oracle.included(c.delta, c.accepting, c.start,
                                                       other.delta, other.accepting, other.start)
    assert B.included(other, c)[0] == oracle.included(other.delta, other.accepting, other.start,
                                                       c.delta, c.accepting, c.start)


def test_product_equivalence_device_api():
    import torch
    d = W.random_dfa(30000, 3, 0.3, 41)
    perm, _ = W.permuted_copy(d, 42)
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x).view(
        np.int32 if x.dtype == np.uint32 else np.uint8)).to(dev)
    got, st = B.equivalent_device(t(d.delta), t(d.accepting), d.start, t(perm.delta),
                                  t(perm.accepting), perm.start, method="product")
    # the reached pairs are (q, pi(q)) for the states q reachable from the start
    assert got and st["reachable"] == int(np.count_nonzero(oracle.reachable(d.delta, d.start)))


# ---------------------------------------------------------------- inclusion

@pytest.mark.parametrize("n", [3, 5, 9, 12, 16])
def test_inclusion_memory_table5(n):
    """Table 5: forgetful memory_n is included in perfect memory_n, and the
    explored product has (2n+1) 2^(n-2) states; the converse fails."""
    F, P = W.memory(n, True), W.memory(n, False)
    ok, visited, _ = B.included(F, P)
    ref_ok, ref_visited = oracle.product_bfs(F.delta, F.accepting, 0, P.delta, P.accepting, 0)
    assert ok and ref_ok and visited == ref_visited
    ok, _, _ = B.included(P, F)
    assert not ok


def test_inclusion_tiny_random_pairs():
    rng = np.random.default_rng(11)
    seen = {True: 0, False: 0}
    for _ in range(300):
        nA, nB, k = int(rng.integers(1, 6)), int(rng.integers(1, 6)), int(rng.integers(1, 3))
        A = W.DFA(rng.integers(0, nA, (nA, k)).astype(np.uint32),
                  rng.integers(0, 2, nA).astype(np.uint8), int(rng.integers(0, nA)))
        Bd = W.DFA(rng.integers(0, nB, (nB, k)).astype(np.uint32),
                   rng.integers(0, 2, nB).astype(np.uint8), int(rng.integers(0, nB)))
        ref, ref_visited = oracle.product_bfs(A.delta, A.accepting, A.start, Bd.delta,
                                              Bd.accepting, Bd.start)
        got, visited, _ = B.included(A, Bd)
        assert got == ref
        if ref:
            assert visited == ref_visited
        seen[ref] += 1
    assert seen[True] > 10 and seen[False] > 10


def test_inclusion_self_products():
    """Table 4: self-products of B'_n and C_n have 2^(n+1) and fib(n) pairs."""
    d = W.extended_bitsplitter(10)
    ok, visited, _ = B.included(d, d)
    assert ok and visited == 2 ** 11
    c = W.cycle(20)
    ok, visited, _ = B.included(c, c)
    assert ok and visited == W.fib_numbers(20)


# ---------------------------------------------------------------- device API

def test_device_api_matches_host_api():
    import torch
    d = W.random_dfa(70000, 4, 0.1, 31)
    ref = _ref(d)
    dev = torch.device("cuda:0")
    delta = torch.from_numpy(d.delta.view(np.int32)).to(dev)
    acc = torch.from_numpy(d.accepting).to(dev)
    res = B.minimise_device(delta, acc, tc="off", quotient=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(res.block.cpu().numpy().view(np.uint32), ref[0])
    qn, qd, qa, qs = oracle.quotient(d.delta, d.accepting, ref[0], 0)
    gn, gd, ga, gs = res.quotient
    assert gn == qn and gs == qs
    np.testing.assert_array_equal(gd.cpu().numpy().view(np.uint32), qd)
    np.testing.assert_array_equal(ga.cpu().numpy(), qa)
    perm, _ = W.permuted_copy(d, 1)
    pdelta = torch.from_numpy(perm.delta.view(np.int32)).to(dev)
    pacc = torch.from_numpy(perm.accepting).to(dev)
    assert B.equivalent_device(delta, acc, 0, pdelta, pacc, perm.start)[0]
    ok, visited, _ = B.included_device(delta, acc, 0, pdelta, pacc, perm.start)
    assert ok


# ---------------------------------------------------------------- full-size workloads

@pytest.fixture(scope="module")
def large():
    d = W.cfg_large()
    block, nb, rounds, changing = oracle.moore(d.delta, d.accepting)
    return d, (block, nb, rounds, changing)


def test_config_large_minimise(large):
    """n = 2^22, k = 4, p = 0.1: every state compared with the oracle."""
    d, ref = large
    for loop in ("graph", "host", "chunk"):
        res = check_minimise(d, tc="auto", loop=loop, ref=ref)
        assert res.stats["tc_used"] == 0
        assert res.stats["changing_rounds"] == ref[3]


def test_config_large_equivalence(large):
    d, _ = large
    perm, _ = W.permuted_copy(d, W.CFG_LARGE_PERM_SEED)
    mut, _ = W.mutate_one(d, W.CFG_LARGE_MUT_SEED)
    assert B.equivalent(d, perm)[0]
    expected = oracle.equiv_hk(d.delta, d.accepting, d.start, mut.delta, mut.accepting, mut.start)
    got, st = B.equivalent(d, mut)
    assert got == expected
    # twins (q and its copy) separate in a few rounds: no closure is built
    assert st["tc_used"] == 0


def test_config_large_bench_step_configuration(large):
    """The benchmark's step as it is timed: device tensors, chunked rounds
    with only the signature kernel carrying events.  Minimisation ids,
    quotient and both verdicts equal the oracle's."""
    import torch
    d, ref = large
    perm, _ = W.permuted_copy(d, W.CFG_LARGE_PERM_SEED)
    mut, _ = W.mutate_one(d, W.CFG_LARGE_MUT_SEED)
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x).view(
        np.int32 if x.dtype == np.uint32 else np.uint8)).to(dev)
    A_d, A_a = t(d.delta), t(d.accepting)
    try:
        B.profile_only("k_signature")
        B.profile_enable(True)
        res = B.minimise_device(A_d, A_a, quotient=True, loop="chunk")
        e1, _ = B.equivalent_device(A_d, A_a, d.start, t(perm.delta), t(perm.accepting),
                                    perm.start, loop="chunk")
        e2, _ = B.equivalent_device(A_d, A_a, d.start, t(mut.delta), t(mut.accepting),
                                    mut.start, loop="chunk")
        timed = B.profile_read()
    finally:
        B.profile_enable(False)
        B.profile_only(None)
    np.testing.assert_array_equal(res.block.cpu().numpy().view(np.uint32), ref[0])
    qn, qd, qa, qs = oracle.quotient(d.delta, d.accepting, ref[0], d.start)
    gn, gd, ga, gs = res.quotient
    assert gn == qn and gs == qs
    np.testing.assert_array_equal(gd.cpu().numpy().view(np.uint32), qd)
    np.testing.assert_array_equal(ga.cpu().numpy(), qa)
    assert e1 is True
    assert e2 == oracle.equiv_hk(d.delta, d.accepting, d.start, mut.delta, mut.accepting,
                                 mut.start)
    assert set(timed) == {"k_signature"}


def test_config_chain_closure():
    """Chain of 2^20 states plus a 2^20-state random tail with the closure
    (on and auto): the partition against Hopcroft, and with the closure built
    first the exact round count of the oracle's Moore rounds over the closure
    letters (19 = log2(2^20) - 1, the chain's closed form)."""
    d = W.cfg_chain()
    hb, nb = oracle.hopcroft(d.delta, d.accepting)
    for tc in ("on", "auto"):
        res = B.minimise(d.delta, d.accepting, tc=tc)
        np.testing.assert_array_equal(res.block, hb)
        assert res.stats["num_blocks"] == nb == d.n
        # on demand (auto) the closure is built once the random tail is all
        # singletons; built first (on), its columns are judged again once a
        # quarter of the states are.  Either way, on the chain the second
        # letter is the identity at every level and the first letter's level
        # 21 repeats level 20, so 21 of the 2 x 22 columns remain
        assert res.stats["k_eff"] == 21 and res.stats["tc_levels"] == 21
    _, tnb, trounds, tchanging = oracle.minimise_tc(d.delta, d.accepting)
    assert tchanging == 19
    res = B.minimise(d.delta, d.accepting, tc="on")
    assert res.stats["changing_rounds"] == tchanging
    assert res.stats["rounds"] == trounds and res.stats["num_blocks"] == tnb


@pytest.mark.timeout(900)
def test_config_chain_plain_full_size():
    """The same DFA refined on its two input letters only: 2^20 - 2 refining
    rounds (the chain's closed form; the tail is stable within a few rounds),
    and the partition equals Hopcroft's."""
    d = W.cfg_chain()
    hb, nb = oracle.hopcroft(d.delta, d.accepting)
    res = B.minimise(d.delta, d.accepting, tc="off")
    np.testing.assert_array_equal(res.block, hb)
    st = res.stats
    assert st["num_blocks"] == nb == d.n and st["tc_used"] == 0
    assert st["changing_rounds"] == (1 << 20) - 2 and st["rounds"] == (1 << 20) - 1


# ---------------------------------------------------------------- kernel variants

@pytest.fixture
def restore_tuning():
    saved = B.get_tuning()
    yield
    B.set_tuning(**saved)


@pytest.mark.parametrize("label_rounds", [0, 1, 2])
@pytest.mark.parametrize("cached_probe", [0, 1])
@pytest.mark.parametrize("grid_cap", [0, 64, 8192])
def test_tuning_variants_agree(restore_tuning, label_rounds, cached_probe, grid_cap):
    """Every launch shape and kernel variant gives the oracle's partition."""
    B.set_tuning(label_rounds=label_rounds, cached_probe=cached_probe, round_grid_cap=grid_cap,
                 label_grid_cap=grid_cap)
    cases = [W.random_dfa(20011, 4, 0.1, 5), W.random_dfa(3001, 2, 0.5, 6),
             W.random_dfa(5003, 7, 0.3, 7), W.fibonacci(11), W.bitsplitter(9)]
    # stable after round 0 and after round 1 (label ids turned into state ids)
    cases.append(W.DFA(np.array([[1], [1]], dtype=np.uint32), np.array([0, 1], np.uint8), 0))
    cases.append(W.DFA(np.array([[2], [1], [2]], dtype=np.uint32), np.array([0, 0, 1], np.uint8), 0))
    for d in cases:
        for lds in (True, False, 2):
            check_minimise(d, tc="off", loop="chunk", lds=lds, quotient=True)
    d = cases[0]
    perm, _ = W.permuted_copy(d, 3)
    assert B.equivalent(d, perm)[0]
    mut, _ = W.mutate_one(d, 4)
    assert B.equivalent(d, mut)[0] == oracle.equiv_hk(d.delta, d.accepting, 0, mut.delta,
                                                     mut.accepting, mut.start)


# ---------------------------------------------------------------- batches

def _mixed_batch(seed, count):
    rng = np.random.default_rng(seed)
    dfas = []
    for i in range(count):
        n = int(np.exp(rng.uniform(0, np.log(6000))))
        k = int(rng.integers(1, 9))
        d = W.random_dfa(n, k, float(rng.uniform(0.0, 0.6)), int(rng.integers(1 << 30)))
        if i % 5 == 0 and n > 4:  # duplicated rows: non-trivial blocks
            src = rng.integers(0, n, n // 2)
            dst = rng.integers(0, n, n // 2)
            d.delta[dst] = d.delta[src]
            d.accepting[dst] = d.accepting[src]
        dfas.append(d)
    dfas.append(W.DFA(np.zeros((1, 3), np.uint32), np.ones(1, np.uint8), 0))   # one state
    dfas.append(W.fibonacci(9))                                                  # 55 rounds
    dfas.append(W.bitsplitter(7))
    return dfas


@pytest.mark.parametrize("loop", ["chunk", "graph"])
def test_minimise_batch_matches_single(loop):
    dfas = _mixed_batch(3, 150)
    blocks, nb, rounds, st = B.minimise_batch(dfas, loop=loop)
    assert st["count"] == len(dfas)
    for i, d in enumerate(dfas):
        ref, rnb, rrounds, rchanging = oracle.moore(d.delta, d.accepting)
        np.testing.assert_array_equal(blocks[i], ref, err_msg=f"dfa {i}")
        assert nb[i] == rnb and rounds[i] == rrounds, i
    assert st["rounds"] == max(rounds)


def test_minimise_batch_offsets_and_errors():
    dfas = _mixed_batch(4, 20)
    sizes = [d.n for d in dfas]
    # reversed placement with gaps
    offsets, pos = [0] * len(dfas), 0
    for i in reversed(range(len(dfas))):
        offsets[i] = pos
        pos += sizes[i] + 3
    blocks, nb, rounds, _ = B.minimise_batch(dfas, offsets=offsets)
    for i, d in enumerate(dfas):
        np.testing.assert_array_equal(blocks[i], oracle.hopcroft(d.delta, d.accepting)[0])
    bad = [W.random_dfa(10, 2, 0.5, 1), W.random_dfa(20, 2, 0.5, 2)]
    bad[1].delta[3, 1] = 20
    with pytest.raises(B.DfaError) as e:
        B.minimise_batch(bad)
    assert e.value.status == B.DFA_EINVAL


def test_equivalent_batch():
    rng = np.random.default_rng(9)
    pairs, expected = [], []
    for i in range(120):
        n = int(rng.integers(1, 3000))
        k = int(rng.integers(1, 7))
        d = W.random_dfa(n, k, float(rng.uniform(0.05, 0.6)), 1000 + i)
        if i % 3 == 0:
            other, _ = W.permuted_copy(d, i)
        elif i % 3 == 1:
            other, _ = W.mutate_one(d, i)
        else:
            m = int(rng.integers(1, 40))
            other = W.random_dfa(m, k, 0.5, 5000 + i)
        pairs.append((d, other))
        expected.append(oracle.equiv_hk(d.delta, d.accepting, d.start, other.delta,
                                        other.accepting, other.start))
    verdicts, st = B.equivalent_batch(pairs)
    assert list(verdicts) == expected
    assert sum(expected) > 20 and len(expected) - sum(expected) > 20


def test_batch_workload_small_slice():
    """The first DFAs of the 4,096-DFA batch workload (sizes log-uniform in
    [64, 65536], k in 2..8) and their equivalence pairs."""
    items = W.batch_workload(count=64, paired_from=32)
    dfas = [it.dfa for it in items]
    blocks, nb, rounds, _ = B.minimise_batch(dfas)
    for i, d in enumerate(dfas):
        ref, rnb, rrounds, _ = oracle.moore(d.delta, d.accepting)
        np.testing.assert_array_equal(blocks[i], ref)
        assert rounds[i] == rrounds
    pairs = [(it.dfa, it.pair) for it in items if it.pair is not None]
    verdicts, _ = B.equivalent_batch(pairs)
    for (a, b), v in zip(pairs, verdicts):
        assert v == oracle.equiv_hk(a.delta, a.accepting, a.start, b.delta, b.accepting, b.start)


def _oracle_map(fn, items):
    """The oracle over many inputs on the host's cores (its C calls release
    the interpreter lock)."""
    workers = max(1, min(16, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


def test_batch_workload_full_size():
    """The 4,096-DFA batch workload at full size, in the launch configuration
    the benchmark times (one batched call per kind): every DFA's partition
    and round count equal the oracle's Moore rounds state by state, and all
    2,048 equivalence verdicts equal union-find Hopcroft-Karp's."""
    items = W.batch_workload(count=4096, paired_from=2048)
    dfas = [it.dfa for it in items]
    blocks, nb, rounds, _ = B.minimise_batch(dfas)
    refs = _oracle_map(lambda d: oracle.moore(d.delta, d.accepting), dfas)
    for i, (d, ref) in enumerate(zip(dfas, refs)):
        np.testing.assert_array_equal(blocks[i], ref[0], err_msg=f"dfa {i}")
        assert (nb[i], rounds[i]) == (ref[1], ref[2]), i
    pairs = [(it.dfa, it.pair) for it in items if it.pair is not None]
    verdicts, _ = B.equivalent_batch(pairs)
    expect = _oracle_map(lambda ab: oracle.equiv_hk(ab[0].delta, ab[0].accepting, ab[0].start,
                                                    ab[1].delta, ab[1].accepting, ab[1].start),
                         pairs)
    assert list(verdicts) == expect
    assert 0 < sum(expect) < len(expect)


def _served_expected(r):
    if r.kind == "minimise":
        return oracle.hopcroft(r.dfa.delta, r.dfa.accepting)
    return oracle.equiv_hk(r.dfa.delta, r.dfa.accepting, r.dfa.start, r.other.delta,
                           r.other.accepting, r.other.start)


def test_server_serving_workload_full_size():
    """All 96 requests of the serving workload at full size (n up to 4.2M,
    alphabets of 2 to 16 letters, chain DFAs included), through a server with
    the default configuration as the benchmark runs it: every partition equals
    Hopcroft's and every verdict union-find Hopcroft-Karp's."""
    reqs = W.serving_workload(96, rate=1.0)
    with B.Server() as srv:
        tickets = [srv.submit_minimise(r.dfa) if r.kind == "minimise" else
                   srv.submit_equivalent(r.dfa, r.other) for r in reqs]
        results = [srv.wait(t) for t in tickets]
    expected = _oracle_map(_served_expected, reqs)
    kinds = set()
    for i, (r, got, exp) in enumerate(zip(reqs, results, expected)):
        assert got["status"] == 0, i
        if r.kind == "minimise":
            np.testing.assert_array_equal(got["blocks"], exp[0], err_msg=f"request {i}")
            assert got["num_blocks"] == exp[1], i
        else:
            assert got["verdict"] == exp, i
        kinds.add(r.kind)
    assert kinds == {"minimise", "equivalent"}


def test_kernel_timing_all_and_one():
    """Per-kernel event timing: every round kernel, or only the one named
    (the others then run without events); results are unchanged."""
    d = W.random_dfa(50000, 4, 0.1, 77)
    ref = _ref(d)
    try:
        B.profile_only(None)
        B.profile_enable(True)
        res = B.minimise(d.delta, d.accepting, tc="off", loop="chunk")
        every = B.profile_read()
        assert {"k_signature", "k_insert", "k_mark", "k_round_end"} <= set(every)
        B.profile_only("k_signature")
        B.profile_enable(True)
        res2 = B.minimise(d.delta, d.accepting, tc="off", loop="chunk")
        one = B.profile_read()
        assert set(one) == {"k_signature"}
        assert one["k_signature"]["launches"] == every["k_signature"]["launches"]
        assert one["k_signature"]["algorithmic_bytes"] == every["k_signature"]["algorithmic_bytes"]
    finally:
        B.profile_enable(False)
        B.profile_only(None)
    np.testing.assert_array_equal(res.block, ref[0])
    np.testing.assert_array_equal(res2.block, ref[0])


# ---------------------------------------------------------------- serving

def _serving_mix(seed, count):
    """Requests shaped like the serving workload at reduced sizes: 80%
    minimise / 20% equivalence, n log-uniform, k in {2, 4, 8, 16}, 10% chain
    with a random tail."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(100), np.log(40000))))
        k = int(rng.choice([2, 4, 8, 16]))
        if rng.random() < 0.1:
            half = max(n // 2, 2)
            d = W.chain_with_tail(half, n - half, int(rng.integers(1 << 30)), k=k)
        else:
            d = W.random_dfa(n, k, float(rng.uniform(0.05, 0.5)), int(rng.integers(1 << 30)))
        if rng.random() < 0.2:
            other = W.permuted_copy(d, i)[0] if i % 2 else W.mutate_one(d, i)[0]
            reqs.append(("eq", d, other))
        else:
            reqs.append(("min", d, None))
    return reqs


def _expected(req):
    kind, a, b = req
    if kind == "min":
        return oracle.hopcroft(a.delta, a.accepting)[0]
    return oracle.equiv_hk(a.delta, a.accepting, a.start, b.delta, b.accepting, b.start)


def _submit(srv, req):
    kind, a, b = req
    return srv.submit_minimise(a) if kind == "min" else srv.submit_equivalent(a, b)


def test_server_results_alone_and_in_mix():
    reqs = _serving_mix(21, 60)
    expected = [_expected(r) for r in reqs]
    with B.Server(lanes=3, max_group=16, batch_max_states=20000) as srv:
        tickets = [_submit(srv, r) for r in reqs]
        mixed = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    assert st["batched_groups"] > 0 and st["p99_ms"] >= st["p50_ms"] > 0
    for req, got, exp in zip(reqs, mixed, expected):
        assert got["status"] == 0
        if req[0] == "min":
            np.testing.assert_array_equal(got["blocks"], exp)
            assert got["num_blocks"] == len(np.unique(exp))
        else:
            assert got["verdict"] == exp
    # each request alone on a fresh server: identical results
    with B.Server(lanes=1) as srv:
        for req, got in zip(reqs[:12], mixed[:12]):
            alone = srv.wait(_submit(srv, req))
            if req[0] == "min":
                np.testing.assert_array_equal(alone["blocks"], got["blocks"])
                assert alone["rounds"] == got["rounds"]
            else:
                assert alone["verdict"] == got["verdict"]


def test_server_round_budget_fallback_to_closure():
    """A chain request inside a group exceeds the round budget and is re-run
    alone with the closure; its result is still exact."""
    chain = W.chain_with_tail(3000, 3000, 7)
    small = [W.random_dfa(500 + i, 3, 0.3, i) for i in range(5)]
    with B.Server(lanes=1, max_group=8, batch_round_budget=16) as srv:
        tickets = [srv.submit_minimise(d) for d in small + [chain]]
        res = [srv.wait(t) for t in tickets]
    for d, r in zip(small + [chain], res):
        np.testing.assert_array_equal(r["blocks"], oracle.hopcroft(d.delta, d.accepting)[0])
    assert res[-1]["batched"] is False and all(r["batched"] for r in res[:-1])


def test_server_admission_and_errors():
    # the budget holds a lane's fixed workspace (96 MiB) and a small request,
    # not the 2^20-state, 8-letter one (with its closure about 1 GB)
    with B.Server(lanes=1, hbm_budget=256 << 20) as srv:
        too_big = W.random_dfa(1 << 20, 8, 0.5, 1)
        with pytest.raises(B.DfaError) as e:
            srv.submit_minimise(too_big)
        assert e.value.status == B.DFA_ENOMEM
        bad = W.random_dfa(50, 2, 0.5, 2)
        bad.delta[3, 0] = 99
        t = srv.submit_minimise(bad)
        assert srv.wait(t)["status"] == B.DFA_EINVAL
        good = W.random_dfa(1000, 2, 0.5, 3)
        r = srv.wait(srv.submit_minimise(good))
        np.testing.assert_array_equal(r["blocks"], oracle.hopcroft(good.delta, good.accepting)[0])
        assert srv.stats()["rejected"] == 1


def test_server_paused_resume_and_cancel():
    """A server created paused queues requests without running them.  After
    resume they run as usual; requests still queued when the server is
    destroyed are cancelled, and a thread blocked in wait on one of them
    returns DFA_ECANCELED (destroy returns only after it left)."""
    import threading
    import time

    dfas = [W.random_dfa(800 + 7 * i, 3, 0.3, 40 + i) for i in range(4)]
    with B.Server(lanes=1, paused=True) as srv:
        tickets = [srv.submit_minimise(d) for d in dfas[:2]]
        time.sleep(0.05)
        assert all(srv.poll(t) is None for t in tickets)  # nothing ran while paused
        assert srv.stats()["completed"] == 0
        srv.resume()
        for d, t in zip(dfas[:2], tickets):
            np.testing.assert_array_equal(srv.wait(t)["blocks"],
                                          oracle.hopcroft(d.delta, d.accepting)[0])
    srv = B.Server(lanes=2, paused=True)
    tickets = [srv.submit_minimise(d) for d in dfas]
    seen = {}

    def waiter(t):
        r = B.Result()
        rc = srv._lib.dfa_server_wait(srv._h, t, ctypes.byref(r))
        seen[t] = (rc, r.status, bool(r.blocks))

    threads = [threading.Thread(target=waiter, args=(t,)) for t in tickets[1:3]]
    for th in threads:
        th.start()
    deadline = time.time() + 30
    while srv.stats()["waiting_threads"] < 2:  # nothing can run while paused
        assert time.time() < deadline
        time.sleep(0.005)
    srv.close()
    for th in threads:
        th.join(timeout=60)
        assert not th.is_alive()
    for t in tickets[1:3]:
        assert seen[t] == (B.DFA_OK, B.DFA_ECANCELED, False)


@pytest.mark.parametrize("n,k", [(2 * 1024 * 1024 + 3, 5), (1 << 21, 4), ((1 << 21) - 1, 1)])
def test_host_copies_through_staging_chunks(n, k):
    """Host-pointer calls move large arrays through two page-locked 16 MiB
    chunks.  Inputs of 2.5, exactly 2 and under one chunk(s), a block array and
    quotient above the direct-copy threshold, and two back-to-back uploads
    (the operands of an equivalence) reusing the chunks: every byte arrives."""
    d = W.random_dfa(n, k, 0.3, 90 + k)
    res = B.minimise(d.delta, d.accepting, tc="off", quotient=True)
    hb, hnb = oracle.hopcroft(d.delta, d.accepting)
    np.testing.assert_array_equal(res.block, hb)
    qn, qd, qa, qs = oracle.quotient(d.delta, d.accepting, hb, d.start)
    gn, gd, ga, gs = res.quotient
    assert gn == qn == hnb and gs == qs
    np.testing.assert_array_equal(gd, qd)
    np.testing.assert_array_equal(ga, qa)
    perm, _ = W.permuted_copy(d, 91 + k)
    mut, _ = W.mutate_one(d, 92 + k)
    assert B.equivalent(d, perm, tc="off")[0]
    want = oracle.equiv_hk(d.delta, d.accepting, d.start, mut.delta, mut.accepting, mut.start)
    assert B.equivalent(d, mut, tc="off")[0] == want
    assert B.included(d, perm)[0]
