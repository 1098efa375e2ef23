"""GPU parity of the persistent round loop (the refinement loop of Algorithms 2
and 4, Section 3, run on the device inside one cooperative launch, its phases
separated by grid barriers) against the CPU oracle.

The persistent loop runs the same phases as the per-kernel loops, so
partitions, rounds and separating rounds match the oracle exactly: Moore
rounds for signature refinement, naivePR rounds for leader refinement.
"""
import numpy as np
import pytest

import oracle
from paper_2508_20735_amd import binding as B
from paper_2508_20735_amd import workloads as W

pytestmark = pytest.mark.gpu

SIZES = [
    (1, 1, 0.5, 1), (2, 1, 0.5, 2), (3, 2, 0.5, 3), (63, 2, 0.3, 4), (64, 3, 0.5, 5),
    (257, 5, 0.5, 9), (4097, 8, 0.4, 11), (12345, 9, 0.3, 12), (5000, 17, 0.5, 13),
    (20000, 16, 0.3, 21), (3000, 15, 0.4, 22),
    (70000, 4, 0.2, 15), (300000, 2, 0.5, 16),
]


def check(d, algorithm="signature", tc="off", quotient=False, chunk=0):
    res = B.minimise(d.delta, d.accepting, tc=tc, loop="persistent", start=d.start,
                     quotient=quotient, algorithm=algorithm, chunk=chunk)
    if algorithm == "leader":
        ref = (oracle.naive_pr_tc(d.delta, d.accepting) if tc == "on"
               else oracle.naive_pr(d.delta, d.accepting))
    else:
        ref = oracle.moore(d.delta, d.accepting)
    block, nb, rounds, changing = ref
    if tc == "auto" or (tc == "on" and algorithm != "leader"):
        block, nb = oracle.hopcroft(d.delta, d.accepting)
    np.testing.assert_array_equal(res.block, block)
    assert res.stats["num_blocks"] == nb
    if tc == "off" or (tc == "on" and algorithm == "leader"):
        assert (res.stats["rounds"], res.stats["changing_rounds"]) == (rounds, changing)
    if quotient:
        qn, qd, qa, qs = oracle.quotient(d.delta, d.accepting, block, d.start)
        gn, gd, ga, gs = res.quotient
        assert gn == qn and gs == qs
        np.testing.assert_array_equal(gd, qd)
        np.testing.assert_array_equal(ga, qa)
    return res


@pytest.mark.parametrize("n,k,p,seed", SIZES)
def test_persistent_signature_random(n, k, p, seed):
    check(W.random_dfa(n, k, p, seed), quotient=True)


@pytest.mark.parametrize("n,k,p,seed", SIZES[:9])
def test_persistent_leader_random(n, k, p, seed):
    check(W.random_dfa(n, k, p, seed), algorithm="leader", quotient=True)


def test_persistent_shared_rows():
    """Large blocks with equal rows: LDS-staged and direct grouping, holder
    compares in the incremental rounds."""
    d = W.random_dfa(60000, 3, 0.3, 99)
    rng = np.random.default_rng(5)
    src = rng.integers(0, 50, 55000)
    dst = rng.integers(50, d.n, 55000)
    d.delta[dst] = d.delta[src]
    d.accepting[dst] = d.accepting[src]
    for lds in (0, 1, 2):
        res = B.minimise(d.delta, d.accepting, tc="off", loop="persistent", lds_stage=lds)
        block, nb, rounds, changing = oracle.moore(d.delta, d.accepting)
        np.testing.assert_array_equal(res.block, block)
        assert (res.stats["rounds"], res.stats["changing_rounds"]) == (rounds, changing)


@pytest.mark.parametrize("algorithm", ["signature", "leader"])
def test_persistent_families(algorithm):
    check(W.fibonacci(12), algorithm=algorithm, tc="off")
    check(W.fibonacci(12), algorithm=algorithm, tc="on")
    check(W.bitsplitter(10), algorithm=algorithm, tc="off")
    check(W.chain_with_tail(1 << 10, 1 << 10, 7), algorithm=algorithm, tc="auto")


@pytest.mark.parametrize("chunk", [1, 7, 4096])
def test_persistent_chunk_lengths(chunk):
    """One launch may hold more rounds than the refinement needs (it stops
    on the device) or fewer (the host launches again)."""
    check(W.fibonacci(13), tc="off", chunk=chunk)
    check(W.fibonacci(13), algorithm="leader", tc="off", chunk=chunk)


def test_persistent_table2_fib18():
    """Table 2 row Fib_18: 6,765 states, all distinct, 6,764 naivePR
    iterations, in one device-side loop."""
    res = check(W.fibonacci(19), algorithm="leader", chunk=8192)
    assert res.stats["rounds"] == 6764 and res.stats["num_blocks"] == 6765


@pytest.mark.parametrize("algorithm", ["signature", "leader"])
def test_persistent_max_rounds(algorithm):
    d = W.fibonacci(12)  # 233 states, 231 refining rounds
    with pytest.raises(B.DfaError) as e:
        B.minimise(d.delta, d.accepting, tc="off", loop="persistent", max_rounds=10,
                   algorithm=algorithm)
    assert e.value.status == B.DFA_ELIMIT


@pytest.mark.parametrize("algorithm", ["signature", "leader"])
def test_persistent_equivalence(algorithm):
    a = W.random_dfa(20000, 4, 0.1, 31)
    perm, _ = W.permuted_copy(a, 32)
    mut, _ = W.mutate_one(a, 33)
    for other in (perm, mut):
        expect = oracle.equiv_hk(a.delta, a.accepting, a.start, other.delta, other.accepting,
                                 other.start)
        for tc in ("off", "auto"):
            got, _ = B.equivalent(a, other, tc=tc, loop="persistent", algorithm=algorithm)
            assert got == expect, (tc, other is perm)


def test_persistent_large_config():
    """The 2^22-state, 4-letter workload (seed 2): the same partition as
    Hopcroft and Moore's round count, with the loop on the device."""
    d = W.cfg_large()
    res = B.minimise(d.delta, d.accepting, tc="off", loop="persistent")
    hb, hnb = oracle.hopcroft(d.delta, d.accepting)
    np.testing.assert_array_equal(res.block, hb)
    assert res.stats["num_blocks"] == hnb


def test_persistent_pruned():
    d = W.random_dfa(20000, 3, 0.3, 61)
    res = B.minimise(d.delta, d.accepting, tc="off", loop="persistent", prune=True, start=3)
    block, nb, nr = oracle.minimise_reachable(d.delta, d.accepting, 3)
    np.testing.assert_array_equal(res.block, block)
    assert res.stats["reachable"] == nr


@pytest.mark.parametrize("cut", [0, 4096])
def test_persistent_batches(cut):
    """Batched calls in the persistent loop: the segmented rounds with their
    per-segment bookkeeping inside the cooperative launch (cut-off 0: every
    DFA segmented; 4096: the small ones in one workgroup each), against the
    oracle's partitions and Moore rounds and Hopcroft-Karp verdicts."""
    before = B.get_tuning()
    try:
        B.set_tuning(batch_lds_states=cut)
        rng = np.random.default_rng(41)
        dfas = [W.random_dfa(int(rng.integers(1, 20000)), int(rng.integers(1, 9)),
                             float(rng.uniform(0.05, 0.6)), 300 + i) for i in range(40)]
        dfas += [W.fibonacci(12), W.bitsplitter(8), W.chain_with_tail(500, 200, 4)]
        print(f"persistent batch, cut-off {cut}: {len(dfas)} DFAs", flush=True)
        for chunk in (0, 3):
            blocks, nb, rounds, st = B.minimise_batch(dfas, tc="off", loop="persistent",
                                                      chunk=chunk)
            for i, d in enumerate(dfas):
                ref, rnb, rrounds, _ = oracle.moore(d.delta, d.accepting)
                np.testing.assert_array_equal(blocks[i], ref, err_msg=f"dfa {i}")
                assert (nb[i], rounds[i]) == (rnb, rrounds), (i, d.n, d.k)
        pairs = []
        for i, d in enumerate(dfas):
            other = (W.permuted_copy(d, i)[0] if i % 2 == 0 or d.n < 2
                     else W.mutate_one(d, i)[0])
            pairs.append((d, other))
        verdicts, _ = B.equivalent_batch(pairs, tc="off", loop="persistent")
        for (a, b), v in zip(pairs, verdicts):
            assert v == oracle.equiv_hk(a.delta, a.accepting, a.start, b.delta, b.accepting,
                                        b.start)
    finally:
        B.set_tuning(**before)
