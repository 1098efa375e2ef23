"""GPU parity of round 0 of segmented (batched) refinements by acceptance
patterns: each state's key is its segment and the acceptance of itself and
its successors, grouped through a segment x pattern table instead of the hash
table.  Batches are refined with it (label_rounds >= 1) and without it
(label_rounds 0, a table round), all through the segmented path (no DFA in
the one-workgroup path), and compared with the oracle's Moore rounds
(partitions, block counts, round counts) and union-find Hopcroft-Karp.
Covered: tiles that span many segments (keys beyond the LDS share go to the
table directly), alphabets of 1 to 15 letters (the widest pattern, 16 bits),
more segments than the table holds for the width (then round 0 is a table
round), identity padding of mixed alphabets, F empty / F = Q, one-state DFAs.
"""
import numpy as np
import pytest

import oracle
from paper_2508_20735_amd import binding as B
from paper_2508_20735_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture
def tuning_restore():
    before = B.get_tuning()
    yield
    B.set_tuning(**before)


def _mixed(count, kmax, seed, nmax=3000):
    rng = np.random.default_rng(seed)
    out = [W.DFA(np.zeros((1, 1), np.uint32), np.ones(1, np.uint8), 0),
           W.random_dfa(40, 2, 1.0, seed + 1), W.random_dfa(40, 2, 0.0, seed + 2)]
    for i in range(count):
        n = int(np.exp(rng.uniform(0, np.log(nmax))))
        k = int(rng.integers(1, kmax + 1))
        d = W.random_dfa(max(n, 1), k, float(rng.uniform(0.05, 0.6)), int(rng.integers(1 << 30)))
        if i % 3 == 0 and d.n > 2:  # duplicated rows: blocks with several members
            src = rng.integers(0, d.n, d.n // 2)
            dst = rng.integers(0, d.n, d.n // 2)
            d.delta[dst] = d.delta[src]
            d.accepting[dst] = d.accepting[src]
        out.append(d)
    return out


def _check_minimise(dfas, label_rounds):
    B.set_tuning(batch_lds_states=0, label_rounds=label_rounds)
    B.profile_only(None)
    B.profile_enable(True)
    blocks, nb, rounds, st = B.minimise_batch(dfas)
    kt = B.profile_read()
    B.profile_enable(False)
    for i, d in enumerate(dfas):
        ref, rnb, rrounds, _ = oracle.moore(d.delta, d.accepting)
        np.testing.assert_array_equal(blocks[i], ref, err_msg=f"dfa {i} n={d.n} k={d.k}")
        assert (nb[i], rounds[i]) == (rnb, rrounds), (i, d.n, d.k)
    return kt


@pytest.mark.parametrize("label_rounds", [0, 2])
@pytest.mark.parametrize("kmax,count,seed", [(4, 300, 1), (8, 120, 2), (15, 12, 3)])
def test_minimise_batch_round0_by_patterns(kmax, count, seed, label_rounds, tuning_restore):
    dfas = _mixed(count, kmax, seed)
    print(f"segmented minimise: {len(dfas)} DFAs, k <= {kmax}, label_rounds {label_rounds}",
          flush=True)
    kt = _check_minimise(dfas, label_rounds)
    assert ("k_seg_pattern" in kt) == (label_rounds > 0)


def test_too_many_segments_for_the_width(tuning_restore):
    """300 DFAs with 15 letters: 300 << 16 keys exceed the table, so round 0
    is a table round even with label rounds on."""
    dfas = [W.random_dfa(30, 15, 0.3, 100 + i) for i in range(300)]
    kt = _check_minimise(dfas, 2)
    assert "k_seg_pattern" not in kt


def test_tiny_dfas_many_segments_per_tile(tuning_restore):
    """2,000 DFAs of 1 to 12 states with 8 letters: a workgroup's tile spans
    hundreds of segments, most of whose keys go to the table directly."""
    rng = np.random.default_rng(9)
    dfas = [W.random_dfa(int(rng.integers(1, 13)), 8, 0.4, 1000 + i) for i in range(2000)]
    kt = _check_minimise(dfas, 2)
    assert "k_seg_pattern" in kt


@pytest.mark.parametrize("label_rounds", [0, 2])
def test_equivalence_batch_round0_by_patterns(label_rounds, tuning_restore):
    B.set_tuning(batch_lds_states=0, label_rounds=label_rounds)
    rng = np.random.default_rng(17)
    pairs = []
    for i, d in enumerate(_mixed(150, 6, 17)):
        if i % 3 == 0:
            other, _ = W.permuted_copy(d, i)
        elif i % 3 == 1 and d.n > 1:
            other, _ = W.mutate_one(d, i)
        else:
            other = W.random_dfa(int(rng.integers(1, 60)), d.k, 0.5, 500 + i)
        pairs.append((d, other))
    print(f"segmented equivalence: {len(pairs)} pairs, label_rounds {label_rounds}", flush=True)
    verdicts, st = B.equivalent_batch(pairs)
    for (a, b), v in zip(pairs, verdicts):
        assert v == oracle.equiv_hk(a.delta, a.accepting, a.start, b.delta, b.accepting, b.start)


def test_batch_workload_slice_segmented(tuning_restore):
    """512 DFAs of the 4,096-DFA workload, all segmented (cut-off 0), with the
    pattern round: partitions and rounds against the oracle; verdicts of the
    256 pairs."""
    B.set_tuning(batch_lds_states=0, label_rounds=2)
    items = W.batch_workload(count=512, paired_from=256)
    dfas = [it.dfa for it in items]
    blocks, nb, rounds, _ = B.minimise_batch(dfas)
    for i, d in enumerate(dfas):
        ref, rnb, rrounds, _ = oracle.moore(d.delta, d.accepting)
        np.testing.assert_array_equal(blocks[i], ref, err_msg=f"dfa {i}")
        assert (nb[i], rounds[i]) == (rnb, rrounds), i
    pairs = [(it.dfa, it.pair) for it in items if it.pair is not None]
    verdicts, _ = B.equivalent_batch(pairs)
    for (a, b), v in zip(pairs, verdicts):
        assert v == oracle.equiv_hk(a.delta, a.accepting, a.start, b.delta, b.accepting, b.start)
