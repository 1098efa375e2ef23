"""GPU parity of the dense rounds that gather successor ids through LDS
slices (edges bucketed by target slice once per refinement): the same DFAs
with the slices on (slice_min_states small enough) and off, against the
oracle's Moore rounds, for several alphabet widths, sizes with a ragged last
slice and source tile, every loop driver, sort grouping, and the unions of
equivalence checks.  Integer work: every comparison is exact.
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


def _run(d, slices, **kw):
    B.set_tuning(slice_min_states=slices)
    return B.minimise(d.delta, d.accepting, quotient=True, **kw)


@pytest.mark.parametrize("n,k,p,seed", [
    ((1 << 15) + 1, 4, 0.1, 1),       # two slices, the second with one state
    (100_003, 3, 0.3, 2),              # ragged last slice and source tile
    (70_000, 16, 0.4, 3),              # the widest bucketed alphabet
    (65_536, 1, 0.5, 4),               # one letter
    (50_000, 5, 0.2, 5), (40_000, 7, 0.2, 6), (30_000, 8, 0.5, 7),
])
def test_slices_match_oracle_and_direct(n, k, p, seed, tuning_restore):
    d = W.random_dfa(n, k, p, seed)
    print(f"slices: n={n} k={k}", flush=True)
    ref, nb, rounds, changing = oracle.moore(d.delta, d.accepting)
    on = _run(d, 1024, tc="off")
    off = _run(d, 0, tc="off")
    for res in (on, off):
        np.testing.assert_array_equal(res.block, ref)
        assert res.stats["num_blocks"] == nb
        assert res.stats["rounds"] == rounds and res.stats["changing_rounds"] == changing
    qn, qd, qa, qs = oracle.quotient(d.delta, d.accepting, ref, d.start)
    gn, gd, ga, gs = on.quotient
    assert gn == qn and gs == qs
    np.testing.assert_array_equal(gd, qd)
    np.testing.assert_array_equal(ga, qa)


@pytest.mark.parametrize("loop", ["host", "chunk", "graph"])
@pytest.mark.parametrize("algorithm", ["signature", "sort"])
def test_slices_loops_and_sort_grouping(loop, algorithm, tuning_restore):
    # duplicated rows: blocks with several members, so the first selective
    # round after the first table round is dense too
    d = W.random_dfa(120_000, 4, 0.3, 11)
    rng = np.random.default_rng(12)
    src = rng.integers(0, d.n, d.n // 2)
    dst = rng.integers(0, d.n, d.n // 2)
    d.delta[dst] = d.delta[src]
    d.accepting[dst] = d.accepting[src]
    print(f"slices: loop={loop} algorithm={algorithm}", flush=True)
    ref, nb, rounds, changing = oracle.moore(d.delta, d.accepting)
    res = _run(d, 1024, tc="off", loop=loop, algorithm=algorithm)
    np.testing.assert_array_equal(res.block, ref)
    assert res.stats["rounds"] == rounds and res.stats["changing_rounds"] == changing


def test_slices_on_unions(tuning_restore):
    """Equivalence with a permuted copy (every state has a twin: the first
    two table rounds are dense) and with a one-transition mutation."""
    B.set_tuning(slice_min_states=1024)
    d = W.random_dfa(90_000, 4, 0.1, 21)
    perm, _ = W.permuted_copy(d, 22)
    mut, _ = W.mutate_one(d, 23)
    assert B.equivalent(d, perm, tc="off")[0]
    want = oracle.equiv_hk(d.delta, d.accepting, d.start, mut.delta, mut.accepting, mut.start)
    assert B.equivalent(d, mut, tc="off")[0] == want
    # the unions' partitions themselves, through their minimisation: with the
    # mutated copy, separations spread back from the mutation over many
    # incremental rounds after the dense ones
    for other in (perm, mut):
        ud, ua = oracle.union(d.delta, d.accepting, other.delta, other.accepting)
        ref, nb, rounds, changing = oracle.moore(ud, ua)
        for loop in ("chunk", "graph", "host"):
            res = B.minimise(ud, ua, tc="off", loop=loop)
            np.testing.assert_array_equal(res.block, ref)
            assert res.stats["rounds"] == rounds and res.stats["changing_rounds"] == changing


def test_slices_kernel_timing_charges_one_path(tuning_restore):
    """With kernel timing on, the rounds that gathered through slices charge
    their bytes to the two passes and the others to the signature kernel:
    the refined states of the two paths add up to the grouping kernel's."""
    B.set_tuning(slice_min_states=1024)
    d = W.random_dfa(200_000, 4, 0.1, 31)
    perm, _ = W.permuted_copy(d, 32)
    B.profile_only(None)
    B.profile_enable(True)
    B.equivalent(d, perm, tc="off", loop="chunk")
    kt = B.profile_read()
    B.profile_enable(False)
    assert kt["k_pb_gather"]["states"] == kt["k_signature_pb"]["states"] > 0
    # every refined state of a table round is charged once to the signature
    # path its round took, and once to the grouping kernel
    assert kt["k_signature"]["states"] + kt["k_signature_pb"]["states"] == \
        kt["k_insert"]["states"]


@pytest.mark.parametrize("label_rounds", [0, 1, 2])
@pytest.mark.parametrize("k", [2, 4, 6])
def test_slices_with_and_without_label_rounds(label_rounds, k, tuning_restore):
    """The label rounds gather their byte labels directly (they come from a
    small, cached array) and the first table round after them through the
    slices; without label rounds, round 0 is a table round over the initial
    labels and gathers through the slices."""
    B.set_tuning(label_rounds=label_rounds)
    d = W.random_dfa(80_021, k, 0.25, 40 + k)
    print(f"slices: label_rounds={label_rounds} k={k}", flush=True)
    ref, nb, rounds, changing = oracle.moore(d.delta, d.accepting)
    for slices in (1024, 0):
        res = _run(d, slices, tc="off")
        np.testing.assert_array_equal(res.block, ref)
        assert res.stats["rounds"] == rounds and res.stats["changing_rounds"] == changing
