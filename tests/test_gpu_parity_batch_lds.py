"""GPU parity of the batched calls' one-workgroup path: DFAs (and equivalence
pairs) of at most `batch_lds_states` states are refined whole inside one
workgroup with their ids and grouping table in LDS; the rest go through the
segmented refinement.  Partitions, block counts and round counts are compared
with the oracle's Moore rounds, verdicts with union-find Hopcroft-Karp, for
several cut-offs (all segmented, mixed, all in LDS) on the same inputs.
"""
import numpy as np
import pytest

import oracle
from paper_2508_20735_amd import binding as B
from paper_2508_20735_amd import workloads as W

pytestmark = pytest.mark.gpu

CUTOFFS = [0, 64, 1024, 16384]


@pytest.fixture
def cutoff_restore():
    before = B.get_tuning()
    yield
    B.set_tuning(**before)


def _edge_dfas():
    rng = np.random.default_rng(77)
    out = [
        W.DFA(np.zeros((1, 1), np.uint32), np.ones(1, np.uint8), 0),   # one accepting state
        W.DFA(np.zeros((1, 4), np.uint32), np.zeros(1, np.uint8), 0),  # one rejecting state
        W.random_dfa(300, 3, 1.0, 5),    # F = Q
        W.random_dfa(300, 3, 0.0, 6),    # F empty
        W.random_dfa(2000, 16, 0.3, 7),  # 16 letters: the largest alphabet of the LDS path
        W.random_dfa(900, 17, 0.3, 8),   # 17 letters: always segmented
        W.fibonacci(11),                 # 144 states, 143 rounds
        W.bitsplitter(9),
        W.chain_with_tail(700, 300, 9),
    ]
    for n in (63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 4095, 4096, 4097, 8191, 16384):
        k = int(rng.integers(1, 9))
        d = W.random_dfa(n, k, float(rng.uniform(0.05, 0.6)), int(rng.integers(1 << 30)))
        if n % 2:  # duplicated rows: blocks with several members
            src = rng.integers(0, n, n // 2)
            dst = rng.integers(0, n, n // 2)
            d.delta[dst] = d.delta[src]
            d.accepting[dst] = d.accepting[src]
        out.append(d)
    return out


@pytest.mark.parametrize("cut", CUTOFFS)
def test_minimise_batch_every_cutoff(cut, cutoff_restore):
    B.set_tuning(batch_lds_states=cut)
    dfas = _edge_dfas()
    print(f"minimise batch, cut-off {cut}: {len(dfas)} DFAs", flush=True)
    blocks, nb, rounds, st = B.minimise_batch(dfas)
    for i, d in enumerate(dfas):
        ref, rnb, rrounds, _ = oracle.moore(d.delta, d.accepting)
        np.testing.assert_array_equal(blocks[i], ref, err_msg=f"dfa {i} n={d.n} k={d.k}")
        assert (nb[i], rounds[i]) == (rnb, rrounds), (i, d.n, d.k)
    assert st["rounds"] == max(rounds)


@pytest.mark.parametrize("cut", CUTOFFS)
def test_equivalent_batch_every_cutoff(cut, cutoff_restore):
    B.set_tuning(batch_lds_states=cut)
    rng = np.random.default_rng(31)
    pairs = []
    for i, d in enumerate(_edge_dfas()):
        if i % 3 == 0:
            other, _ = W.permuted_copy(d, i)
        elif i % 3 == 1 and d.n > 1:
            other, _ = W.mutate_one(d, i)
        else:
            other = W.random_dfa(int(rng.integers(1, 50)), d.k, 0.5, 700 + i)
        pairs.append((d, other))
    print(f"equivalence batch, cut-off {cut}: {len(pairs)} pairs", flush=True)
    verdicts, st = B.equivalent_batch(pairs)
    for (a, b), v in zip(pairs, verdicts):
        assert v == oracle.equiv_hk(a.delta, a.accepting, a.start, b.delta, b.accepting, b.start)


def test_batch_workload_slice_all_in_lds(cutoff_restore):
    """The first 512 DFAs of the 4,096-DFA workload with the largest cut-off
    (DFAs up to 16,384 states, pairs up to 16,384 states together, in LDS)."""
    B.set_tuning(batch_lds_states=16384)
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


def test_small_path_bad_target_and_recovery(cutoff_restore):
    B.set_tuning(batch_lds_states=4096)
    good = W.random_dfa(200, 3, 0.4, 1)
    bad = W.random_dfa(100, 3, 0.4, 2)
    bad.delta[17, 2] = 100  # one past the last state
    with pytest.raises(B.DfaError) as e:
        B.minimise_batch([good, bad])
    assert e.value.status == B.DFA_EINVAL
    with pytest.raises(B.DfaError) as e:
        B.equivalent_batch([(good, bad)])
    assert e.value.status == B.DFA_EINVAL
    blocks, nb, rounds, _ = B.minimise_batch([good])
    np.testing.assert_array_equal(blocks[0], oracle.hopcroft(good.delta, good.accepting)[0])


def test_tuning_range(cutoff_restore):
    with pytest.raises(B.DfaError) as e:
        B.set_tuning(batch_lds_states=16385)
    assert e.value.status == B.DFA_EINVAL
    assert B.default_tuning()["batch_lds_states"] == 4096


def test_autotuned_batch_parity(tmp_path, cutoff_restore):
    """The autotuner on a 300-DFA slice of the batch workload (a small search
    space, one timed run per candidate): it caches the fastest tuning for the
    device and shape, and the batch under that tuning equals the oracle."""
    import torch

    from paper_2508_20735_amd import autotune as T

    items = W.batch_workload(count=300, paired_from=300)
    dfas = [it.dfa for it in items]
    dev = torch.device("cuda:0")
    deltas = [torch.from_numpy(d.delta.view(np.int32)).to(dev) for d in dfas]
    accs = [torch.from_numpy(d.accepting).to(dev) for d in dfas]
    path = str(tmp_path / "tuning.json")
    space = {"batch_lds_states": [0, 2048, 8192], "chunk": [4, 8]}
    res = T.autotune_batch(deltas, accs, space=space, reps=1, path=path)
    shape = T.batch_shape([d.n for d in dfas], [d.k for d in dfas], "minimise")
    assert list(res) == [shape]
    best = T.lookup(shape, path)
    assert best is not None and best["batch_lds_states"] in (0, 2048, 4096, 8192)
    B.set_tuning(**B.default_tuning())
    out = torch.empty(sum(d.n for d in dfas), dtype=torch.int32, device=dev)
    with T.tuned(shape, path):
        assert B.get_tuning() == best
        nb, rounds, _ = B.minimise_batch_device(deltas, accs, out)
    assert B.get_tuning() == B.default_tuning()
    got = out.cpu().numpy().view(np.uint32)
    pos = 0
    for i, d in enumerate(dfas):
        ref, rnb, rrounds, _ = oracle.moore(d.delta, d.accepting)
        np.testing.assert_array_equal(got[pos:pos + d.n], ref, err_msg=f"dfa {i}")
        assert (nb[i], rounds[i]) == (rnb, rrounds), i
        pos += d.n


def test_packed_batch_matches_tensor_lists(cutoff_restore):
    """PackedBatch (two flat tensors per operand list, views computed in bulk)
    gives the same blocks, counts, rounds and verdicts as lists of tensors,
    and both equal the oracle."""
    import torch

    B.set_tuning(batch_lds_states=1024)
    dfas = _edge_dfas()
    others = [W.permuted_copy(d, i)[0] if i % 2 == 0 or d.n < 2 else W.mutate_one(d, i)[0]
              for i, d in enumerate(dfas)]
    dev = torch.device("cuda:0")

    def t(d):
        return (torch.from_numpy(np.ascontiguousarray(d.delta).view(np.int32)).to(dev),
                torch.from_numpy(d.accepting).to(dev), d.start)

    lists = [t(d) for d in dfas]
    total = sum(d.n for d in dfas)
    out_a = torch.empty(total, dtype=torch.int32, device=dev)
    out_b = torch.empty(total, dtype=torch.int32, device=dev)
    nb_a, r_a, _ = B.minimise_batch_device([x[0] for x in lists], [x[1] for x in lists], out_a)
    pack = B.PackedBatch.from_dfas(dfas)
    assert pack.count == len(dfas) and pack.states == total
    nb_b, r_b, _ = B.minimise_batch_device(pack, None, out_b)
    assert torch.equal(out_a, out_b)
    np.testing.assert_array_equal(nb_a, nb_b)
    np.testing.assert_array_equal(r_a, r_b)
    got = out_b.cpu().numpy()
    off = 0
    for i, d in enumerate(dfas):
        ref, rnb, rrounds, _ = oracle.moore(d.delta, d.accepting)
        np.testing.assert_array_equal(got[off:off + d.n], ref, err_msg=f"dfa {i}")
        assert (nb_b[i], r_b[i]) == (rnb, rrounds)
        off += d.n
    v_lists, _ = B.equivalent_batch_device(lists, [t(o) for o in others])
    v_pack, _ = B.equivalent_batch_device(pack, B.PackedBatch.from_dfas(others))
    np.testing.assert_array_equal(v_lists, v_pack)
    for (a, b), v in zip(zip(dfas, others), v_pack):
        assert v == oracle.equiv_hk(a.delta, a.accepting, a.start, b.delta, b.accepting, b.start)
    with pytest.raises(ValueError):
        B.equivalent_batch_device(pack, lists)
