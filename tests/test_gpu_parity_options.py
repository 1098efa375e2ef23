"""GPU parity of every option combination on tiny and degenerate DFAs (one
state, all states accepting or rejecting, identity letters, a self-loop
chain): algorithm x closure mode x loop mode x pruning, each against the
oracle (Hopcroft's partition, or the reachable part's with pruning).
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2508_20735_amd import binding as B
from paper_2508_20735_amd import workloads as W

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(2024)
    out = []
    for n, k in ((1, 1), (1, 3), (2, 1), (2, 3), (5, 2), (40, 3)):
        delta = rng.integers(0, n, (n, k)).astype(np.uint32)
        for acc_kind in ("random", "all", "none"):
            acc = {"random": rng.integers(0, 2, n), "all": np.ones(n),
                   "none": np.zeros(n)}[acc_kind].astype(np.uint8)
            out.append((f"n{n}k{k}{acc_kind}", W.DFA(delta.copy(), acc, 0)))
    # identity letters next to a moving one, and a chain
    ident = np.tile(np.arange(7, dtype=np.uint32)[:, None], (1, 3))
    ident[:, 1] = (np.arange(7) + 1) % 7
    out.append(("ident", W.DFA(ident, np.array([1, 0, 0, 1, 0, 0, 0], dtype=np.uint8), 2)))
    out.append(("chain", W.chain_with_tail(33, 17, 9)))
    return out


CASES = _cases()


@pytest.mark.parametrize("name,d", CASES, ids=[c[0] for c in CASES])
def test_every_option_combination(name, d):
    hb, hnb = oracle.hopcroft(d.delta, d.accepting)
    rb, rnb, rn = oracle.minimise_reachable(d.delta, d.accepting, d.start)
    for alg, tc, loop, prune in itertools.product(("signature", "sort", "leader"),
                                                  ("off", "on", "auto"),
                                                  ("host", "chunk", "graph", "persistent"),
                                                  (False, True)):
        if loop == "persistent" and alg == "sort":
            continue  # rejected (EINVAL), checked in the ABI tests
        res = B.minimise(d.delta, d.accepting, tc=tc, loop=loop, algorithm=alg, prune=prune,
                         start=d.start, quotient=True)
        want, wnb = (rb, rnb) if prune else (hb, hnb)
        np.testing.assert_array_equal(res.block, want, err_msg=f"{alg} {tc} {loop} {prune}")
        assert res.stats["num_blocks"] == wnb, (alg, tc, loop, prune)
        gn, gd, ga, gs = res.quotient
        assert gn == wnb
        # the quotient is minimal and equivalent to the input from its start
        assert oracle.hopcroft(gd, ga)[1] == gn
        assert oracle.equiv_hk(d.delta, d.accepting, d.start, gd, ga, gs)


def _pairs():
    by_k = {}
    for name, d in CASES:
        by_k.setdefault(d.k, []).append((name, d))
    out = []
    for k, group in sorted(by_k.items()):
        for (na, a), (nb, b) in itertools.product(group, group):
            out.append((f"{na}-{nb}", a, b))
    return out


PAIRS = _pairs()


@pytest.mark.parametrize("k", sorted({d.k for _, d in CASES}))
def test_equivalence_and_inclusion_every_method(k):
    """Equivalence (union refinement under each algorithm, closure and loop
    mode, and the product search) and inclusion in both directions, on every
    ordered pair of the cases above over the same alphabet."""
    for name, a, b in (p for p in PAIRS if p[1].k == k):
        want = oracle.equiv_hk(a.delta, a.accepting, a.start, b.delta, b.accepting, b.start)
        for alg, tc, loop in itertools.product(("signature", "sort", "leader"),
                                               ("off", "auto"), ("host", "graph", "persistent")):
            if loop == "persistent" and alg == "sort":
                continue
            got, _ = B.equivalent(a, b, tc=tc, loop=loop, algorithm=alg)
            assert got == want, (name, alg, tc, loop)
        got, st = B.equivalent(a, b, method="product")
        assert got == want, (name, "product")
        for x, y in ((a, b), (b, a)):
            inc = oracle.included(x.delta, x.accepting, x.start, y.delta, y.accepting, y.start)
            got, pairs, _ = B.included(x, y)
            assert got == inc, (name, "included")
            assert pairs >= 1


@pytest.mark.parametrize("k", [33, 64, 130])
def test_large_alphabets(k):
    """Alphabets above the specialised signature widths (the generic path)
    and closures of more than 64 columns (k * (floor(log2 n) + 1) up to
    1,560): every algorithm and closure mode gives Hopcroft's partition;
    Moore's round count without the closure.  Some letters are the identity
    and some repeat another letter, so column dropping has work to do."""
    # 60 copies of a 50-state chain (letter a steps 0, 1 or 2 states towards
    # the one accepting state), each transition going to a random copy of
    # its target: blocks of 60 states, separated over about 25 rounds
    rng = np.random.default_rng(k)
    step = rng.integers(0, 3, k)
    step[0], step[1], step[k - 1] = 1, 0, 1
    i = np.arange(50)
    chain = np.minimum(i[:, None] + step[None, :], 49)
    q = np.arange(3000)
    delta = (chain[q % 50] + 50 * rng.integers(0, 60, (3000, k))).astype(np.uint32)
    delta[:, 1] = q
    delta[:, k - 1] = delta[:, 0]
    d = W.DFA(delta, (q % 50 == 49).astype(np.uint8), 0)
    hb, hnb = oracle.hopcroft(d.delta, d.accepting)
    mb, mnb, mrounds, mchanging = oracle.moore(d.delta, d.accepting)
    for alg, tc in itertools.product(("signature", "sort", "leader"), ("off", "auto", "on")):
        res = B.minimise(d.delta, d.accepting, tc=tc, algorithm=alg, quotient=True)
        np.testing.assert_array_equal(res.block, hb, err_msg=f"{alg} {tc}")
        assert res.stats["num_blocks"] == hnb
        if tc == "off" and alg != "leader":
            assert (res.stats["rounds"], res.stats["changing_rounds"]) == (mrounds, mchanging)
        gn, gd, ga, gs = res.quotient
        assert gn == hnb and oracle.hopcroft(gd, ga)[1] == gn
    # a larger instance through the segmented batch path as well
    big = W.random_dfa(100000, 40, 0.2, 800)
    hb2, _ = oracle.hopcroft(big.delta, big.accepting)
    np.testing.assert_array_equal(B.minimise(big.delta, big.accepting, tc="off").block, hb2)
    blocks, _, _, _ = B.minimise_batch([d, big], tc="off")
    np.testing.assert_array_equal(blocks[0], hb)
    np.testing.assert_array_equal(blocks[1], hb2)


@pytest.mark.parametrize("n,k", [(2047, 2), (6139, 4), (130972, 3), (2 * 1024 * 1024 + 3, 4)])
def test_xcd_sliced_tiles(n, k):
    """Grids that are multiples of 8 give each XCD a contiguous share of the
    tiles (ragged shares and a ragged last tile here; the label rounds' grid
    is capped at 2,048 and the round kernels' at 8,192), others stride over
    all tiles: Moore's partition and round count, and the equivalence
    verdicts on unions of twice the size, both label rounds included."""
    d = W.random_dfa(n, k, 0.3, 31 + k)
    res = B.minimise(d.delta, d.accepting, tc="off")
    block, nb, rounds, changing = oracle.moore(d.delta, d.accepting)
    np.testing.assert_array_equal(res.block, block)
    assert (res.stats["num_blocks"], res.stats["rounds"], res.stats["changing_rounds"]) == \
        (nb, rounds, changing)
    perm, _ = W.permuted_copy(d, 32 + k)
    mut, _ = W.mutate_one(d, 33 + k)
    assert B.equivalent(d, perm, tc="off")[0]
    want = oracle.equiv_hk(d.delta, d.accepting, d.start, mut.delta, mut.accepting, mut.start)
    assert B.equivalent(d, mut, tc="off")[0] == want
