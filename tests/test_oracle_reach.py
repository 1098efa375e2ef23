"""Pins of the oracle's reachability and reachable-part minimisation.

The paper partitions every state and assumes all of them reachable (Section
2); the usual minimal DFA is the quotient of the part reachable from the
start.  The oracle's breadth-first search is checked against word enumeration
(the definition: q is reachable iff some word leads from the start to q) and
closed forms; the reachable minimisation against the full minimisation and
language equivalence.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2508_20735_amd import workloads as W


def reachable_by_words(delta, start):
    """States reached by some word of length <= n - 1 (a shortest path never
    repeats a state), by enumerating the words."""
    n, k = delta.shape
    seen = {start}
    for length in range(1, n):
        for w in itertools.product(range(k), repeat=length):
            q = start
            for a in w:
                q = int(delta[q, a])
            seen.add(q)
    return seen


def test_reachable_matches_word_enumeration():
    rng = np.random.default_rng(3)
    for _ in range(300):
        n = int(rng.integers(1, 6))
        k = int(rng.integers(1, 3))
        delta = rng.integers(0, n, size=(n, k), dtype=np.uint32)
        start = int(rng.integers(0, n))
        mask = oracle.reachable(delta, start)
        assert set(np.flatnonzero(mask).tolist()) == reachable_by_words(delta, start)


def test_reachable_closed_forms():
    # the chain part of the chain-with-tail workload is reached from 0, the
    # tail (targets inside the tail) is not
    d = W.chain_with_tail(256, 300, 5)
    mask = oracle.reachable(d.delta, 0)
    assert mask[:256].all() and not mask[256:].any()
    # Fibonacci DFAs: a path through every state from the start
    f = W.fibonacci(9)
    assert oracle.reachable(f.delta, f.start).all()
    # a DFA whose every letter is the identity reaches only its start
    ident = np.tile(np.arange(7, dtype=np.uint32)[:, None], (1, 3))
    assert np.flatnonzero(oracle.reachable(ident, 4)).tolist() == [4]


@pytest.mark.parametrize("seed", range(6))
def test_minimise_reachable_against_full_minimisation(seed):
    """On reachable states the reachable minimisation is the full one, except
    that a block's id is its smallest reachable member; unreachable states
    carry no block."""
    d = W.random_dfa(2000, 2 + seed % 3, 0.4, 40 + seed)
    start = seed * 7
    block, nb, nr = oracle.minimise_reachable(d.delta, d.accepting, start)
    mask = oracle.reachable(d.delta, start)
    assert nr == mask.sum()
    assert (block[~mask] == oracle.UNREACHABLE).all()
    full, _ = oracle.hopcroft(d.delta, d.accepting)
    r = np.flatnonzero(mask)
    # same relation on the reachable states
    np.testing.assert_array_equal(full[r][:, None] == full[r][None, :],
                                  block[r][:, None] == block[r][None, :])
    # ids: smallest reachable member
    for b in np.unique(block[r]):
        members = r[block[r] == b]
        assert b == members.min()
    assert nb == len(np.unique(block[r]))


@pytest.mark.parametrize("seed", range(4))
def test_reachable_quotient_is_language_equivalent_and_minimal(seed):
    d = W.random_dfa(300, 2, 0.5, 90 + seed)
    block, nb, _ = oracle.minimise_reachable(d.delta, d.accepting, 0)
    mask = block != oracle.UNREACHABLE
    # quotient of the reachable part, built by hand from the block ids
    leaders = np.flatnonzero(mask & (block == np.arange(d.n)))
    dense = {int(l): i for i, l in enumerate(leaders)}
    qd = np.array([[dense[int(block[d.delta[l, a]])] for a in range(d.k)] for l in leaders],
                  dtype=np.uint32)
    qa = d.accepting[leaders]
    assert len(leaders) == nb
    assert oracle.equiv_hk(d.delta, d.accepting, 0, qd, qa, dense[int(block[0])])
    # minimal: Hopcroft finds nothing to merge, and every state is reachable
    _, qnb = oracle.hopcroft(qd, qa)
    assert qnb == nb
    assert oracle.reachable(qd, dense[int(block[0])]).all()
