"""Pins of the oracle (and of the input generators) to values the paper prints.

Each test names the figure, table or passage it checks.  No expected value
here comes from the GPU path.
"""
import numpy as np
import pytest

import oracle
from goldenio import load_automaton, load_table
from paper_2508_20735_amd import workloads as W


def _reindex(g, name_to_gen):
    """Golden automaton expressed in the generator's state numbering."""
    names = g["names"]
    gen = np.array([name_to_gen(s) for s in names], dtype=np.int64)
    n, k = g["delta"].shape
    delta = np.empty((n, k), dtype=np.uint32)
    acc = np.empty(n, dtype=np.uint8)
    delta[gen] = gen[g["delta"]]
    acc[gen] = g["accepting"]
    start = None if g["start"] is None else int(gen[g["start"]])
    return delta, acc, start


def _qi(s):
    return int(s[1:])


def _bits(s):
    return int(s, 2)


def _cbits(s):
    c, sigma = s.split(".")
    return (int(c) << len(sigma)) | int(sigma, 2)


# ---------------------------------------------------------------- figures

@pytest.mark.parametrize("fixture,gen,key", [
    ("fig1_chain.txt", lambda: W.fig1_chain(), _qi),
    ("fib5.txt", lambda: W.fibonacci(5), _qi),
    ("b3.txt", lambda: W.bitsplitter(3), _bits),
    ("c5.txt", lambda: W.cycle(5), _qi),
    ("b3prime.txt", lambda: W.extended_bitsplitter(3), _cbits),
    ("memory2.txt", lambda: W.memory(2, False), _bits),
    ("memory3_perfect.txt", lambda: W.memory(3, False), _bits),
    ("memory3_forgetful.txt", lambda: W.memory(3, True), _bits),
])
def test_generators_reproduce_figures(fixture, gen, key):
    """Figs. 1, 2, 5, 6, 7: the generators build exactly the drawn automata."""
    g = load_automaton(fixture)
    delta, acc, start = _reindex(g, key)
    d = gen()
    np.testing.assert_array_equal(d.delta, delta)
    np.testing.assert_array_equal(d.accepting, acc)
    if start is not None:
        assert d.start == start


def test_fig1_closure_arrows_and_rounds():
    """Fig. 1: pointer jumping gives q0 -a^2-> q2, -a^4-> q4, -a^8-> q8, and
    plain refinement needs 8 rounds to separate q0 from q1."""
    g = load_automaton("fig1_chain.txt")
    ext = oracle.pointer_jump(g["delta"])
    assert oracle.floor_log2(10) == 3
    closure = {tok[2]: tok[3] for tok in g["extra"] if tok[0] == "closure"}
    assert ext.shape == (10, 4)
    for i, power in enumerate(["a", "a^2", "a^4", "a^8"]):
        if power in closure:
            assert ext[0, i] == g["index"][closure[power]]
    assert ext[0, 0] == 1
    rounds_needed = int([t for t in g["extra"] if t[0] == "min_rounds_plain"][0][1])
    # q0 and q1 are first separated in round 8: after 7 rounds they share a block
    block = np.where(g["accepting"] == 1, 9, 0).astype(np.uint32)
    block = oracle.canonicalise(block)
    for r in range(1, rounds_needed + 1):
        block, _ = oracle.moore_round(g["delta"], block)
        assert (block[0] == block[1]) == (r < rounds_needed)
    _, nb, rounds, changing = oracle.moore(g["delta"], g["accepting"])
    assert nb == 10 and changing == rounds_needed and rounds == rounds_needed + 1
    # language: accepts a^j iff j > 8, i.e. q0 is distinguished from q1 by a^8 only
    hb, _ = oracle.hopcroft(g["delta"], g["accepting"])
    np.testing.assert_array_equal(hb, np.arange(10))


# ---------------------------------------------------------------- Fibonacci

def test_fibonacci_words():
    """Section 5.1: w_2 = 01, w_3 = 010, w_4 = 01001, w_5 = 01001010."""
    assert [W.fibonacci_word(i) for i in (2, 3, 4, 5)] == ["01", "010", "01001", "01001010"]


@pytest.mark.parametrize("i", range(4, 16))
def test_fibonacci_distinguishing_depth(i):
    """Section 3.3 (end): Fib with n states has a pair whose shortest
    distinguishing word has length n-2, so n-2 refining rounds; Table 2: every
    Fib DFA is already minimal (output size = N) and sortPR iterates N-1 times
    (the n-2 refining rounds plus the one that confirms stability)."""
    d = W.fibonacci(i)
    n = d.n
    block, nb, rounds, changing = oracle.moore(d.delta, d.accepting)
    assert nb == n
    assert changing == n - 2
    assert rounds == n - 1
    hb, hnb = oracle.hopcroft(d.delta, d.accepting)
    assert hnb == n
    np.testing.assert_array_equal(hb, block)


def test_table2_fibonacci_sizes():
    """Table 2, N and output-size columns for Fib_18 .. Fib_30 (table index =
    word index - 1), and sortPR iterations = N - 1 where reported."""
    for name, N, k, out, iters in load_table("table2.txt"):
        if not name.startswith("Fib"):
            continue
        i = int(name[3:]) + 1
        assert len(W.fibonacci_word(i)) == int(N)
        assert int(k) == 1 and int(out) == int(N)
        if iters != "-":
            assert int(iters) == int(N) - 1


def test_table2_fib18_full():
    """Table 2 row Fib_18: N = 6765, output 6765 states, 6764 iterations."""
    d = W.fibonacci(19)
    assert d.n == 6765
    hb, hnb = oracle.hopcroft(d.delta, d.accepting)
    assert hnb == 6765
    _, nb, rounds, changing = oracle.moore(d.delta, d.accepting)
    assert nb == 6765 and rounds == 6764 and changing == 6763


# ---------------------------------------------------------------- bit-splitters

@pytest.mark.parametrize("n", range(2, 13))
def test_bitsplitter_halving(n):
    """Section 5.1 and Table 2: B_n has 2^n states and n-1 letters, is minimal,
    every split halves a block, and the iteration count is n-1."""
    d = W.bitsplitter(n)
    assert d.n == 2 ** n and d.k == n - 1
    block = oracle.canonicalise(d.accepting.astype(np.uint32))
    sizes = [2]
    for _ in range(n - 1):
        block, c = oracle.moore_round(d.delta, block)
        sizes.append(c)
    # every round doubles the block count: each block splits into two halves
    assert sizes == [2 ** (r + 1) for r in range(n)]
    _, counts = np.unique(block, return_counts=True)
    assert (counts == 1).all()
    _, nb, rounds, changing = oracle.moore(d.delta, d.accepting)
    assert nb == 2 ** n and changing == n - 1
    hb, hnb = oracle.hopcroft(d.delta, d.accepting)
    assert hnb == 2 ** n


def test_table2_bitsplitter_rows():
    """Table 2, B_15 .. B_26: N = 2^n, |Sigma| = n - 1, output N, iterations
    n - 1 (checked by Moore up to B_16)."""
    for name, N, k, out, iters in load_table("table2.txt"):
        if not name.startswith("B"):
            continue
        n = int(name[1:])
        assert int(N) == 2 ** n and int(k) == n - 1 and int(out) == int(N)
        assert int(iters) == n - 1
        if n <= 16:
            d = W.bitsplitter(n)
            _, nb, _, changing = oracle.moore(d.delta, d.accepting)
            assert nb == int(out) and changing == int(iters)


# ---------------------------------------------------------------- equivalence / inclusion

def test_table4_self_equivalence_counts():
    """Table 4: the self-equivalence product of B'_n has 2^(n+1) states and
    that of C_n has fib(n) states (checked by exploration up to B'_16 and
    C_28, by the generator's size beyond)."""
    for name, count in load_table("table4.txt"):
        count = int(count)
        if name.startswith("B"):
            n = int(name[1:])
            assert 2 ** (n + 1) == count
            if n <= 16:
                d = W.extended_bitsplitter(n)
                ok, visited = oracle.product_bfs(d.delta, d.accepting, 0, d.delta, d.accepting, 0,
                                                 "equivalence")
                assert ok and visited == count
        else:
            n = int(name[1:])
            assert W.fib_numbers(n) == count
    for n in (10, 20, 28):
        d = W.cycle(n)
        ok, visited = oracle.product_bfs(d.delta, d.accepting, 0, d.delta, d.accepting, 0,
                                         "equivalence")
        assert ok and visited == W.fib_numbers(n)
        assert oracle.equiv_hk(d.delta, d.accepting, 0, d.delta, d.accepting, 0)


def test_table5_inclusion_counts():
    """Table 5 and Section 6.2: L(forgetful memory_n) is included in
    L(perfect memory_n) and the explored product has the printed number of
    states (checked by exploration up to n = 18); the converse inclusion
    fails (forgetting only rejects words the perfect DFA accepts)."""
    for n, count in load_table("table5.txt"):
        n, count = int(n), int(count)
        if n > 18:
            continue
        F = W.memory(n, True)
        P = W.memory(n, False)
        ok, visited = oracle.product_bfs(F.delta, F.accepting, 0, P.delta, P.accepting, 0)
        assert ok and visited == count
        assert not oracle.included(P.delta, P.accepting, 0, F.delta, F.accepting, 0)
        assert not oracle.equiv_hk(F.delta, F.accepting, 0, P.delta, P.accepting, 0)


def test_memory2_self_equivalence():
    """Fig. 3 checks two copies of memory_2 for equivalence: they are equal."""
    d = W.memory(2, False)
    assert oracle.equiv_hk(d.delta, d.accepting, 0, d.delta, d.accepting, 0)
    ok, visited = oracle.product_bfs(d.delta, d.accepting, 0, d.delta, d.accepting, 0,
                                     "equivalence")
    assert ok and visited == 4
