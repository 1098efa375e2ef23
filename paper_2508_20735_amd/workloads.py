"""Seeded synthetic DFA generators.

Shared by the tests, the benchmark and the oracle checks.  This module only
builds input automata (row-major ``delta[q, a]`` uint32 arrays and ``accepting``
uint8 arrays); it contains none of the minimisation / equivalence arithmetic.

Families follow Section 5.1 of Heemstra, Martens, Wijs (Fibonacci DFAs,
bit-splitters, cycle DFAs, extended bit-splitters, memory DFAs) and the
Fig. 1 chain of Section 3.4.  Random workloads use numpy's PCG64 with fixed
seeds: targets are drawn first (``integers(0, n, (n, k))``), then the
acceptance coins (``random(n) < p``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class DFA:
    delta: np.ndarray      # uint32 [n, k], row-major
    accepting: np.ndarray  # uint8 [n]
    start: int = 0

    @property
    def n(self) -> int:
        return int(self.delta.shape[0])

    @property
    def k(self) -> int:
        return int(self.delta.shape[1])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# random complete DFAs
# --------------------------------------------------------------------------

def random_dfa(n: int, k: int, p: float, seed: int) -> DFA:
    """Uniform random complete DFA: every target uniform in [0, n), every
    state accepting with probability p, start state 0."""
    rng = _rng(seed)
    delta = rng.integers(0, n, size=(n, k), dtype=np.uint32)
    acc = (rng.random(n) < p).astype(np.uint8)
    return DFA(delta, acc, 0)


def permuted_copy(dfa: DFA, seed: int) -> tuple[DFA, np.ndarray]:
    """Rename states by a random permutation pi: delta'[pi(q)][a] = pi(delta[q][a]),
    acc'[pi(q)] = acc[q], start' = pi(start).  Returns (copy, pi)."""
    rng = _rng(seed)
    pi = rng.permutation(dfa.n).astype(np.uint32)
    delta = np.empty_like(dfa.delta)
    delta[pi] = pi[dfa.delta]
    acc = np.empty_like(dfa.accepting)
    acc[pi] = dfa.accepting
    return DFA(delta, acc, int(pi[dfa.start])), pi


def mutate_one(dfa: DFA, seed: int) -> tuple[DFA, tuple[int, int]]:
    """Redirect one uniformly chosen transition (q, a) to a different target,
    uniform over the other n - 1 states.  Returns (copy, (q, a))."""
    rng = _rng(seed)
    q = int(rng.integers(0, dfa.n))
    a = int(rng.integers(0, dfa.k))
    old = int(dfa.delta[q, a])
    t = int(rng.integers(0, max(dfa.n - 1, 1)))
    if dfa.n > 1 and t >= old:
        t += 1
    delta = dfa.delta.copy()
    delta[q, a] = t if dfa.n > 1 else old
    return DFA(delta, dfa.accepting.copy(), dfa.start), (q, a)


# --------------------------------------------------------------------------
# the paper's families
# --------------------------------------------------------------------------

def fig1_chain(length: int = 10) -> DFA:
    """Fig. 1: q0 -a-> q1 -a-> ... -a-> q_{len-1}, the last state accepting with
    an a-loop.  With 10 states it accepts a^j for j > 8."""
    delta = np.minimum(np.arange(length) + 1, length - 1).astype(np.uint32)[:, None]
    acc = np.zeros(length, dtype=np.uint8)
    acc[-1] = 1
    return DFA(delta, acc, 0)


def fibonacci_word(i: int) -> str:
    """w_0 = 1, w_1 = 0, w_{i+1} = w_i w_{i-1}."""
    if i == 0:
        return "1"
    prev, cur = "1", "0"
    for _ in range(i - 1):
        prev, cur = cur, cur + prev
    return cur


def fibonacci(i: int) -> DFA:
    """Fib_i: a unary cycle over the bits of w_i; q_j accepting iff w_i[j] = 1."""
    w = fibonacci_word(i)
    n = len(w)
    delta = ((np.arange(n) + 1) % n).astype(np.uint32)[:, None]
    acc = np.frombuffer(w.encode(), dtype=np.uint8) - ord("0")
    return DFA(delta, acc.astype(np.uint8), 0)


def bitsplitter(n: int) -> DFA:
    """B_n: 2^n states (bit strings, most significant bit first), letters
    a_1..a_{n-1} at columns 0..n-2.  Letter a_j acts on the low j+1 bits
    b sigma: if sigma's leading bit (bit j-1) is 1 they become (not b) 0^j,
    otherwise the state loops.  Accepting iff the leading bit is 1.  The
    family has no initial state; start is reported as 0."""
    if n < 2:
        raise ValueError("bit-splitters need n >= 2 (B_1 has no letters)")
    N = 1 << n
    s = np.arange(N, dtype=np.uint32)
    delta = np.empty((N, n - 1), dtype=np.uint32)
    for j in range(1, n):
        # moved = high bits kept, bit j inverted, bits below j cleared
        moved = (s >> np.uint32(j + 1)) << np.uint32(j + 1)
        moved |= (~(s >> np.uint32(j)) & np.uint32(1)) << np.uint32(j)
        lead = (s >> np.uint32(j - 1)) & np.uint32(1)
        delta[:, j - 1] = np.where(lead == 1, moved, s)
    acc = ((s >> np.uint32(n - 1)) & np.uint32(1)).astype(np.uint8)
    return DFA(delta, acc, 0)


def fib_numbers(i: int) -> int:
    """fib(0) = fib(1) = 1, fib(i) = fib(i-1) + fib(i-2)."""
    a, b = 1, 1
    for _ in range(i - 1):
        a, b = b, a + b
    return b if i >= 1 else a


def round_half_up(x: float) -> int:
    return int(math.floor(x + 0.5))


def cycle(i: int) -> DFA:
    """C_i: fib(i) states, letters a_0..a_m with m = max(round(log10 fib(i)), 1),
    delta(q_j, a_l) = q_{(j + 100 l + 1) mod fib(i)}, F = {q_fib(i-1)}."""
    N = fib_numbers(i)
    m = max(round_half_up(math.log10(N)), 1)
    j = np.arange(N, dtype=np.int64)
    delta = np.stack([(j + 100 * l + 1) % N for l in range(m + 1)], axis=1).astype(np.uint32)
    acc = np.zeros(N, dtype=np.uint8)
    acc[fib_numbers(i - 1)] = 1
    return DFA(delta, acc, 0)


def extended_bitsplitter(n: int) -> DFA:
    """B'_n: states (c, sigma), sigma an n-bit string; index c*2^n + sigma.
    Columns: b_0..b_{n-1}, then a_1..a_{n-1}, then r.
      b_j: if c = 0 and bit j = 0, set bit j; otherwise loop.
      a_j: if c = 1 and bit j-1 = 1, the low j+1 bits (b sigma') become
           (not b) 0^j; otherwise loop.
      r:   c := 1.
    Accepting iff c = 1 and the leading bit of sigma is 1.  Start (0, 0^n)."""
    if n < 1:
        raise ValueError("n >= 1")
    N = 1 << n
    idx = np.arange(2 * N, dtype=np.int64)
    c = idx >> n
    s = idx & (N - 1)
    cols = []
    for j in range(n):
        bit = (s >> j) & 1
        cols.append(np.where((c == 0) & (bit == 0), idx | (1 << j), idx))
    for j in range(1, n):
        b = (s >> j) & 1
        lead = (s >> (j - 1)) & 1
        high = (s >> (j + 1)) << (j + 1)
        moved = (c << n) | high | ((1 - b) << j)
        cols.append(np.where((c == 1) & (lead == 1), moved, idx))
    cols.append(idx | N)
    delta = np.stack(cols, axis=1).astype(np.uint32)
    acc = ((c == 1) & (((s >> (n - 1)) & 1) == 1)).astype(np.uint8)
    return DFA(delta, acc, 0)


def memory(n: int, forgetful: bool) -> DFA:
    """memory_n: states are the last n bits read (most significant = oldest),
    letters 0 and 1 shift the read bit in.  The forgetful variant resets to
    0^{n-1}x when the two most significant bits are 10.  Accepting iff the most
    significant bit is 1.  Start 0^n."""
    if n < 2:
        raise ValueError("n >= 2")
    N = 1 << n
    s = np.arange(N, dtype=np.int64)
    cols = []
    for x in (0, 1):
        nxt = ((s << 1) | x) & (N - 1)
        if forgetful:
            top2 = s >> (n - 2)
            nxt = np.where(top2 == 0b10, x, nxt)
        cols.append(nxt)
    delta = np.stack(cols, axis=1).astype(np.uint32)
    acc = ((s >> (n - 1)) & 1).astype(np.uint8)
    return DFA(delta, acc, 0)


# --------------------------------------------------------------------------
# benchmark workloads
# --------------------------------------------------------------------------

def chain_with_tail(N: int, tail: int, seed: int, p: float = 0.5, k: int = 2) -> DFA:
    """Chain part: N states, letter 0: i -> min(i+1, N-1), every other letter
    the identity, only N-1 accepting.  Random tail: ``tail`` states with all k
    letters uniform over the tail [N, N+tail) and acceptance probability p.
    With k = 2 this is the chain-structured workload (letters a and b)."""
    if k < 1:
        raise ValueError("k >= 1")
    rng = _rng(seed)
    i = np.arange(N, dtype=np.uint32)
    chain = np.stack([np.minimum(i + 1, N - 1)] + [i] * (k - 1), axis=1).astype(np.uint32)
    tail_delta = rng.integers(N, N + tail, size=(tail, k), dtype=np.uint32) if tail else \
        np.zeros((0, k), dtype=np.uint32)
    tail_acc = (rng.random(tail) < p).astype(np.uint8)
    acc = np.zeros(N, dtype=np.uint8)
    acc[N - 1] = 1
    return DFA(np.concatenate([chain, tail_delta]), np.concatenate([acc, tail_acc]), 0)


# the five workload configurations
CFG_SMALL = dict(n=10_000, k=2, p=0.5, seed=1)
CFG_LARGE = dict(n=1 << 22, k=4, p=0.1, seed=2)
CFG_LARGE_PERM_SEED = 20
CFG_LARGE_MUT_SEED = 21
CFG_CHAIN = dict(N=1 << 20, tail=1 << 20, seed=3)


def cfg_small() -> DFA:
    return random_dfa(**CFG_SMALL)


def cfg_large() -> DFA:
    return random_dfa(**CFG_LARGE)


def cfg_chain() -> DFA:
    return chain_with_tail(**CFG_CHAIN)


@dataclass
class BatchItem:
    dfa: DFA
    pair: DFA | None = None       # second operand of an equivalence check
    pair_kind: str | None = None  # "permuted" or "mutated"


def batch_workload(count: int = 4096, seed: int = 4, nmin: int = 64, nmax: int = 65_536,
                   kmin: int = 2, kmax: int = 8, paired_from: int | None = None) -> list[BatchItem]:
    """Independent random DFAs: n = round(exp(U[ln nmin, ln nmax])),
    k uniform in {kmin..kmax}, p uniform in [0.05, 0.5].  Items with index >=
    paired_from (default count/2) also carry an equivalence operand: even
    index -> permuted copy (equivalent), odd -> one-transition mutation."""
    rng = _rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=count))).astype(np.int64)
    ks = rng.integers(kmin, kmax + 1, size=count)
    ps = rng.uniform(0.05, 0.5, size=count)
    sub = rng.integers(0, 2**62, size=count)
    if paired_from is None:
        paired_from = count // 2
    items = []
    for i in range(count):
        d = random_dfa(int(ns[i]), int(ks[i]), float(ps[i]), int(sub[i]))
        item = BatchItem(d)
        if i >= paired_from:
            if i % 2 == 0:
                item.pair, item.pair_kind = permuted_copy(d, int(sub[i]) + 1)[0], "permuted"
            else:
                item.pair, item.pair_kind = mutate_one(d, int(sub[i]) + 2)[0], "mutated"
        items.append(item)
    return items


@dataclass
class ServeRequest:
    kind: str            # "minimise" or "equivalent"
    dfa: DFA
    other: DFA | None    # second operand of an equivalence request
    arrival: float       # seconds after the start of the stream


def serving_workload(count: int, rate: float, seed: int = 5, nmin: int = 1000,
                     nmax: int = 4_194_304, letters=(2, 4, 8, 16), p_equivalent: float = 0.2,
                     p_chain: float = 0.1) -> list[ServeRequest]:
    """Request stream: Poisson arrivals at `rate` per second, 80% minimise /
    20% equivalence (against a permuted copy or a one-transition mutation,
    alternately), n log-uniform in [nmin, nmax], k uniform in `letters`, and
    a fraction p_chain of chain DFAs (half chain, half random tail, with the
    drawn k: letter 0 steps the chain, the others are the identity on it)."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=count))).astype(np.int64)
    ks = rng.choice(np.asarray(letters), size=count)
    kinds = rng.random(count) < p_equivalent
    chains = rng.random(count) < p_chain
    ps = rng.uniform(0.05, 0.5, size=count)
    sub = rng.integers(0, 2**62, size=count)
    out = []
    for i in range(count):
        n, k = int(ns[i]), int(ks[i])
        if chains[i]:
            d = chain_with_tail(max(n // 2, 2), n - max(n // 2, 2), int(sub[i]), k=k)
        else:
            d = random_dfa(n, k, float(ps[i]), int(sub[i]))
        if kinds[i]:
            other = permuted_copy(d, int(sub[i]) + 1)[0] if i % 2 == 0 else \
                mutate_one(d, int(sub[i]) + 2)[0]
            out.append(ServeRequest("equivalent", d, other, float(arrivals[i])))
        else:
            out.append(ServeRequest("minimise", d, None, float(arrivals[i])))
    return out
