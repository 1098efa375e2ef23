"""Brute-force word enumeration (TEST INFRASTRUCTURE ONLY).

This is the plain definition of language equivalence from Section 2 of the
paper: states p and q are equivalent iff for every word w, delta*(p, w) is
accepting exactly when delta*(q, w) is.  Only words up to a finite length need
checking: the refinement chain {F, Q\\F} = P_0 >= P_1 >= ... strictly grows the
number of blocks until it is stable, and it has at most n blocks, so states
that agree on every word of length <= max(n - 2, 0) are equivalent.  For two
DFAs the same bound applies to their disjoint union (length nA + nB - 2); for
inclusion every reachable pair of the synchronous product is reached by a word
of length < nA * nB.

Exponential in the word length: for tiny inputs only.  Vectorised over many
instances of one shape so the exhaustive tests stay fast.
"""
from __future__ import annotations

import numpy as np


def _accept_matrix(delta: np.ndarray, acc: np.ndarray, max_len: int) -> np.ndarray:
    """acc_after[..., q, w] for all words w of length 0..max_len.

    delta: [..., n, k] targets, acc: [..., n] bool.  Words are enumerated
    length by length; the column order is irrelevant to the callers."""
    delta = np.asarray(delta, dtype=np.int64)
    acc = np.asarray(acc) != 0
    lead = delta.shape[:-2]
    n, k = delta.shape[-2:]
    # cur[..., q, j] = state reached from q by the j-th word of the current length
    cur = np.broadcast_to(np.arange(n), lead + (n,))[..., None].copy()
    cols = []
    for length in range(max_len + 1):
        cols.append(np.take_along_axis(acc, cur.reshape(lead + (-1,)), axis=-1)
                    .reshape(cur.shape))
        if length == max_len:
            break
        # extend every word by every letter: next state = delta[cur, a]
        nxt = []
        for a in range(k):
            da = delta[..., :, a]  # [..., n]
            nxt.append(np.take_along_axis(da, cur.reshape(lead + (-1,)), axis=-1)
                       .reshape(cur.shape))
        cur = np.concatenate(nxt, axis=-1)
    return np.concatenate(cols, axis=-1)


def partition_by_words(delta, acc, max_len: int | None = None) -> np.ndarray:
    """Canonical partition (block[q] = smallest equivalent state) of one DFA or
    a stack of DFAs of one shape ([..., n, k]), by comparing acceptance on all
    words up to ``max_len`` (default max(n - 2, 0))."""
    delta = np.asarray(delta)
    n = delta.shape[-2]
    if max_len is None:
        max_len = max(n - 2, 0)
    sig = _accept_matrix(delta, acc, max_len)  # [..., n, W]
    same = np.all(sig[..., :, None, :] == sig[..., None, :, :], axis=-1)  # [..., n, n]
    # smallest q' equal to q: first True along the last axis
    return np.argmax(same, axis=-1).astype(np.uint32)


def equivalent_by_words(dA, accA, sA, dB, accB, sB) -> bool:
    """L(A) == L(B), checked on every word of length <= nA + nB - 2."""
    dA = np.asarray(dA, dtype=np.int64)
    dB = np.asarray(dB, dtype=np.int64)
    nA, nB = dA.shape[0], dB.shape[0]
    d = np.concatenate([dA, dB + nA])
    acc = np.concatenate([np.asarray(accA) != 0, np.asarray(accB) != 0])
    sig = _accept_matrix(d, acc, max(nA + nB - 2, 0))
    return bool(np.array_equal(sig[sA], sig[nA + sB]))


def included_by_words(dA, accA, sA, dB, accB, sB) -> bool:
    """L(A) <= L(B), checked on every word of length < nA * nB."""
    dA = np.asarray(dA, dtype=np.int64)
    dB = np.asarray(dB, dtype=np.int64)
    nA, nB = dA.shape[0], dB.shape[0]
    d = np.concatenate([dA, dB + nA])
    acc = np.concatenate([np.asarray(accA) != 0, np.asarray(accB) != 0])
    sig = _accept_matrix(d, acc, max(nA * nB - 1, 0))
    a, b = sig[sA], sig[nA + sB]
    return bool(np.all(~a | b))
