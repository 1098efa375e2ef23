"""Reader for the fixtures under tests/golden (automata typed from the paper's
figures, and table columns)."""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for raw in f:
            line = raw.strip()
            if line and not line.startswith("#"):
                yield line.split()


def load_automaton(name):
    """Returns dict(names, letters, delta [n,k] uint32 or -1 where unset,
    accepting uint8 [n], start index or None, extra lines)."""
    names, letters, start, acc_names, edges, extra = [], [], None, [], [], []
    default_loop = False
    for tok in _lines(name):
        if tok[0] == "names":
            names = tok[1:]
        elif tok[0] == "letters":
            letters = tok[1:]
        elif tok[0] == "start":
            start = tok[1]
        elif tok[0] == "accepting":
            acc_names = tok[1:]
        elif tok[0] == "edge":
            edges.append(tok[1:])
        elif tok[0] == "default" and tok[1] == "loop":
            default_loop = True
        else:
            extra.append(tok)
    idx = {s: i for i, s in enumerate(names)}
    lidx = {a: j for j, a in enumerate(letters)}
    n, k = len(names), len(letters)
    delta = np.full((n, k), -1, dtype=np.int64)
    if default_loop:
        delta[:] = np.arange(n)[:, None]
    for src, a, dst in edges:
        delta[idx[src], lidx[a]] = idx[dst]
    assert (delta >= 0).all(), f"{name}: incomplete transition function"
    acc = np.zeros(n, dtype=np.uint8)
    for s in acc_names:
        acc[idx[s]] = 1
    return dict(names=names, letters=letters, delta=delta.astype(np.uint32), accepting=acc,
                start=None if start is None else idx[start], extra=extra, index=idx)


def load_table(name):
    return [tok for tok in _lines(name)]
