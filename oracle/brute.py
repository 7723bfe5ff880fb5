"""Exact brute force for tiny graphs -- TEST INFRASTRUCTURE ONLY.

Betweenness straight from its definition (the paper's Eq. (1)): enumerate
every simple path between every ordered pair (s, t), keep those of minimum
length, and credit each inner vertex v with (paths through v) / (all shortest
paths), as exact fractions.  No BFS, no recursion over dependencies: it
shares nothing with Brandes' method, which makes it a pin for the oracle.
Exponential in n; use n <= 10.
"""
from __future__ import annotations

from fractions import Fraction


def _adj(g):
    return [list(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]) for v in range(g.n)]


def shortest_paths(g, s: int):
    """For every target t: (length, list of shortest s-t paths as tuples)."""
    adj = _adj(g)
    best = {}
    stack = [(s, (s,))]
    while stack:
        v, p = stack.pop()
        L = len(p) - 1
        cur = best.get(v)
        if cur is None or L < cur[0]:
            best[v] = (L, [p])
        elif L == cur[0]:
            cur[1].append(p)
        for w in adj[v]:
            if w not in p:
                stack.append((int(w), p + (int(w),)))
    return best


def bc_exact(g):
    """RAW betweenness (ordered pairs) as a list of Fractions; also returns
    d[s][t] (None = unreachable) and sigma[s][t]."""
    n = g.n
    raw = [Fraction(0)] * n
    d = [[None] * n for _ in range(n)]
    sig = [[0] * n for _ in range(n)]
    for s in range(n):
        sp = shortest_paths(g, s)
        for t, (L, paths) in sp.items():
            d[s][t] = L
            sig[s][t] = len(paths)
            if t == s:
                continue
            through = [0] * n
            for p in paths:
                for v in p[1:-1]:
                    through[v] += 1
            for v in range(n):
                if through[v]:
                    raw[v] += Fraction(through[v], len(paths))
    return raw, d, sig
