"""Brute-force shortest paths by enumerating every simple path (tiny graphs).

TEST INFRASTRUCTURE ONLY.  With non-negative weights some shortest walk is a
simple path, so the minimum over simple paths is the shortest distance; the
empty path gives d(i,i) = 0.  This is the definition of the quantity that
repeated squaring (Sec. III) and Floyd-Warshall (Algorithm 2) compute, written
as a search that shares nothing with either.  Exponential: n <= 7 only.
"""
from __future__ import annotations

import math


def brute_force_apsp(W, absent):
    """W: n x n nested sequence or array; ``absent`` marks a missing edge.

    Returns an n x n list of Python numbers (ints stay ints); pairs with no
    path get ``absent``.  Diagonal entries of W are ignored (self loops never
    shorten a path when weights are non-negative).
    """
    n = len(W)
    if n > 9:
        raise ValueError("brute force is for tiny graphs")
    w = [[W[i][j] for j in range(n)] for i in range(n)]
    best = [[None] * n for _ in range(n)]

    def walk(src, node, dist, seen):
        cur = best[src][node]
        if cur is None or dist < cur:
            best[src][node] = dist
        for nxt in range(n):
            if nxt in seen:
                continue
            wt = w[node][nxt]
            if wt == absent or (isinstance(wt, float) and math.isinf(wt)):
                continue
            walk(src, nxt, dist + wt, seen | {nxt})

    for s in range(n):
        walk(s, s, 0, {s})
    return [[absent if best[i][j] is None else best[i][j] for j in range(n)] for i in range(n)]
