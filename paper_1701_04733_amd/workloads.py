"""Seeded synthetic inputs for the tropical GEMM and APSP workloads.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic, so both the GPU path and the CPU oracle can be fed from
it.  Everything is numpy ``Generator(PCG64(seed))``; per-graph streams come
from ``SeedSequence(seed).spawn``.  The paper's own experiments use "random
matrices" of 4 to 128 vertices with an unstated weight law (Sec. IV, Table II);
the recipes below are the shapes and distributions of the workloads this
library is measured on.

Sentinels used to mark absent entries (min-plus +INF, max-plus -INF) are the
library-wide constants restated here as plain numbers so that this module
imports nothing from either side.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

I32_INF = 0x7FFFFFFF
I32_NINF = -0x7FFFFFFF


def rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# Dense tropical GEMM operands (8192^3 workload and smaller parity shapes)
# --------------------------------------------------------------------------

def gemm_operand(shape, dtype: str, semiring: str, seed: int, inf_frac: float = 0.1,
                 int_hi: int = 10**6) -> np.ndarray:
    """fp32: uniform [0,1); int32: uniform integers in [0, int_hi].

    A fraction ``inf_frac`` of entries is set to the semiring's absent value
    (+inf / +INF for min-plus, -inf / -INF for max-plus).
    """
    g = rng(seed)
    if dtype == "f32":
        x = g.random(shape, dtype=np.float32)
        absent = np.float32(np.inf if semiring == "min" else -np.inf)
    elif dtype == "i32":
        x = g.integers(0, int_hi, size=shape, endpoint=True, dtype=np.int32)
        absent = np.int32(I32_INF if semiring == "min" else I32_NINF)
    else:
        raise ValueError(dtype)
    if inf_frac > 0:
        mask = g.random(shape, dtype=np.float32) < inf_frac
        x[mask] = absent
    return x


def semiring_identity_matrix(shape, dtype: str, semiring: str) -> np.ndarray:
    """A matrix filled with the (+)-identity (the accumulator's start value)."""
    if dtype == "f32":
        return np.full(shape, np.inf if semiring == "min" else -np.inf, dtype=np.float32)
    return np.full(shape, I32_INF if semiring == "min" else I32_NINF, dtype=np.int32)


def signed_operand(shape, dtype: str, semiring: str, seed: int, inf_frac: float = 0.1,
                   bound: int = (1 << 29) - 1) -> np.ndarray:
    """Signed values over the whole int32 contract range, or signed fp32 values
    spanning many binades, with absent entries.  Used for edge-case parity."""
    g = rng(seed)
    if dtype == "i32":
        x = g.integers(-bound, bound, size=shape, endpoint=True, dtype=np.int64).astype(np.int32)
        absent = np.int32(I32_INF if semiring == "min" else I32_NINF)
    else:
        mant = g.random(shape) * 2.0 - 1.0
        expo = g.integers(-40, 40, size=shape)
        x = (mant * np.exp2(expo)).astype(np.float32)
        absent = np.float32(np.inf if semiring == "min" else -np.inf)
    if inf_frac > 0:
        x[g.random(shape) < inf_frac] = absent
    return x


# --------------------------------------------------------------------------
# Graphs
# --------------------------------------------------------------------------

def er_digraph_i32(n: int, p: float, w_lo: int, w_hi: int, seed) -> np.ndarray:
    """Directed Erdos-Renyi graph as a dense int32 weight matrix.

    Each ordered pair i != j is an edge with probability p; weights are uniform
    integers in [w_lo, w_hi]; absent edges are +INF; the diagonal is 0.
    """
    g = rng(seed)
    mask = g.random((n, n)) < p
    w = g.integers(w_lo, w_hi, size=(n, n), endpoint=True, dtype=np.int32)
    W = np.where(mask, w, np.int32(I32_INF)).astype(np.int32)
    np.fill_diagonal(W, 0)
    return W


def _sparse_rows(g: np.random.Generator, n: int, p: float):
    """Edges (rows, cols) of an ER digraph without self loops, sorted.

    The edge count is Binomial(n(n-1), p) and the edge set a uniform subset of
    that size of the n(n-1) ordered pairs, which is the same law as one
    independent coin per pair."""
    if n < 2:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    pairs = n * (n - 1)
    m = int(g.binomial(pairs, p))
    idx = np.sort(g.choice(pairs, size=m, replace=False))
    r = idx // (n - 1)
    c = idx % (n - 1)
    c = c + (c >= r)
    return r.astype(np.int64), c.astype(np.int64)


def sparse_digraph_f32_exp(n: int, mean_degree: float, seed, mean_weight: float = 1.0):
    """COO digraph: pair i != j is an edge w.p. mean_degree/(n-1); weights are
    exponential(mean_weight) rounded to fp32.  Returns (rows, cols, w)."""
    g = rng(seed)
    p = min(1.0, mean_degree / max(1, n - 1))
    r, c = _sparse_rows(g, n, p)
    w = g.exponential(mean_weight, size=r.size).astype(np.float32)
    return r, c, w


def coo_to_dense_f32(n: int, rows, cols, w) -> np.ndarray:
    """Dense fp32 weight matrix: absent +inf, diagonal 0 (layout only)."""
    W = np.full((n, n), np.inf, dtype=np.float32)
    W[rows, cols] = w
    np.fill_diagonal(W, 0.0)
    return W


def apsp_large_f32(n: int = 16384, mean_degree: float = 16.0, seed: int = 4) -> np.ndarray:
    """Large single APSP: mean out-degree 16, exponential(1) fp32 weights."""
    r, c, w = sparse_digraph_f32_exp(n, mean_degree, seed)
    return coo_to_dense_f32(n, r, c, w)


def log_uniform_sizes(count: int, lo: int, hi: int, g: np.random.Generator) -> np.ndarray:
    u = g.uniform(math.log(lo), math.log(hi), size=count)
    return np.clip(np.rint(np.exp(u)), lo, hi).astype(np.int64)


def batched_graphs_i32(count: int = 4096, lo: int = 16, hi: int = 512, seed: int = 5,
                       deg: float = 8.0, w_lo: int = 1, w_hi: int = 1000):
    """Many independent ER digraphs with n log-uniform in [lo, hi], edge
    probability deg/n, int32 weights uniform in [w_lo, w_hi]."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(count)
    out = []
    for g_ss in children:
        g = np.random.Generator(np.random.PCG64(g_ss))
        n = int(log_uniform_sizes(1, lo, hi, g)[0])
        p = min(1.0, deg / n)
        mask = g.random((n, n)) < p
        w = g.integers(w_lo, w_hi, size=(n, n), endpoint=True, dtype=np.int32)
        W = np.where(mask, w, np.int32(I32_INF)).astype(np.int32)
        np.fill_diagonal(W, 0)
        out.append(W)
    return out


@dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    rows: np.ndarray
    cols: np.ndarray
    w: np.ndarray


def served_requests(count: int, rate: float, lo: int = 32, hi: int = 4096, deg: float = 12.0,
                    seed: int = 6):
    """Open-loop Poisson stream of fp32 APSP requests sent as COO edge lists.

    Arrival gaps are exponential(1/rate); n is log-uniform in [lo, hi]; each
    pair i != j is an edge w.p. deg/n; weights are 10*(1-U) in (0, 10].
    """
    ss = np.random.SeedSequence(seed)
    g0 = np.random.Generator(np.random.PCG64(ss.spawn(1)[0]))
    gaps = g0.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i, child in enumerate(np.random.SeedSequence(seed + 1000).spawn(count)):
        g = np.random.Generator(np.random.PCG64(child))
        n = int(log_uniform_sizes(1, lo, hi, g)[0])
        r, c = _sparse_rows(g, n, min(1.0, deg / n))
        w = (10.0 * (1.0 - g.random(r.size))).astype(np.float32)
        reqs.append(Request(i, float(arrivals[i]), n, r.astype(np.int32), c.astype(np.int32), w))
    return reqs


# --------------------------------------------------------------------------
# Max-plus inputs (absent entries -INF).

def maxplus_digraph_i32(n: int, mean_degree: float, w_lo: int, w_hi: int, seed) -> np.ndarray:
    """Directed graph as a max-plus matrix: each ordered pair (self loops
    included) is an edge with probability mean_degree / n, integer weights
    U{w_lo..w_hi}; absent = -INF.  Cycles of every length occur."""
    g = rng(seed)
    A = np.full((n, n), I32_NINF, np.int32)
    mask = g.random((n, n)) < mean_degree / n
    A[mask] = g.integers(w_lo, w_hi, mask.sum(), endpoint=True)
    return A


def precedence_dag_f32(n: int, mean_degree: float, seed) -> np.ndarray:
    """Precedence DAG of a schedule as a max-plus matrix: edge i -> j only for
    i < j in a random topological order, with probability mean_degree / n,
    durations uniform in (0, 10]; absent = -inf."""
    g = rng(seed)
    perm = g.permutation(n)
    mask = np.triu(g.random((n, n)) < mean_degree / n, 1)
    A = np.where(mask, 10.0 * (1.0 - g.random((n, n))), -np.inf).astype(np.float32)
    return A[np.ix_(perm, perm)]
