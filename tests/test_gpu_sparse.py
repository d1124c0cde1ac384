"""Sparse-aware squarings (early-exit APSP): while the distance matrix is
sparse, a squaring runs as a row-by-row sparse product.  Forced on at small
sizes it must match the oracle bit for bit (steps too), through the switch
to dense steps; the automatic choice (n >= 4096) is checked against the
dense-only path and Dijkstra at n = 4096 and against the dense-only path at
n = 16384."""
import os

import numpy as np
import pytest

import oracle
from paper_1701_04733_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _bits(x):
    x = np.ascontiguousarray(x).copy()
    if x.dtype == np.float32:
        x[x == 0] = 0.0
    return x.view(np.uint32)


def _dev(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _graph(dt, n, seed, deg):
    if dt == "i32":
        return wl.er_digraph_i32(n, min(1.0, deg / max(n, 1)), 1, 1000, seed=seed)
    r, c, w = wl.sparse_digraph_f32_exp(n, deg, seed=seed)
    return wl.coo_to_dense_f32(n, r, c, w)


class _Env:
    def __init__(self, value):
        self.value = value

    def __enter__(self):
        self.old = os.environ.get("BTAS_SPARSE_STEPS")
        os.environ["BTAS_SPARSE_STEPS"] = self.value

    def __exit__(self, *exc):
        if self.old is None:
            del os.environ["BTAS_SPARSE_STEPS"]
        else:
            os.environ["BTAS_SPARSE_STEPS"] = self.old


@pytest.mark.parametrize("dt", ["i32", "f32"])
@pytest.mark.parametrize("n,deg", [(1, 1.0), (2, 1.0), (5, 1.0), (65, 2.0), (200, 3.0), (513, 2.5),
                                   (1000, 1.5), (300, 80.0)])
def test_forced_sparse_steps_match_oracle(dev, dt, n, deg):
    """Sparse while at most n^2/8 entries are finite, then dense; the last
    case is dense from the first step."""
    import paper_1701_04733_amd as btas
    W = _graph(dt, n, seed=9100 + n, deg=deg)
    want, wsteps, _ = oracle.apsp(W, early_exit=True)
    with _Env("force"):
        D, steps, _ = btas.apsp(_dev(W, dev), early_exit=True)
    assert steps == wsteps
    assert np.array_equal(_bits(D.cpu().numpy()), _bits(want)), f"{dt} n={n}"


def test_forced_sparse_negative_weights_and_views(dev):
    """int32 weights of both signs on a DAG (no cycles), in place and with a
    padded leading dimension."""
    import torch

    import paper_1701_04733_amd as btas
    n = 180
    g = np.random.default_rng(5)
    W = np.full((n, n), wl.I32_INF, np.int32)
    np.fill_diagonal(W, 0)
    for _ in range(3 * n):
        i, j = sorted(g.integers(0, n, 2))
        if i != j:
            W[i, j] = g.integers(-50, 100)
    want, wsteps, _ = oracle.apsp(W, early_exit=True)
    with _Env("force"):
        t = _dev(W, dev)
        _, steps, _ = btas.apsp(t, out=t, early_exit=True)
        assert steps == wsteps and np.array_equal(t.cpu().numpy(), want)
        big = torch.full((n, n + 3), 5, dtype=torch.int32, device=dev)
        big[:, :n] = _dev(W, dev)
        out = torch.zeros((n, n + 7), dtype=torch.int32, device=dev)
        btas.apsp(big[:, :n], out=out[:, :n], early_exit=True)
        assert np.array_equal(out[:, :n].cpu().numpy(), want)
        assert (out[:, n:] == 0).all() and (big[:, n:] == 5).all()


@pytest.mark.parametrize("dt", ["i32", "f32"])
def test_forced_sparse_1024_matches_oracle(dev, dt):
    import paper_1701_04733_amd as btas
    W = _graph(dt, 1024, seed=77, deg=6.0)
    want, wsteps, _ = oracle.apsp(W, early_exit=True)
    with _Env("force"):
        D, steps, _ = btas.apsp(_dev(W, dev), early_exit=True)
    assert steps == wsteps
    assert np.array_equal(_bits(D.cpu().numpy()), _bits(want))


@pytest.mark.parametrize("dt", ["i32", "f32"])
def test_auto_sparse_4096_equals_dense_path_and_dijkstra(dev, dt):
    """n = 4096 (the smallest size the automatic choice considers): same bits
    and steps as dense steps only; sampled rows equal fp64 Dijkstra (int32:
    exactly; fp32: within the rounding bound of T squarings)."""
    from scipy.sparse.csgraph import dijkstra

    import paper_1701_04733_amd as btas
    n = 4096
    W = _graph(dt, n, seed=4096, deg=8.0)
    t = _dev(W, dev)
    D1, s1, _ = btas.apsp(t, early_exit=True)
    with _Env("0"):
        D2, s2, _ = btas.apsp(t, early_exit=True)
    assert s1 == s2
    assert np.array_equal(_bits(D1.cpu().numpy()), _bits(D2.cpu().numpy()))
    src = [0, 1, 2047, 4095]
    Wf = W.astype(np.float64)
    Wf[(W == wl.I32_INF) if dt == "i32" else ~np.isfinite(W)] = np.inf
    np.fill_diagonal(Wf, np.inf)
    from scipy.sparse.csgraph import csgraph_from_dense
    exact = dijkstra(csgraph_from_dense(Wf, null_value=np.inf), directed=True, indices=src)
    got = D1[src].cpu().numpy().astype(np.float64)
    if dt == "i32":
        got[got == wl.I32_INF] = np.inf
        assert np.array_equal(got, exact)
    else:
        fin = np.isfinite(exact)
        assert np.array_equal(fin, np.isfinite(got))
        T = oracle.apsp_steps(n)
        u = 2.0 ** -24
        assert np.all(got[fin] <= exact[fin] * (1 + u) ** T)
        assert np.all(got[fin] >= exact[fin] * (1 - u) ** T)


def test_auto_sparse_16384_equals_dense_path(dev):
    """The n=16384 benchmark graph: the default early-exit solve (sparse
    first squarings) gives the same bits and steps as dense steps only."""
    import torch

    import paper_1701_04733_amd as btas
    n = 16384
    W = torch.from_numpy(wl.apsp_large_f32(n, 16.0, seed=4)).to(dev)
    D1, s1, _ = btas.apsp(W, early_exit=True)
    with _Env("0"):
        D2, s2, _ = btas.apsp(W, early_exit=True)
    assert s1 == s2
    assert torch.equal(D1, D2)
    del D1, D2, W
    torch.cuda.empty_cache()
