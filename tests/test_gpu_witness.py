"""Witnesses on the GPU: the argmin-carrying tropical product and successor
matrices, bit-exact against the oracle (values and indices) on tie-heavy
inputs across ragged tile edges, leading-dimension views and both
semirings; successor walks checked against Dijkstra up to n=16384."""
import numpy as np
import pytest

import oracle
from oracle import INF32, NINF32
from paper_1701_04733_amd import workloads as wl

pytestmark = pytest.mark.gpu

SR = ["min", "max"]
DT = ["i32", "f32"]


def _bits(x):
    x = np.ascontiguousarray(x).copy()
    if x.dtype == np.float32:
        x[x == 0] = 0.0
    return x.view(np.uint32)


def _dev(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _absent(dt, sr):
    if dt == "i32":
        return INF32 if sr == "min" else NINF32
    return np.float32(np.inf if sr == "min" else -np.inf)


def _tie_heavy(dt, sr, shape, seed, absent_frac=0.15, spread=4):
    g = np.random.default_rng(seed)
    if dt == "i32":
        X = g.integers(-spread, spread + 1, shape).astype(np.int32)
    else:
        X = (g.integers(-2 * spread, 2 * spread + 1, shape) * 0.25).astype(np.float32)
    X[g.random(shape) < absent_frac] = _absent(dt, sr)
    return X


def _wide(dt, sr, shape, seed, absent_frac=0.1):
    """The product benchmark's value distribution: few ties."""
    g = np.random.default_rng(seed)
    if dt == "i32":
        X = g.integers(0, 10 ** 6, shape, endpoint=True).astype(np.int32)
    else:
        X = g.random(shape, dtype=np.float32)
    X[g.random(shape) < absent_frac] = _absent(dt, sr)
    return X


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 7, 3), (64, 64, 16), (65, 63, 17),
                                   (130, 200, 257), (256, 192, 300)])
def test_gemm_witness_matches_oracle(dev, sr, dt, shape):
    import paper_1701_04733_amd as btas
    m, n, k = shape
    for gen in (_tie_heavy, _wide):
        A = gen(dt, sr, (m, k), 1)
        B = gen(dt, sr, (k, n), 2)
        C = _tie_heavy(dt, sr, (m, n), 3, absent_frac=0.6, spread=12)
        K = np.random.default_rng(4).integers(-1, 1000, (m, n)).astype(np.int32)
        want_c, want_k = oracle.gemm_witness(sr, A, B, C, K)
        Cg, Kg = btas.tropical_gemm_witness(_dev(A, dev), _dev(B, dev), _dev(C, dev), _dev(K, dev),
                                            semiring=sr)
        assert np.array_equal(_bits(Cg.cpu().numpy()), _bits(want_c)), f"{gen.__name__} C"
        assert np.array_equal(Kg.cpu().numpy(), want_k), f"{gen.__name__} K"
        # the values are the value-only product's
        Cv = btas.tropical_gemm(_dev(A, dev), _dev(B, dev), _dev(C, dev), semiring=sr)
        assert np.array_equal(_bits(Cv.cpu().numpy()), _bits(Cg.cpu().numpy()))


@pytest.mark.parametrize("dt", DT)
def test_gemm_witness_views_and_errors(dev, dt):
    """Odd leading dimensions (the scalar staging path) and sub-matrix views;
    entries outside the views untouched; aliasing rejected."""
    import torch

    import paper_1701_04733_amd as btas
    m, n, k = 70, 90, 45
    A = _tie_heavy(dt, "min", (m, k), 5)
    B = _tie_heavy(dt, "min", (k, n), 6)
    C = np.full((m, n), _absent(dt, "min"), A.dtype)
    K = np.full((m, n), -1, np.int32)
    want_c, want_k = oracle.gemm_witness("min", A, B, C, K)
    Ab = torch.zeros((m, k + 3), dtype=_dev(A, dev).dtype, device=dev)
    Ab[:, :k] = _dev(A, dev)
    Bb = torch.zeros((k, n + 1), dtype=Ab.dtype, device=dev)
    Bb[:, :n] = _dev(B, dev)
    Cb = torch.full((m + 1, n + 5), 9, dtype=Ab.dtype, device=dev)
    Cb[:m, :n] = _dev(C, dev)
    Kb = torch.full((m, n + 2), -7, dtype=torch.int32, device=dev)
    Kb[:, :n] = -1
    btas.tropical_gemm_witness(Ab[:, :k], Bb[:, :n], Cb[:m, :n], Kb[:, :n])
    assert np.array_equal(_bits(Cb[:m, :n].cpu().numpy()), _bits(want_c))
    assert np.array_equal(Kb[:, :n].cpu().numpy(), want_k)
    assert (Cb[m, :] == 9).all() and (Cb[:, n:] == 9).all() and (Kb[:, n:] == -7).all()
    M = torch.zeros((8, 8), dtype=torch.int32, device=dev)
    with pytest.raises(btas.BtasError, match="ALIAS"):
        btas.tropical_gemm_witness(M, M, torch.zeros_like(M), M)


def _graph(dt, n, seed, deg=4.0):
    if dt == "i32":
        return wl.er_digraph_i32(n, min(1.0, deg / max(n, 1)), 1, 1000, seed=seed)
    r, c, w = wl.sparse_digraph_f32_exp(n, deg, seed=seed)
    return wl.coo_to_dense_f32(n, r, c, w)


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("n", [1, 2, 5, 63, 64, 65, 200, 257])
def test_successors_match_oracle(dev, dt, n):
    import paper_1701_04733_amd as btas
    W = _graph(dt, n, seed=7000 + n)
    D, _, _ = oracle.apsp(W)
    want = oracle.successors(W, D)
    Wg = _dev(W, dev)
    Dg, _, _ = btas.apsp(Wg)
    assert np.array_equal(_bits(Dg.cpu().numpy()), _bits(D))
    S = btas.apsp_successors(Wg, Dg)
    assert np.array_equal(S.cpu().numpy(), want)


def test_successors_after_floyd_warshall_and_views(dev):
    """int32: FW's distances are the squaring's, so are the successors; a
    padded output view leaves its margin alone; aliasing is rejected."""
    import torch

    import paper_1701_04733_amd as btas
    n = 300
    W = _graph("i32", n, seed=31, deg=6.0)
    want = oracle.successors(W, oracle.apsp(W)[0])
    Wg = _dev(W, dev)
    Dfw, _ = btas.floyd_warshall(Wg)
    Sb = torch.full((n + 2, n + 3), -9, dtype=torch.int32, device=dev)
    btas.apsp_successors(Wg, Dfw, out=Sb[:n, :n])
    assert np.array_equal(Sb[:n, :n].cpu().numpy(), want)
    assert (Sb[n:, :] == -9).all() and (Sb[:, n:] == -9).all()
    with pytest.raises(btas.BtasError, match="ALIAS"):
        btas.apsp_successors(Wg, Dfw, out=Wg)


def test_successors_walks_1000_i32(dev):
    """n = 1000, positive integer weights: every walk along S reaches its
    target with exactly the shortest length."""
    import paper_1701_04733_amd as btas
    n = 1000
    W = _graph("i32", n, seed=99, deg=8.0)
    Wg = _dev(W, dev)
    D, _ = btas.floyd_warshall(Wg)
    S = btas.apsp_successors(Wg, D).cpu().numpy()
    Dh = D.cpu().numpy().astype(np.int64)
    fin = Dh != INF32
    assert np.array_equal(S == -1, ~fin & ~np.eye(n, dtype=bool))
    # walk all pairs at once: cur[i, j] advances along S toward j
    cur = np.tile(np.arange(n)[:, None], (1, n))
    length = np.zeros((n, n), np.int64)
    cols = np.tile(np.arange(n), (n, 1))
    for _ in range(n):
        live = fin & (cur != cols)
        if not live.any():
            break
        nxt = np.where(live, S[cur, cols], cur)
        length += np.where(live, W[cur, nxt].astype(np.int64), 0)
        cur = nxt
    assert np.array_equal(cur[fin], cols[fin])
    assert np.array_equal(length[fin], Dh[fin])


def test_successors_16384_f32_sampled_walks(dev):
    """The n=16384 benchmark graph (mean out-degree 16, exponential(1)
    weights), distances by blocked Floyd-Warshall: from sampled sources every
    walk along S reaches its target, S_ij = -1 exactly where j is
    unreachable, and each walk is a real path (fp64 length >= the exact
    distance) whose length matches the distance to a relative 2^-12: each
    hop picks the best next vertex up to the rounding of a few binary32
    values, so the excess per hop is a few units of 2^-24."""
    import torch
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra

    import paper_1701_04733_amd as btas
    n = 16384
    r, c, w = wl.sparse_digraph_f32_exp(n, 16.0, seed=4)
    W = wl.coo_to_dense_f32(n, r, c, w)
    Wg = _dev(W, dev)
    D, _ = btas.floyd_warshall(Wg)
    S = btas.apsp_successors(Wg, D)
    torch.cuda.synchronize()
    assert torch.equal(torch.diagonal(S).cpu(), torch.arange(n, dtype=torch.int32))
    src = list(range(0, n, n // 16))
    Sh = S.cpu().numpy()
    Dh = D[src].cpu().numpy().astype(np.float64)
    del S, D
    torch.cuda.empty_cache()
    exact = dijkstra(csr_matrix((w.astype(np.float64), (r, c)), shape=(n, n)), directed=True,
                     indices=src)
    fin = np.isfinite(exact)
    assert np.array_equal(fin, np.isfinite(Dh))
    cols = np.arange(n)
    for row, s in enumerate(src):
        assert np.array_equal(Sh[s][~fin[row]], np.full((~fin[row]).sum(), -1, np.int32))
        cur = np.full(n, s)
        length = np.zeros(n)
        hops = np.zeros(n)
        for _ in range(n):
            live = fin[row] & (cur != cols)
            if not live.any():
                break
            nxt = np.where(live, Sh[cur, cols], cur)
            assert (nxt[live] >= 0).all()
            length += np.where(live, W[cur, nxt].astype(np.float64), 0.0)
            hops += live
            cur = nxt
        f = fin[row]
        assert np.array_equal(cur[f], cols[f])
        assert np.all(length[f] >= exact[row][f] * (1 - 1e-12))
        assert np.all(length[f] <= exact[row][f] * (1 + 2.0 ** -12) + 1e-300)


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("n", [5, 65, 300, 700])
def test_successors_sparse_and_dense_paths_match_oracle(dev, dt, n, monkeypatch):
    """Successors from W's edge lists (the default for n >= 256 while W has at
    most n^2/32 edges; forced here at every size) and from the dense witness
    product (BTAS_SPARSE_STEPS=0) both equal the oracle."""
    import paper_1701_04733_amd as btas
    W = _graph(dt, n, seed=8800 + n, deg=5.0)
    W[np.arange(n), np.arange(n)] = 0 if dt == "i32" else np.float32(0)
    if n > 2:
        W[1, 1] = 3 if dt == "i32" else np.float32(3)    # a self loop is not an edge to use
    D, _, _ = oracle.apsp(W)
    want = oracle.successors(W, D)
    Wg = _dev(W, dev)
    Dg, _, _ = btas.apsp(Wg)
    for mode in ("force", "0"):
        monkeypatch.setenv("BTAS_SPARSE_STEPS", mode)
        S = btas.apsp_successors(Wg, Dg)
        assert np.array_equal(S.cpu().numpy(), want), f"{dt} n={n} mode={mode}"
