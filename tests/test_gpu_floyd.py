"""Blocked Floyd-Warshall on the GPU: bit-exact against the oracle's blocked
order (pivot blocks of 64), for int32 (then also equal to repeated squaring)
and binary32, across ragged and full-block sizes, padded leading dimensions,
in place, and the full n=16384 benchmark graph by sampled exact references."""
import numpy as np
import pytest

import oracle
from paper_1701_04733_amd import workloads as wl

pytestmark = pytest.mark.gpu

BLOCK = 64


def _bits(x):
    x = np.ascontiguousarray(x).copy()
    if x.dtype == np.float32:
        x[x == 0] = 0.0
    return x.view(np.uint32)


def _graph(dt, n, seed, deg=4.0):
    if dt == "i32":
        return wl.er_digraph_i32(n, min(1.0, deg / max(n, 1)), 1, 1000, seed=seed)
    r, c, w = wl.sparse_digraph_f32_exp(n, deg, seed=seed)
    return wl.coo_to_dense_f32(n, r, c, w)


def _dev(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


@pytest.mark.parametrize("dt", ["i32", "f32"])
@pytest.mark.parametrize("n", [1, 2, 5, 63, 64, 65, 127, 128, 200, 256, 257, 320, 513])
def test_fw_matches_blocked_oracle(dev, dt, n):
    import paper_1701_04733_amd as btas
    W = _graph(dt, n, seed=4000 + n)
    want = oracle.floyd_warshall_blocked(W, BLOCK)
    D, st = btas.floyd_warshall(_dev(W, dev))
    assert st == btas.OK
    assert np.array_equal(_bits(D.cpu().numpy()), _bits(want)), f"{dt} n={n}"
    if dt == "i32":
        sq, _, _ = oracle.apsp(W)
        assert np.array_equal(D.cpu().numpy(), sq)


@pytest.mark.parametrize("dt", ["i32", "f32"])
def test_fw_in_place_padded_and_errors(dev, dt):
    import torch

    import paper_1701_04733_amd as btas
    for n in (100, 192):                                    # ragged, and full blocks
        W = _graph(dt, n, seed=77 + n, deg=6.0)
        want = oracle.floyd_warshall_blocked(W, BLOCK)
        t = _dev(W, dev)
        btas.floyd_warshall(t, out=t)
        assert np.array_equal(_bits(t.cpu().numpy()), _bits(want)), f"in place n={n}"
        big = torch.full((n, n + 4), 7, dtype=t.dtype, device=dev)
        big[:, :n] = _dev(W, dev)
        out = torch.zeros((n + 1, n + 8), dtype=t.dtype, device=dev)
        btas.floyd_warshall(big[:, :n], out=out[:n, :n])
        got = out.cpu().numpy()
        assert np.array_equal(_bits(got[:n, :n]), _bits(want)), f"padded n={n}"
        assert (got[n, :] == 0).all() and (got[:, n:] == 0).all()
        assert (big[:, n:] == 7).all()
    INF = wl.I32_INF
    Wn = np.array([[0, 1, INF], [-3, 0, INF], [INF, 2, 0]], np.int32)
    _, st = btas.floyd_warshall(_dev(Wn, dev), check_neg_cycle=True)
    assert st == btas.WARN_NEG_CYCLE
    M = torch.zeros((8, 9), dtype=torch.int32, device=dev)
    with pytest.raises(btas.BtasError, match="ALIAS"):
        btas.floyd_warshall(M[:, :8], out=M[:, 1:9])


def test_fw_f32_larger_vs_oracle(dev):
    """n = 1024 (16 pivot blocks, the direct-load phase 3) against the oracle."""
    import paper_1701_04733_amd as btas
    n = 1024
    W = _graph("f32", n, seed=11, deg=12.0)
    want = oracle.floyd_warshall_blocked(W, BLOCK)
    D, _ = btas.floyd_warshall(_dev(W, dev))
    assert np.array_equal(_bits(D.cpu().numpy()), _bits(want))


def test_fw_benchmark_generator_2048_bit_exact(dev):
    """The n=16384 benchmark graph's generator (mean out-degree 16,
    exponential(1) weights, seed 4) at n = 2048: every entry equals the
    blocked-FW oracle bit for bit, through the same kernels as n = 16384
    (n a multiple of 128: pivot pairs on the direct-load tiles)."""
    import paper_1701_04733_amd as btas
    n = 2048
    r, c, w = wl.sparse_digraph_f32_exp(n, 16.0, seed=4)
    W = wl.coo_to_dense_f32(n, r, c, w)
    want = oracle.floyd_warshall_blocked(W, BLOCK)
    D, st = btas.floyd_warshall(_dev(W, dev))
    assert st == btas.OK
    assert np.array_equal(_bits(D.cpu().numpy()), _bits(want))


@pytest.mark.parametrize("n", [384, 640, 1536])
def test_fw_groups_of_four_equal_pairs_and_oracle(dev, n):
    """fp32 with n a multiple of 128 can take pivot blocks in groups of four
    (one k=256 update per group; a last pair when n/64 is not a multiple of
    4: n = 384, 640), the default from n = 8192 on and forced here with
    BTAS_FW_GROUP=4: the same bits as pivot pairs (BTAS_FW_GROUP=2) and as
    the oracle's blocked order."""
    import os

    import paper_1701_04733_amd as btas
    r, c, w = wl.sparse_digraph_f32_exp(n, 12.0, seed=n)
    W = wl.coo_to_dense_f32(n, r, c, w)
    want = _bits(oracle.floyd_warshall_blocked(W, BLOCK))
    prev = os.environ.get("BTAS_FW_GROUP")
    got = {}
    try:
        for mode in ("4", "2"):
            os.environ["BTAS_FW_GROUP"] = mode
            D, st = btas.floyd_warshall(_dev(W, dev))
            assert st == btas.OK
            got[mode] = _bits(D.cpu().numpy())
    finally:
        if prev is None:
            del os.environ["BTAS_FW_GROUP"]
        else:
            os.environ["BTAS_FW_GROUP"] = prev
    assert np.array_equal(got["4"], want)
    assert np.array_equal(got["2"], want)
    if n == 384:
        # groups of four in place in a padded matrix (ld = n + 16)
        import torch
        big = torch.full((n, n + 16), 7.0, dtype=torch.float32, device=dev)
        big[:, :n] = _dev(W, dev)
        prev = os.environ.get("BTAS_FW_GROUP")
        os.environ["BTAS_FW_GROUP"] = "4"
        try:
            _, st = btas.floyd_warshall(big[:, :n], out=big[:, :n])
        finally:
            if prev is None:
                del os.environ["BTAS_FW_GROUP"]
            else:
                os.environ["BTAS_FW_GROUP"] = prev
        assert st == btas.OK
        assert np.array_equal(_bits(big[:, :n].cpu().numpy()), want)
        assert (big[:, n:] == 7.0).all()


def test_fw_16384_f32_sampled_sources(dev):
    """The n=16384 benchmark graph (mean out-degree 16, exponential(1)
    weights): the diagonal is 0 and rows from sampled sources equal fp64
    Dijkstra within the rounding bounds of non-negative sums: at most
    (1+u)^(h-1) above the exact distance for a shortest path of h edges, at
    least (1-u)^(n-2) below."""
    import torch
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra

    import paper_1701_04733_amd as btas
    n = 16384
    r, c, w = wl.sparse_digraph_f32_exp(n, 16.0, seed=4)
    W = wl.coo_to_dense_f32(n, r, c, w)
    D, _ = btas.floyd_warshall(_dev(W, dev))
    torch.cuda.synchronize()
    assert torch.all(torch.diagonal(D) == 0)
    src = list(range(0, n, n // 32))
    got = D[src].cpu().numpy().astype(np.float64)
    G = csr_matrix((w.astype(np.float64), (r, c)), shape=(n, n))
    exact, pred = dijkstra(G, directed=True, indices=src, return_predecessors=True)
    fin = np.isfinite(exact)
    assert np.array_equal(fin, np.isfinite(got))
    # hops h of each shortest path (from the predecessor trees): that path,
    # summed in any association, is within (1+u)^(h-1) of its exact length,
    # and the computed distance is at most that sum
    hops = np.zeros_like(exact)
    cur = np.tile(np.arange(n), (len(src), 1))
    rows = np.arange(len(src))[:, None]
    for _ in range(n):
        step = pred[rows, cur]
        live = step >= 0
        if not live.any():
            break
        hops += live
        cur = np.where(live, step, cur)
    u = 2.0 ** -24
    assert np.all(got[fin] <= exact[fin] * (1 + u) ** np.maximum(hops[fin] - 1, 0) + 1e-300)
    assert np.all(got[fin] >= exact[fin] * (1 - u) ** (n - 1) - 1e-300)
    del D
    torch.cuda.empty_cache()


def _fw_mixed(dt, seed):
    g = np.random.default_rng(seed)
    sizes = [0, 1, 2, 63, 64, 65, 128, 200, 300, 513] + list(g.integers(3, 260, 14))
    return [_graph(dt, int(n), seed=seed * 100 + i, deg=4.0) for i, n in enumerate(sizes)]


@pytest.mark.parametrize("dt", ["i32", "f32"])
def test_fw_batched_matches_oracle(dev, dt):
    """Many graphs of mixed sizes in one captured launch sequence: int32 equals
    the squaring oracle exactly, binary32 the blocked-FW oracle graph by graph,
    also on replay."""
    import torch

    import paper_1701_04733_amd as btas
    Ws = _fw_mixed(dt, seed=5)
    tW = [_dev(W, dev) for W in Ws]
    Ds = [torch.empty_like(t) for t in tW]
    for rep in range(2):
        btas.floyd_warshall_batched(tW, Ds)
        torch.cuda.synchronize()
        for W, D in zip(Ws, Ds):
            n = W.shape[0]
            if n == 0:
                continue
            want = oracle.apsp(W)[0] if dt == "i32" else oracle.floyd_warshall_blocked(W, BLOCK)
            assert np.array_equal(_bits(D.cpu().numpy()), _bits(want)), f"rep {rep} {dt} n={n}"
        for D in Ds:
            D.fill_(0)


@pytest.mark.parametrize("dt", ["i32", "f32"])
def test_fw_batched_aligned_rows(dev, dt):
    """Every leading dimension a multiple of 4 (16-byte rows): the tiles take
    vector loads; odd and even block counts, ragged last tiles."""
    import torch

    import paper_1701_04733_amd as btas
    sizes = [4, 64, 128, 132, 196, 260, 320, 384, 452, 512]
    Ws = [_graph(dt, n, seed=700 + n, deg=4.0) for n in sizes]
    tW = [_dev(W, dev) for W in Ws]
    Ds = btas.floyd_warshall_batched(tW)
    torch.cuda.synchronize()
    for W, D in zip(Ws, Ds):
        want = oracle.apsp(W)[0] if dt == "i32" else oracle.floyd_warshall_blocked(W, BLOCK)
        assert np.array_equal(_bits(D.cpu().numpy()), _bits(want)), f"{dt} n={W.shape[0]}"


def test_fw_batched_in_place_views_and_aliasing(dev):
    import torch

    import paper_1701_04733_amd as btas
    Ws = [_graph("f32", n, seed=40 + n) for n in (70, 130, 5)]
    want = [oracle.floyd_warshall_blocked(W, BLOCK) for W in Ws]
    tW = [_dev(W, dev) for W in Ws]
    btas.floyd_warshall_batched(tW, tW)                      # in place
    for t, w in zip(tW, want):
        assert np.array_equal(_bits(t.cpu().numpy()), _bits(w))
    # outputs as padded views of one buffer (ld 140, not a multiple of 4 apart)
    big = torch.full((300, 141), 3.0, device=dev)
    outs = [big[0:70, :70], big[70:200, :130], big[200:205, :5]]
    btas.floyd_warshall_batched([_dev(W, dev) for W in Ws], outs)
    for o, w in zip(outs, want):
        assert np.array_equal(_bits(o.cpu().numpy()), _bits(w))
    assert (big[:, 130:] == 3.0).all() and (big[205:, :] == 3.0).all()
    t = _dev(Ws[0], dev)
    with pytest.raises(btas.BtasError, match="ALIAS"):
        btas.floyd_warshall_batched([t, _dev(Ws[0], dev)], [torch.empty_like(t), t])


def test_fw_batched_full_config_equals_batched_squaring(dev):
    """The 4096-graph int32 workload: blocked FW gives the squaring's bits."""
    import torch

    import paper_1701_04733_amd as btas
    Ws = wl.batched_graphs_i32(count=4096, seed=5)
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    sq = btas.apsp_batched(tW, early_exit=True)
    fw = btas.floyd_warshall_batched(tW)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(sq, fw)):
        assert torch.equal(a, b), f"graph {i} (n={Ws[i].shape[0]})"
