"""Batched APSP (one hipGraph launch for many graphs) against the oracle and
against the plain one-solve-per-call path: bit-identical results."""
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


def _mixed_graphs(dt, count, seed, lo=1, hi=300):
    g = wl.rng(seed)
    out = []
    for i in range(count):
        n = int(g.integers(lo, hi + 1))
        W = wl.er_digraph_i32(n, min(1.0, 4.0 / max(n, 1)), 1, 1000, seed=seed * 1000 + i)
        if dt == "f32":
            w2 = wl.rng(seed * 7 + i).exponential(1.0, (n, n))
            W = np.where(W == wl.I32_INF, np.inf, w2).astype(np.float32)
            np.fill_diagonal(W, 0)
        out.append(W)
    return out


@pytest.mark.parametrize("dt", ["i32", "f32"])
def test_batched_matches_oracle(dev, dt):
    import torch

    import paper_1701_04733_amd as btas
    Ws = _mixed_graphs(dt, 37, seed=3)
    Ws += [np.zeros((0, 0), Ws[0].dtype)]                    # an empty graph is allowed
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    runner = btas.BatchedAPSP(tW)
    Ds = runner.run()
    torch.cuda.synchronize()
    for W, D in zip(Ws, Ds):
        if W.shape[0] == 0:
            continue
        want, _, _ = oracle.apsp(W)
        assert np.array_equal(_bits(D.cpu().numpy()), _bits(want)), f"n={W.shape[0]}"
    # replay of the captured graph gives the same bits
    for D in Ds:
        D.fill_(0)
    Ds2 = runner.run()
    torch.cuda.synchronize()
    for W, D in zip(Ws, Ds2):
        if W.shape[0]:
            want, _, _ = oracle.apsp(W)
            assert np.array_equal(_bits(D.cpu().numpy()), _bits(want))
    info = runner.plan_info()
    assert info["launches"] >= 2


@pytest.mark.parametrize("tile", ["128", "64", "mixed", "w64", "wmix", "w64d"])
def test_batched_tile_shapes_same_bits(dev, tile, monkeypatch):
    """Every tile shape the autotuner may pick gives the same bits."""
    import torch

    import paper_1701_04733_amd as btas
    monkeypatch.setenv("BTAS_BATCHED_TILE", tile)
    h = btas.Handle(0)
    h.bind_stream()
    Ws = _mixed_graphs("i32", 12, seed=9, lo=60, hi=520)
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    r = btas.BatchedAPSP(tW, handle=h)
    Ds = r.run()
    torch.cuda.synchronize()
    for W, D in zip(Ws, Ds):
        want, _, _ = oracle.apsp(W)
        assert np.array_equal(D.cpu().numpy(), want)
    h.close()


@pytest.mark.parametrize("tile", [None, "w64d", "mixed"])
def test_batched_int32_storage_modes(dev, tile, monkeypatch):
    """int32 graphs whose squarings stay within +-(2^23-1) are stored and
    squared as binary32, the others as int32; one batch mixes both (and a
    graph that is wide only because of a negative diagonal entry), with the
    autotuned shapes and forced ones (the direct kernel's integer path)."""
    import torch

    import paper_1701_04733_amd as btas
    if tile is not None:
        monkeypatch.setenv("BTAS_BATCHED_TILE", tile)
    Ws = []
    for i in range(12):
        n = [40, 130, 257, 300][i % 4]
        hi = 1000 if i % 2 == 0 else (1 << 20)              # odd: 2^T * max|w| > 2^23 - 1
        Ws.append(wl.er_digraph_i32(n, min(1.0, 5.0 / n), 1, hi, seed=700 + i))
    W = wl.er_digraph_i32(90, 0.05, 1, 100, seed=799)
    W[3, 3] = -(1 << 17)                                   # D_33 = W_33 < 0: wide, negative cycle
    Ws.append(W)
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    h = btas.Handle(0)
    h.bind_stream()
    Ds = btas.apsp_batched(tW, handle=h)
    torch.cuda.synchronize()
    for i, (W, D) in enumerate(zip(Ws, Ds)):
        want, _, _ = oracle.apsp(W)
        assert np.array_equal(D.cpu().numpy(), want), f"graph {i} n={W.shape[0]}"
    h.close()


def test_batched_padded_views(dev):
    """W and D given as views with padded leading dimensions (16-byte rows):
    the copy passes take their vector path with ragged last quads, and
    nothing outside the n x n views is written."""
    import torch

    import paper_1701_04733_amd as btas
    Ws, tW, tD, bigD = [], [], [], []
    for i, n in enumerate((37, 64, 130, 255)):
        W = wl.er_digraph_i32(n, min(1.0, 6.0 / n), 1, 500, seed=900 + i)
        ld = (n + 3) // 4 * 4 + 4
        bw = torch.full((n, ld), -7, dtype=torch.int32, device=dev)
        bw[:, :n] = torch.from_numpy(W).to(dev)
        bd = torch.full((n + 1, ld), -9, dtype=torch.int32, device=dev)
        Ws.append(W)
        tW.append(bw[:, :n])
        tD.append(bd[:n, :n])
        bigD.append(bd)
    btas.apsp_batched(tW, tD)
    torch.cuda.synchronize()
    for W, bd in zip(Ws, bigD):
        n = W.shape[0]
        want, _, _ = oracle.apsp(W)
        got = bd.cpu().numpy()
        assert np.array_equal(got[:n, :n], want), f"n={n}"
        assert (got[:, n:] == -9).all() and (got[n, :] == -9).all(), f"n={n}: wrote outside D"


def test_batched_in_place_and_errors(dev):
    import torch

    import paper_1701_04733_amd as btas
    Ws = _mixed_graphs("i32", 5, seed=4, lo=2, hi=90)
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    btas.apsp_batched(tW, tW)                                    # D[i] is W[i]
    torch.cuda.synchronize()
    for W, D in zip(Ws, tW):
        want, _, _ = oracle.apsp(W)
        assert np.array_equal(D.cpu().numpy(), want)
    big = torch.zeros((10, 10), dtype=torch.int32, device=dev)
    with pytest.raises(btas.BtasError, match="ALIAS"):
        btas.apsp_batched([big[:5, :5].clone(), big[:5, :5].clone()], [big[:5, :5], big[2:7, 2:7]])


def test_batched_full_config_vs_plain_and_oracle(dev):
    """4096 graphs, n log-uniform in [16,512], p = 8/n, weights U{1..1000}:
    every result equals the plain per-graph path bit for bit, and a sample of
    graphs equals the oracle."""
    import torch

    import paper_1701_04733_amd as btas
    Ws = wl.batched_graphs_i32(count=4096, seed=5)
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    Ds = btas.apsp_batched(tW)
    plain = [btas.apsp(w, return_steps=False)[0] for w in tW]
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(Ds, plain)):
        assert torch.equal(a, b), f"graph {i} (n={Ws[i].shape[0]}) differs from the plain path"
    sample = list(range(0, 4096, 128)) + [int(np.argmax([w.shape[0] for w in Ws]))]
    for i in sample:
        want, _, _ = oracle.apsp(Ws[i])
        assert np.array_equal(Ds[i].cpu().numpy(), want), f"graph {i}"


def _convergence_mix(dt, seed):
    """Graphs that reach their fixpoint at different squarings: complete
    graphs (first squaring unchanged), long directed paths (need all T),
    sparse random graphs in between."""
    g = wl.rng(seed)
    Ws = _mixed_graphs(dt, 20, seed=seed, lo=2, hi=260)
    for n in (17, 64, 129):
        W = np.full((n, n), 5, np.int32)
        np.fill_diagonal(W, 0)
        Ws.append(W)
        P = np.full((n, n), wl.I32_INF, np.int32)
        np.fill_diagonal(P, 0)
        P[np.arange(n - 1), np.arange(1, n)] = g.integers(1, 9, n - 1)
        Ws.append(P)
    if dt == "f32":
        Ws = [w if w.dtype == np.float32 else
              np.where(w == wl.I32_INF, np.inf, w).astype(np.float32) for w in Ws]
    return Ws


@pytest.mark.parametrize("dt", ["i32", "f32"])
@pytest.mark.parametrize("tile", [None, "w64d", "128", "w64"])
def test_batched_early_exit_matches_oracle(dev, dt, tile, monkeypatch):
    """Early exit skips a graph's squarings after its fixpoint, on the
    device; every result equals the oracle (fixed T) bit for bit, also on
    replay, for each kernel family."""
    import torch

    import paper_1701_04733_amd as btas
    if tile is not None:
        monkeypatch.setenv("BTAS_BATCHED_TILE", tile)
    Ws = _convergence_mix(dt, seed=11)
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    runner = btas.BatchedAPSP(tW, early_exit=True)
    for rep in range(2):
        Ds = runner.run()
        torch.cuda.synchronize()
        for W, D in zip(Ws, Ds):
            want, _, _ = oracle.apsp(W)
            assert np.array_equal(_bits(D.cpu().numpy()), _bits(want)), f"rep {rep} n={W.shape[0]}"
        for D in Ds:
            D.fill_(0)


def test_batched_early_exit_full_config_equals_fixed(dev):
    """The 4096-graph workload with early exit gives the fixed-T bits."""
    import torch

    import paper_1701_04733_amd as btas
    Ws = wl.batched_graphs_i32(count=4096, seed=5)
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    fixed = btas.apsp_batched(tW)
    early = btas.apsp_batched(tW, early_exit=True)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(fixed, early)):
        assert torch.equal(a, b), f"graph {i} (n={Ws[i].shape[0]})"


@pytest.mark.parametrize("dt", ["i32", "f32"])
@pytest.mark.parametrize("early", [False, True])
def test_batched_small_graphs_in_lds(dev, dt, early, monkeypatch):
    """With BTAS_BATCH_LDS=1, graphs of at most 64 vertices are solved whole
    by one workgroup each, on a branch of the captured graph beside the
    squaring launches of the larger ones: the bits equal the oracle's and
    those of the default plan (small graphs inside the grid-wide launches); a
    batch of small graphs only (no grid-wide launch at all), in place, and
    replays of the captured graph give the same bits."""
    import torch

    import paper_1701_04733_amd as btas
    Ws = _mixed_graphs(dt, 40, seed=11, lo=1, hi=140)
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    monkeypatch.setenv("BTAS_BATCH_LDS", "1")
    h1 = btas.Handle(0)
    h1.bind_stream()
    D1 = btas.BatchedAPSP(tW, handle=h1, early_exit=early).run()
    monkeypatch.delenv("BTAS_BATCH_LDS")
    h0 = btas.Handle(0)
    h0.bind_stream()
    D0 = btas.BatchedAPSP(tW, handle=h0, early_exit=early).run()
    torch.cuda.synchronize()
    for W, a, b in zip(Ws, D1, D0):
        assert np.array_equal(_bits(a.cpu().numpy()), _bits(b.cpu().numpy())), f"n={W.shape[0]}"
        if W.shape[0] <= 64:
            want, _, _ = oracle.apsp(W, early_exit=early)
            assert np.array_equal(_bits(a.cpu().numpy()), _bits(want)), f"n={W.shape[0]}"
    # small graphs only, solved in place, replayed three times
    small = [w for w in Ws if w.shape[0] <= 64]
    tS = [torch.from_numpy(w).to(dev) for w in small]
    monkeypatch.setenv("BTAS_BATCH_LDS", "1")
    runner = btas.BatchedAPSP(tS, Ds=tS, handle=h1, early_exit=early)
    runner.run()                                   # plans with the LDS branch
    monkeypatch.delenv("BTAS_BATCH_LDS")
    for rep in range(3):
        for t, w in zip(tS, small):
            t.copy_(torch.from_numpy(w))
        runner.run()
        torch.cuda.synchronize()
        for t, w in zip(tS, small):
            want, _, _ = oracle.apsp(w, early_exit=early)
            assert np.array_equal(_bits(t.cpu().numpy()), _bits(want)), f"replay {rep} n={w.shape[0]}"
    # graphs needing no squaring only (n <= 2), inside the grid-wide path:
    # empty work lists
    tiny = [w for w in Ws if w.shape[0] <= 2] or [np.zeros((1, 1), Ws[0].dtype)]
    tT = [torch.from_numpy(w).to(dev) for w in tiny]
    DT = btas.BatchedAPSP(tT, handle=h0, early_exit=early).run()
    torch.cuda.synchronize()
    for w, d in zip(tiny, DT):
        want, _, _ = oracle.apsp(w)
        assert np.array_equal(_bits(d.cpu().numpy()), _bits(want))
    h0.close()
    h1.close()


@pytest.mark.parametrize("early", [False, True])
def test_batched_uncaptured_plan_same_bits(dev, early, monkeypatch):
    """BTAS_BATCH_GRAPH=0 issues the plan's launches in order on every call
    instead of replaying a captured graph: the same bits, call after call."""
    import torch

    import paper_1701_04733_amd as btas
    Ws = _mixed_graphs("i32", 30, seed=21, lo=1, hi=300)
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    want = [d.cpu().numpy() for d in btas.BatchedAPSP(tW, early_exit=early).run()]
    monkeypatch.setenv("BTAS_BATCH_GRAPH", "0")
    h = btas.Handle(0)
    h.bind_stream()
    r = btas.BatchedAPSP(tW, handle=h, early_exit=early)
    for _ in range(2):
        for D in r.Ds:
            D.fill_(0)
        Ds = r.run()
        torch.cuda.synchronize()
        for a, b in zip(Ds, want):
            assert np.array_equal(_bits(a.cpu().numpy()), _bits(b))
    h.close()


@pytest.mark.parametrize("early", [False, True])
def test_batched_one_or_two_small_graphs(dev, early):
    """A batch of one or two graphs of n <= 352 is solved by one single launch
    per graph: the oracle's bits and step semantics (early exit included), in
    place; with an earlier output overlapping a later input (allowed: the
    batched contract reads every W first) or a larger graph, the batched plan
    runs instead, with the same bits."""
    import torch

    import paper_1701_04733_amd as btas
    kinds = [("i32", (256,)), ("f32", (100, 300)), ("i32", (352, 17))]
    for dt, ns in kinds:
        Ws = [_mixed_graphs(dt, 1, seed=60 + n, lo=n, hi=n)[0] for n in ns]
        tW = [torch.from_numpy(w).to(dev) for w in Ws]
        Ds = btas.apsp_batched(tW, early_exit=early)
        torch.cuda.synchronize()
        for W, D in zip(Ws, Ds):
            want, _, _ = oracle.apsp(W, early_exit=early)
            assert np.array_equal(_bits(D.cpu().numpy()), _bits(want)), f"{dt} n={W.shape[0]}"
        btas.apsp_batched(tW, tW, early_exit=early)           # in place
        torch.cuda.synchronize()
        for W, D in zip(Ws, tW):
            want, _, _ = oracle.apsp(W)
            assert np.array_equal(_bits(D.cpu().numpy()), _bits(want)), f"{dt} n={W.shape[0]} in place"
    # graph 0's output is graph 1's input buffer: every W must be read first
    W0 = _mixed_graphs("i32", 1, seed=71, lo=200, hi=200)[0]
    W1 = _mixed_graphs("i32", 1, seed=72, lo=200, hi=200)[0]
    t0, t1 = torch.from_numpy(W0).to(dev), torch.from_numpy(W1).to(dev)
    out1 = torch.empty_like(t1)
    btas.apsp_batched([t0, t1], [t1, out1], early_exit=early)
    torch.cuda.synchronize()
    assert np.array_equal(t1.cpu().numpy(), oracle.apsp(W0)[0])
    assert np.array_equal(out1.cpu().numpy(), oracle.apsp(W1)[0])
    # above the single-launch size: the plan
    Ws = [_mixed_graphs("i32", 1, seed=73, lo=400, hi=400)[0], W0]
    Ds = btas.apsp_batched([torch.from_numpy(w).to(dev) for w in Ws], early_exit=early)
    torch.cuda.synchronize()
    for W, D in zip(Ws, Ds):
        assert np.array_equal(D.cpu().numpy(), oracle.apsp(W)[0])
