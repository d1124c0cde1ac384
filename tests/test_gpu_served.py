"""Served APSP: every request's result equals the oracle, and is the same bits
alone and in a mix of concurrently served requests; admission respects the
memory budget; early exit gives the fixed-T result."""
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


def _requests(count, seed, lo=32, hi=600):
    return wl.served_requests(count, rate=1000.0, lo=lo, hi=hi, seed=seed)


def _dense(req, dtype=np.float32):
    if dtype == np.float32:
        return wl.coo_to_dense_f32(req.n, req.rows, req.cols, req.w)
    W = np.full((req.n, req.n), wl.I32_INF, np.int32)
    W[req.rows, req.cols] = req.w
    np.fill_diagonal(W, 0)
    return W


def _max_overlap(spans):
    events = sorted([(a, 1) for a, _ in spans] + [(d, -1) for _, d in spans])
    live = peak = 0
    for _, e in events:
        live += e
        peak = max(peak, live)
    return peak


def _fetch(srv, rid, n, dev, dtype):
    import torch
    out = torch.empty((n, n), dtype=dtype, device=dev)
    srv.result_into(rid, out)
    return out.cpu().numpy()


@pytest.mark.parametrize("mode", ["continuous", "fifo"])
def test_served_mix_matches_oracle_and_alone(dev, mode):
    import torch

    import paper_1701_04733_amd as btas
    reqs = _requests(24, seed=31)
    with btas.Server("f32", budget_bytes=4 << 30, mode=mode, quantum_terms=2e8) as srv:
        ids = [srv.submit(r.n, r.rows, r.cols, r.w) for r in reqs]      # all at once: a mix
        mixed, spans = {}, []
        for r, rid in zip(reqs, ids):
            assert srv.wait(rid, timeout=120)
            mixed[r.rid] = _fetch(srv, rid, r.n, dev, torch.float32)
            assert srv.steps(rid) == oracle.apsp_steps(r.n)
            spans.append(srv.times(rid)[1:])
            srv.release(rid)
        st = srv.stats()
        assert st["active"] == 0 and st["pending"] == 0 and st["pool_used_bytes"] == 0
        # continuous batching: requests are resident and advancing together;
        # FIFO: one at a time
        assert (_max_overlap(spans) >= 2) == (mode == "continuous")
    with btas.Server("f32", budget_bytes=4 << 30, mode="continuous") as alone_srv:
        for r in reqs:
            rid = alone_srv.submit(r.n, r.rows, r.cols, r.w)
            assert alone_srv.wait(rid, timeout=120)
            alone = _fetch(alone_srv, rid, r.n, dev, torch.float32)
            alone_srv.release(rid)
            assert np.array_equal(_bits(alone), _bits(mixed[r.rid])), f"request {r.rid} n={r.n}"
            want, _, _ = oracle.apsp(_dense(r))
            assert np.array_equal(_bits(alone), _bits(want)), f"request {r.rid} vs oracle"


def test_served_early_exit_same_bits(dev):
    import torch

    import paper_1701_04733_amd as btas
    reqs = _requests(10, seed=32, lo=40, hi=400)
    with btas.Server("f32", budget_bytes=2 << 30) as srv:
        fixed = [srv.submit(r.n, r.rows, r.cols, r.w) for r in reqs]
        early = [srv.submit(r.n, r.rows, r.cols, r.w, early_exit=True) for r in reqs]
        for r, a, b in zip(reqs, fixed, early):
            assert srv.wait(a, 120) and srv.wait(b, 120)
            da = _fetch(srv, a, r.n, dev, torch.float32)
            db = _fetch(srv, b, r.n, dev, torch.float32)
            assert np.array_equal(_bits(da), _bits(db))
            want, wsteps, _ = oracle.apsp(_dense(r), early_exit=True)
            assert srv.steps(b) == wsteps <= srv.steps(a)
            srv.release(a)
            srv.release(b)


def test_served_budget_admission(dev):
    """A budget that holds only a couple of requests at a time still serves all
    of them, never exceeding the pool."""
    import torch

    import paper_1701_04733_amd as btas
    reqs = _requests(12, seed=33, lo=200, hi=300)
    per = max(2 * ((r.n + 3) // 4 * 4) * r.n * 4 for r in reqs)
    budget = 3 * per
    with btas.Server("f32", budget_bytes=budget) as srv:
        ids = [srv.submit(r.n, r.rows, r.cols, r.w) for r in reqs]
        spans = []
        for r, rid in zip(reqs, ids):
            assert srv.wait(rid, 120)
            got = _fetch(srv, rid, r.n, dev, torch.float32)
            spans.append(srv.times(rid)[1:])
            srv.release(rid)
            want, _, _ = oracle.apsp(_dense(r))
            assert np.array_equal(_bits(got), _bits(want))
        st = srv.stats()
        assert st["pool_peak_bytes"] <= st["pool_bytes"] <= budget + 256
        # no more requests were resident at once than the budget holds
        least = min(2 * ((r.n + 3) // 4 * 4) * r.n * 4 for r in reqs)
        assert _max_overlap(spans) <= budget // least


def test_served_int32_and_errors(dev):
    import torch

    import paper_1701_04733_amd as btas
    g = wl.rng(7)
    with btas.Server("i32", budget_bytes=1 << 30) as srv:
        for n in (1, 2, 3, 57, 130):
            r, c = wl._sparse_rows(g, n, min(1.0, 5.0 / max(n, 1)))
            w = g.integers(1, 100, size=r.size, endpoint=True).astype(np.int32)
            rid = srv.submit(n, r, c, w)
            assert srv.wait(rid, 60)
            got = _fetch(srv, rid, n, dev, torch.int32)
            W = np.full((n, n), wl.I32_INF, np.int32)
            W[r, c] = w
            np.fill_diagonal(W, 0)
            want, _, _ = oracle.apsp(W)
            assert np.array_equal(got, want)
            srv.release(rid)
        with pytest.raises(btas.BtasError, match="INVALID_ARG"):
            srv.submit(4, np.array([0, 4]), np.array([1, 2]), np.array([1, 1], np.int32))
        with pytest.raises(btas.BtasError, match="DOMAIN"):
            srv.submit(4, np.array([0]), np.array([1]), np.array([1 << 29], np.int32))


def test_served_many_requests_share_grouped_launches(dev):
    """Enough concurrent work to fill the GPU: squarings of different
    requests share grouped launches (fewer launches than squarings), and the
    results still equal the oracle."""
    import torch

    import paper_1701_04733_amd as btas
    reqs = _requests(40, seed=34, lo=300, hi=700)
    with btas.Server("f32", budget_bytes=8 << 30) as srv:
        ids = [srv.submit(r.n, r.rows, r.cols, r.w) for r in reqs]
        got = {}
        for r, rid in zip(reqs, ids):
            assert srv.wait(rid, 120)
            got[r.rid] = _fetch(srv, rid, r.n, dev, torch.float32)
            srv.release(rid)
        st = srv.stats()
        assert st["launches"] < sum(oracle.apsp_steps(r.n) for r in reqs)
    for r in reqs[:6]:
        want, _, _ = oracle.apsp(_dense(r))
        assert np.array_equal(_bits(got[r.rid]), _bits(want))


@pytest.mark.parametrize("cap", [None, "2e8"])
def test_served_two_lanes_large_and_small(dev, cap, monkeypatch):
    """Requests above and below the small-lane bound (1024 vertices) served
    together: both lanes are used, the shared pool is empty afterwards, and
    every result is the single-solve path's bits (also with the large lane's
    launches capped in size)."""
    import torch

    import paper_1701_04733_amd as btas
    if cap is not None:
        monkeypatch.setenv("BTAS_SERVE_LAUNCH_TERMS", cap)
    big = _requests(3, seed=35, lo=1100, hi=1400)
    small = _requests(10, seed=36, lo=32, hi=400)
    reqs = big + small
    with btas.Server("f32", budget_bytes=4 << 30) as srv:
        ids = [srv.submit(r.n, r.rows, r.cols, r.w) for r in reqs]
        assert {rid & 1 for rid in ids} == {0, 1}          # the lane is bit 0 of the id
        got = []
        for r, rid in zip(reqs, ids):
            assert srv.wait(rid, 120)
            got.append(_fetch(srv, rid, r.n, dev, torch.float32))
            assert srv.steps(rid) == oracle.apsp_steps(r.n)
            srv.release(rid)
        st = srv.stats()
        assert st["active"] == 0 and st["pending"] == 0 and st["pool_used_bytes"] == 0
    for r, g in zip(reqs, got):
        W = torch.from_numpy(_dense(r)).to(dev)
        want, _, _ = btas.apsp(W)
        assert np.array_equal(_bits(g), _bits(want.cpu().numpy())), f"request {r.rid} n={r.n}"


def test_served_early_exit_release_while_speculating(dev):
    """Early-exit requests are planned one squaring ahead; a request released
    as soon as it finishes may still have that squaring in flight, so its
    memory is handed back only when the launch retires.  Later requests
    reuse the pool and every result equals the oracle; the pool drains to
    zero once the engine is idle."""
    import time

    import torch

    import paper_1701_04733_amd as btas
    reqs = _requests(16, seed=37, lo=60, hi=500)
    per = max(2 * ((r.n + 3) // 4 * 4) * r.n * 4 + 3 * 4 * (r.rows.size + 64) for r in reqs)
    with btas.Server("f32", budget_bytes=3 * per, quantum_terms=2e7) as srv:
        ids = [srv.submit(r.n, r.rows, r.cols, r.w, early_exit=True) for r in reqs]
        for r, rid in zip(reqs, ids):
            assert srv.wait(rid, 120)
            got = _fetch(srv, rid, r.n, dev, torch.float32)
            steps = srv.steps(rid)
            srv.release(rid)                       # possibly before the last launch retired
            with pytest.raises(btas.BtasError):
                srv.release(rid)                   # released once only
            want, wsteps, _ = oracle.apsp(_dense(r), early_exit=True)
            assert steps == wsteps
            assert np.array_equal(_bits(got), _bits(want)), f"request {r.rid} n={r.n}"
        deadline = time.time() + 30
        while srv.stats()["pool_used_bytes"] != 0 and time.time() < deadline:
            time.sleep(0.01)
        st = srv.stats()
        assert st["pool_used_bytes"] == 0 and st["active"] == 0 and st["pending"] == 0


def test_served_small_lane_not_behind_large(dev):
    """A small request submitted right after several large ones, which need
    far more device time, completes while every large one is still running:
    the small lane does not wait for the large lane's squarings.  Ordering,
    not a time bound: the large requests take tens of milliseconds on the
    device, the small one a few launches."""
    import torch

    import paper_1701_04733_amd as btas
    big = _requests(3, seed=38, lo=3000, hi=3500)
    small = _requests(1, seed=39, lo=48, hi=64)[0]
    with btas.Server("f32", budget_bytes=8 << 30) as srv:
        bids = [srv.submit(r.n, r.rows, r.cols, r.w) for r in big]
        sid = srv.submit(small.n, small.rows, small.cols, small.w)
        assert sid & 1 == 1 and all(b & 1 == 0 for b in bids)
        assert srv.wait(sid, 120)
        done_small = srv.times(sid)[2]
        for b in bids:
            assert srv.wait(b, 120)
        assert all(srv.times(b)[2] > done_small for b in bids)
        got = _fetch(srv, sid, small.n, dev, torch.float32)
        want, _, _ = oracle.apsp(_dense(small))
        assert np.array_equal(_bits(got), _bits(want))
        # the first large request against the oracle as well (n >= 3000 would
        # take minutes on the host: compare its sampled rows with one more
        # squaring's fixpoint instead)
        r0 = big[0]
        D = _fetch(srv, bids[0], r0.n, dev, torch.float32)
        for b in bids:
            srv.release(b)
        srv.release(sid)
    W = _dense(r0)
    rows = [0, 1, r0.n // 2, r0.n - 1]
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    G = csr_matrix((r0.w.astype(np.float64), (r0.rows, r0.cols)), shape=(r0.n, r0.n))
    exact = dijkstra(G, directed=True, indices=rows)
    T = oracle.apsp_steps(r0.n)
    u = 2.0 ** -24
    fin = np.isfinite(exact)
    got = D[rows].astype(np.float64)
    assert np.array_equal(fin, np.isfinite(got))
    assert np.all(got[fin] <= exact[fin] * (1 + u) ** T) and np.all(got[fin] >= exact[fin] * (1 - u) ** T)
    del W
