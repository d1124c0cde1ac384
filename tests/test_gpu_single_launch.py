"""APSP as one cooperative launch (BTAS_APSP_SINGLE_LAUNCH): bit-identical to
the oracle and to the per-squaring path, with early exit decided on the
device, in place and with padded leading dimensions, and stable over many
launches in a row.  Sizes up to about 350 take the tagged mode (one
workgroup per tile, squarings ordered by the launch/step tags of the data
words, early exit from per-workgroup change words one squaring late); larger
ones the device-wide barrier, whose arrival words alternate between two sets
and carry the launch's epoch.  Launches of both kinds and of many sizes
follow each other on one handle."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1701_04733_amd import workloads as wl

pytestmark = pytest.mark.gpu

DT = ["i32", "f32"]


def _bits(x):
    x = np.ascontiguousarray(x).copy()
    if x.dtype == np.float32:
        x[x == 0] = 0.0
    return x.view(np.uint32)


def _graph(dt, n, seed, deg=3.0):
    Wi = wl.er_digraph_i32(n, min(1.0, deg / max(n, 1)), 1, 1000, seed=seed)
    if dt == "i32":
        return Wi
    g = wl.rng(seed + 1)
    W = np.where(Wi == wl.I32_INF, np.inf, g.exponential(1.0, (n, n))).astype(np.float32)
    np.fill_diagonal(W, 0)
    return W


def _dev(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 17, 100, 255, 256, 300, 500])
def test_single_launch_matches_oracle(dev, dt, n):
    import paper_1701_04733_amd as btas
    W = _graph(dt, n, seed=1000 + n)
    want, wsteps, _ = oracle.apsp(W)
    D, steps, _ = btas.apsp(_dev(W, dev), single_launch=True)
    assert steps == wsteps
    assert np.array_equal(_bits(D.cpu().numpy()), _bits(want)), f"{dt} n={n}"
    want_e, wsteps_e, _ = oracle.apsp(W, early_exit=True)
    D, steps, _ = btas.apsp(_dev(W, dev), single_launch=True, early_exit=True)
    assert steps == wsteps_e
    assert np.array_equal(_bits(D.cpu().numpy()), _bits(want_e)), f"{dt} n={n} early exit"


def test_single_launch_small_config_golden(dev):
    """n=256 ER digraph (p=0.05, weights U{1..100}, seed 1), T=8 squarings."""
    import paper_1701_04733_amd as btas
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "apsp_er256.json")))
    W = wl.er_digraph_i32(256, 0.05, 1, 100, seed=1)
    D, steps, _ = btas.apsp(_dev(W, dev), single_launch=True)
    assert steps == 8
    assert hashlib.sha256(D.cpu().numpy().tobytes()).hexdigest() == gold["apsp_er256_i32_seed1"]["D_sha256"]
    D2, steps2, _ = btas.apsp(_dev(W, dev), single_launch=True, early_exit=True)
    assert steps2 == gold["apsp_er256_i32_seed1_early_exit"]["steps"]
    assert hashlib.sha256(D2.cpu().numpy().tobytes()).hexdigest() == gold["apsp_er256_i32_seed1"]["D_sha256"]


@pytest.mark.parametrize("dt", DT)
def test_single_launch_in_place_padded_and_plain_path(dev, dt):
    import torch

    import paper_1701_04733_amd as btas
    for n in (133, 100):                                     # T = 8 (even), 7 (odd)
        W = _graph(dt, n, seed=77 + n, deg=5.0)
        want, _, _ = oracle.apsp(W)
        t = _dev(W, dev)
        plain, _, _ = btas.apsp(t)
        btas.apsp(t, out=t, single_launch=True)              # in place
        assert np.array_equal(_bits(t.cpu().numpy()), _bits(want)), f"in place n={n}"
        assert torch.equal(t, plain)
        big = torch.full((n, n + 5), 7, dtype=t.dtype, device=dev)
        big[:, :n] = _dev(W, dev)
        out = torch.zeros((n + 1, n + 3), dtype=t.dtype, device=dev)
        btas.apsp(big[:, :n], out=out[:n, :n], single_launch=True, early_exit=True)
        assert np.array_equal(_bits(out.cpu().numpy()[:n, :n]), _bits(want)), f"padded n={n}"
        assert (out[n, :] == 0).all() and (out[:, n:] == 0).all()   # nothing outside D written
        assert (big[:, n:] == 7).all()


def test_single_launch_many_in_a_row_and_async(dev):
    """Launches back to back without host synchronisation: every result is
    right, so the barrier state carries over correctly between launches."""
    import torch

    import paper_1701_04733_amd as btas
    Ws = [_graph("f32", 64 + 37 * i, seed=500 + i, deg=4.0) for i in range(12)]
    ts = [_dev(W, dev) for W in Ws]
    outs = [torch.empty_like(t) for t in ts]
    for _ in range(3):
        for t, o in zip(ts, outs):
            btas.apsp(t, out=o, single_launch=True, early_exit=True, return_steps=False)
    torch.cuda.synchronize()
    for W, o in zip(Ws, outs):
        want, _, _ = oracle.apsp(W)
        assert np.array_equal(_bits(o.cpu().numpy()), _bits(want)), f"n={W.shape[0]}"


def test_single_launch_neg_cycle_large_n_and_errors(dev):
    import paper_1701_04733_amd as btas
    INF = wl.I32_INF
    W = np.array([[0, 1, INF], [-3, 0, INF], [INF, 2, 0]], np.int32)
    _, _, st = btas.apsp(_dev(W, dev), single_launch=True, check_neg_cycle=True)
    assert st == btas.WARN_NEG_CYCLE
    # n above the single-launch limit takes the per-squaring path, same bits
    W = _graph("i32", 600, seed=9)
    want, wsteps, _ = oracle.apsp(W)
    D, steps, _ = btas.apsp(_dev(W, dev), single_launch=True)
    assert steps == wsteps and np.array_equal(D.cpu().numpy(), want)
    with pytest.raises(btas.BtasError, match="INVALID_ARG"):
        btas.apsp(_dev(W[:10, :10], dev), single_launch=True, graph=True)


def test_single_launch_repeated_small_config(dev):
    """The n=256 workload solved 40 times back to back, alternating fixed T
    and early exit: every result and step count equals the oracle's, so every
    workgroup took the same early-exit decision in every launch."""
    import torch

    import paper_1701_04733_amd as btas
    W = wl.er_digraph_i32(256, 0.05, 1, 100, seed=1)
    want, wsteps, _ = oracle.apsp(W)
    _, wsteps_e, _ = oracle.apsp(W, early_exit=True)
    t = _dev(W, dev)
    outs = [torch.empty_like(t) for _ in range(40)]
    for i, o in enumerate(outs):
        btas.apsp(t, out=o, single_launch=True, early_exit=bool(i & 1), return_steps=False)
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert np.array_equal(o.cpu().numpy(), want), f"launch {i}"
    for ee, ws in ((False, wsteps), (True, wsteps_e)):
        _, steps, st = btas.apsp(t, single_launch=True, early_exit=ee)
        assert st == btas.OK and steps == ws


@pytest.mark.parametrize("return_steps", [False, True])
def test_single_launch_barrier_timeout_is_reported(dev, monkeypatch, return_steps):
    """A barrier wait that hits its bound invalidates D and is reported also
    when the caller does not read the step count: by the handle's next call
    and by synchronize().  BTAS_TEST_SPIN_LIMIT=-1 makes every wait report a
    timeout at once, so every kernel still runs to its end."""
    import torch

    import paper_1701_04733_amd as btas
    monkeypatch.setenv("BTAS_TEST_SPIN_LIMIT", "-1")
    h = btas.Handle(0)          # reads the bound at creation
    monkeypatch.delenv("BTAS_TEST_SPIN_LIMIT")
    try:
        h.bind_stream()
        W = _dev(_graph("i32", 200, seed=77), dev)
        if return_steps:
            with pytest.raises(btas.BtasError) as ei:
                btas.apsp(W, handle=h)          # n=200 takes the single launch by default
            assert ei.value.status == 5 and "timed out" in str(ei.value)
            h.synchronize()                     # reported once, not again
        else:
            _, steps, st = btas.apsp(W, handle=h, return_steps=False)
            assert steps is None and st == btas.OK
            with pytest.raises(btas.BtasError) as ei:
                h.synchronize()
            assert ei.value.status == 5 and "timed out" in str(ei.value)
            h.synchronize()
            # the next call of any entry point reports it when the caller
            # synchronised some other way
            btas.apsp(W, handle=h, return_steps=False)
            torch.cuda.synchronize()
            C = torch.full((4, 4), btas.I32_INF, dtype=torch.int32, device=dev)
            with pytest.raises(btas.BtasError) as ei:
                btas.tropical_gemm(C.clone(), C.clone(), C, handle=h)
            assert ei.value.status == 5
        # with the normal bound, a fresh handle solves the same graph
        ok = btas.Handle(0)
        ok.bind_stream()
        D, steps, _ = btas.apsp(W, handle=ok)
        want, wsteps, _ = oracle.apsp(W.cpu().numpy())
        assert steps == wsteps and np.array_equal(D.cpu().numpy(), want)
        ok.close()
    finally:
        h.close()


def _u16_graph(n, seed, wmax, deg=4.0, zero_frac=0.1):
    """int32 ER digraph with weights in [0, wmax] (some zero-weight edges)."""
    g = wl.rng(seed)
    W = np.full((n, n), wl.I32_INF, dtype=np.int32)
    mask = g.random((n, n)) < min(1.0, deg / max(n - 1, 1))
    w = g.integers(0, wmax, size=(n, n), endpoint=True).astype(np.int32)
    w[g.random((n, n)) < zero_frac] = 0
    W[mask] = w[mask]
    np.fill_diagonal(W, 0)
    return W


def _gate(n):
    return 65534 // (2 * (n - 1))


@pytest.mark.parametrize("early", [False, True])
@pytest.mark.parametrize("n", [65, 100, 129, 200, 255, 256, 301, 500])
def test_single_launch_packed16_matches_oracle(dev, n, early, monkeypatch):
    """With BTAS_U16=1, int32 graphs whose weights pass the 16-bit gate run the
    packed mode (v_pk_add_u16 clamp + v_pk_min_u16) and give the oracle's
    bits; without it the same call takes the int32 squarings, same bits."""
    import paper_1701_04733_amd as btas
    W = _u16_graph(n, 500 + n, _gate(n))
    want, wsteps, _ = oracle.apsp(W, early_exit=early)
    monkeypatch.setenv("BTAS_U16", "1")
    D, steps, _ = btas.apsp(_dev(W, dev), single_launch=True, early_exit=early)
    assert btas.apsp_last_packed16()
    assert steps == wsteps and np.array_equal(D.cpu().numpy(), want), f"n={n} early={early}"
    monkeypatch.delenv("BTAS_U16")
    D2, steps2, _ = btas.apsp(_dev(W, dev), single_launch=True, early_exit=early)
    assert not btas.apsp_last_packed16()
    assert steps2 == wsteps and np.array_equal(D2.cpu().numpy(), want)


@pytest.mark.parametrize("n", [80, 256])
def test_single_launch_packed16_sums_at_the_limit(dev, n, monkeypatch):
    """A directed cycle whose every edge weighs the gate's maximum: distances
    reach (n-1) * gate and sums of two reach 2 (n-1) gate <= 65534, the top
    of the 16-bit range below the absent value; plus one unreachable vertex
    (absent rows and columns)."""
    import paper_1701_04733_amd as btas
    g = _gate(n)
    W = np.full((n, n), wl.I32_INF, dtype=np.int32)
    m = n - 1                                  # vertex n-1 is isolated
    for i in range(m):
        W[i, (i + 1) % m] = g
    np.fill_diagonal(W, 0)
    monkeypatch.setenv("BTAS_U16", "1")
    want, wsteps, _ = oracle.apsp(W)
    assert want.max(where=want != wl.I32_INF, initial=0) == (m - 1) * g
    D, steps, _ = btas.apsp(_dev(W, dev), single_launch=True)
    assert btas.apsp_last_packed16()
    assert steps == wsteps and np.array_equal(D.cpu().numpy(), want)


@pytest.mark.parametrize("case", ["above_gate", "negative_edge", "negative_diagonal"])
def test_single_launch_packed16_gate_rejects(dev, case, monkeypatch):
    """One weight outside the gate keeps the whole graph on the int32
    squarings (decided on the device), with the oracle's bits."""
    import paper_1701_04733_amd as btas
    n = 200
    W = _u16_graph(n, 77, _gate(n))
    if case == "above_gate":
        W[5, 17] = _gate(n) + 1
    elif case == "negative_edge":
        W[5, 17] = -1
    else:
        W[9, 9] = -3
    monkeypatch.setenv("BTAS_U16", "1")
    want, wsteps, _ = oracle.apsp(W)
    D, steps, _ = btas.apsp(_dev(W, dev), single_launch=True)
    assert not btas.apsp_last_packed16()
    assert steps == wsteps and np.array_equal(D.cpu().numpy(), want)


def test_small_workload_packed16_opt_in(dev, monkeypatch):
    """The n=256 latency workload (weights U{1..100}) passes the gate
    (floor(65534/510) = 128): the 16-bit mode with BTAS_U16=1, the int32
    squarings by default, the oracle's bits either way."""
    import paper_1701_04733_amd as btas
    W = wl.er_digraph_i32(256, 0.05, 1, 100, seed=1)
    want, _, _ = oracle.apsp(W)
    D, steps, _ = btas.apsp(_dev(W, dev))
    assert not btas.apsp_last_packed16() and steps == 8
    assert np.array_equal(D.cpu().numpy(), want)
    monkeypatch.setenv("BTAS_U16", "1")
    D, steps, _ = btas.apsp(_dev(W, dev))
    assert btas.apsp_last_packed16() and steps == 8
    assert np.array_equal(D.cpu().numpy(), want)
