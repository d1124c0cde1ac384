"""The APSP entry point that allocates nothing during the call
(btas_apsp_squaring_noalloc, workspace in a fixed per-GPU device array):
same bits and step counts as btas_apsp_squaring on every path it can take
(one workgroup in LDS, the cooperative single launch, one launch per
squaring with split-K, early exit read back per squaring), on two calls in a
row with the second smaller, at the size limit, and with size and flag
errors reported before anything runs."""
import numpy as np
import pytest

import oracle
from paper_1701_04733_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _graph(dt, n, seed):
    W = wl.er_digraph_i32(n, min(1.0, 4.0 / max(n, 1)), 1, 1000, seed=seed)
    if dt == "f32":
        g = wl.rng(seed + 7)
        W = np.where(W == wl.I32_INF, np.inf, g.exponential(1.0, (n, n))).astype(np.float32)
        np.fill_diagonal(W, 0)
    return W


def _bits(x):
    x = np.ascontiguousarray(x).copy()
    if x.dtype == np.float32:
        x[x == 0] = 0.0
    return x.view(np.uint32)


# (first n, second smaller n, flags): the pairs cover the one-workgroup LDS
# solve (n <= 64), the cooperative single launch (by default n <= 256 here
# and n <= 352 in the allocating call; up to 500 with single_launch), one
# launch per squaring with split-K partials in the fixed array, and early
# exit on either path.  Without the handle's tag
# buffer a single launch here waits on panel words (fixed T) or device-wide
# barriers (early exit) where the allocating call runs the tagged mode, so
# the first two pairs also compare those orderings.
CASES = [
    (200, 100, {}),
    (250, 129, {"early_exit": True}),
    (60, 21, {}),
    (420, 300, {"single_launch": True}),
    (1000, 700, {}),
    (900, 300, {"early_exit": True}),
    (2896, 513, {"early_exit": True}),
]


@pytest.mark.parametrize("dt", ["i32", "f32"])
@pytest.mark.parametrize("big,small,kw", CASES)
def test_noalloc_matches_allocating_entry_point(dev, dt, big, small, kw):
    import torch

    import paper_1701_04733_amd as btas
    h = btas.default_handle(0)
    for n, seed in ((big, 10 + big), (small, 20 + small)):
        W = torch.from_numpy(_graph(dt, n, seed)).to(dev)
        ref, rsteps, rst = btas.apsp(W, handle=h, **kw)
        out = torch.full_like(W, 7)                   # stale contents must not matter
        got, steps, st = btas.apsp_noalloc(W, out, handle=h, **kw)
        assert (steps, st) == (rsteps, rst), f"n={n}"
        assert torch.equal(got.view(torch.int32), ref.view(torch.int32)), f"{dt} n={n} {kw}"
        if n <= 300:
            want, wsteps, _ = oracle.apsp(W.cpu().numpy(), early_exit=kw.get("early_exit", False))
            assert wsteps == steps
            assert np.array_equal(_bits(got.cpu().numpy()), _bits(want))


def test_noalloc_allocates_nothing(dev):
    """A fresh handle solving through the fixed array leaves the device's free
    memory unchanged (the allocating entry point would grow an n x n
    partner and split-K partials on this handle)."""
    import torch

    import paper_1701_04733_amd as btas
    h = btas.Handle(0)
    try:
        h.bind_stream()
        Ws = [torch.from_numpy(_graph("f32", n, n)).to(dev) for n in (1500, 1000, 40)]
        outs = [torch.empty_like(w) for w in Ws]
        btas.apsp_noalloc(Ws[2], outs[2], handle=h)   # first use of the handle's kernels
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for w, o in zip(Ws, outs):
            btas.apsp_noalloc(w, o, handle=h)
            btas.apsp_noalloc(w, o, handle=h, early_exit=True)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        for w, o in zip(Ws, outs):
            ref, _, _ = btas.apsp(w)
            assert torch.equal(o.view(torch.int32), ref.view(torch.int32))
    finally:
        h.close()


def test_noalloc_rejects_before_launch(dev):
    import torch

    import paper_1701_04733_amd as btas
    n = btas.NOALLOC_MAX_N + 1
    W = torch.zeros((n, n), dtype=torch.float32, device=dev)
    out = torch.full_like(W, 3.0)
    with pytest.raises(btas.BtasError) as ei:
        btas.apsp_noalloc(W, out)
    assert ei.value.status == 1 and "n=2897" in str(ei.value)
    assert bool((out == 3.0).all())                    # nothing ran
    h = btas.default_handle(0)
    D = torch.empty((8, 8), dtype=torch.float32, device=dev)
    st = btas.lib().btas_apsp_squaring_noalloc(h.ptr, btas.FLOAT32, 8, btas._mat(D, "W")[0], 8,
                                                btas._mat(D, "D")[0], 8, btas.APSP_GRAPH, None)
    assert st == 1 and b"GRAPH" in btas.lib().btas_last_error(h.ptr)
