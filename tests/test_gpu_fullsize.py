"""Parity at the full benchmark sizes, in the launch configuration the
benchmark times.  The oracle cannot redo these products in seconds, so it
checks sampled outputs one row at a time (8192^3 GEMM), or properties that
hold at any size plus single-source references (n=16384 APSP)."""
import numpy as np
import pytest

import oracle
from paper_1701_04733_amd import workloads as wl

pytestmark = pytest.mark.gpu

SEED_A, SEED_B = 2, 3


def _bits(x):
    x = np.ascontiguousarray(x).copy()
    if x.dtype == np.float32:
        x[x == 0] = 0.0
    return x.view(np.uint32)


@pytest.mark.parametrize("dt", ["f32", "i32"])
@pytest.mark.parametrize("sr", ["min", "max"])
def test_gemm_8192_sampled_rows(dev, sr, dt):
    import torch

    import paper_1701_04733_amd as btas
    n = 8192
    A = wl.gemm_operand((n, n), dt, sr, seed=SEED_A)
    B = wl.gemm_operand((n, n), dt, sr, seed=SEED_B)
    C = wl.semiring_identity_matrix((n, n), dt, sr)
    tA, tB, tC = (torch.from_numpy(x).to(dev) for x in (A, B, C))
    btas.tropical_gemm(tA, tB, tC, semiring=sr)
    rows = [0, 1, 127, 128, 4095, 5000, 8190, 8191]
    got = tC[rows].cpu().numpy()
    want = oracle.gemm(sr, A[rows], B, C[rows])
    for i, r in enumerate(rows):
        assert np.array_equal(_bits(got[i]), _bits(want[i])), f"row {r}"
    # a column sample too (transposes the roles of the tiles)
    cols = [0, 4097, 8191]
    gotc = tC[:, cols].cpu().numpy()
    sample_rows = np.arange(0, n, 97)
    for j, c in enumerate(cols):
        want = oracle.gemm(sr, A[sample_rows], B[:, c:c + 1].copy(), C[sample_rows, c:c + 1].copy())[:, 0]
        assert np.array_equal(_bits(gotc[sample_rows, j]), _bits(want)), f"col {c}"


def test_apsp_16384_f32_properties(dev):
    """n=16384, mean out-degree 16, exponential(1) weights, early exit, on the
    path the benchmark times (sparse first squarings, then 128x128 tiles).

    Checked three ways: (1) 64 sampled sources against binary64 Dijkstra
    within the (1 -+ u)^T rounding bound of a depth-T tree of binary32 adds;
    (2) the same squarings chained through the GEMM entry point
    (E = D (+) D (.) D, out of place) give the same bits; (3) the last
    squaring of that chain, D_s = D_{s-1} (+) D_{s-1} (.) D_{s-1}, equals the
    oracle's product bit for bit on 16 sampled rows, whatever s is."""
    import torch
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra

    import paper_1701_04733_amd as btas
    n = 16384
    r, c, w = wl.sparse_digraph_f32_exp(n, 16.0, seed=4)
    W = wl.coo_to_dense_f32(n, r, c, w)
    tW = torch.from_numpy(W).to(dev)
    del W
    D, steps, _ = btas.apsp(tW, early_exit=True)
    T = oracle.apsp_steps(n)
    assert 1 <= steps <= T
    assert (torch.diagonal(D) == 0).all()
    g = np.random.default_rng(40)
    sources = sorted({0, n - 1, *g.choice(n, size=62, replace=False).tolist()})
    assert len(sources) == 64
    rows = D[sources].cpu().numpy().astype(np.float64)
    G = csr_matrix((w.astype(np.float64), (r, c)), shape=(n, n))
    exact = dijkstra(G, directed=True, indices=sources)
    fin = np.isfinite(exact)
    assert np.array_equal(fin, np.isfinite(rows))
    u = 2.0 ** -24
    assert np.all(rows[fin] <= exact[fin] * (1 + u) ** T)
    assert np.all(rows[fin] >= exact[fin] * (1 - u) ** T)
    del rows, exact, G
    # (2) the squarings one product call at a time (W has a zero diagonal,
    # so D_0 = I (+) W = W); keep D_{s-1} on the host for (3)
    prev, Dh = tW, None
    for t in range(steps):
        cur = prev.clone()
        btas.tropical_gemm(prev, prev, cur, semiring="min")
        if t == steps - 1:
            Dh = prev.cpu().numpy()
        prev = cur
    assert torch.equal(prev.view(torch.int32), D.view(torch.int32)), "chained products != apsp"
    del prev, cur
    # (3) the last squaring against the oracle on sampled rows
    pick = [0, 1, 127, 128, 4096, 8191, 12000, n - 1] + g.choice(n, size=8, replace=False).tolist()
    want = oracle.gemm("min", Dh[pick], Dh, Dh[pick])
    got = D[pick].cpu().numpy()
    assert np.array_equal(_bits(got), _bits(want))
    # early exit fired before T: D is a fixpoint of one more squaring
    if steps < T:
        assert np.array_equal(_bits(Dh[pick]), _bits(got))


def test_apsp_large_generator_4096_golden(dev):
    """The APSP-large generator at n=4096 (fp32, out-degree 16, exponential(1)
    weights, seed 4) with early exit takes the code path of the n=16384
    workload (sparse first squarings, then full 128x128 tiles with the
    changed flag); the whole D equals the oracle's (digest written by
    tests/golden/make_golden.py --large), and so does the dense-only path."""
    import hashlib
    import json
    import os

    import torch

    import paper_1701_04733_amd as btas
    with open(os.path.join(os.path.dirname(__file__), "golden", "apsp_large4096.json")) as f:
        gold = json.load(f)["apsp_large_f32_n4096_seed4_early_exit"]
    W = wl.apsp_large_f32(4096, 16.0, seed=4)
    assert hashlib.sha256(W.tobytes()).hexdigest() == gold["input_sha256"]
    tW = torch.from_numpy(W).to(dev)
    for sparse in (None, "0"):
        prev = os.environ.get("BTAS_SPARSE_STEPS")
        if sparse is not None:
            os.environ["BTAS_SPARSE_STEPS"] = sparse
        try:
            D, steps, _ = btas.apsp(tW, early_exit=True)
        finally:
            if sparse is not None:
                if prev is None:
                    del os.environ["BTAS_SPARSE_STEPS"]
                else:
                    os.environ["BTAS_SPARSE_STEPS"] = prev
        Dn = _bits(D.cpu().numpy())
        assert steps == gold["steps"], f"sparse={sparse}"
        assert hashlib.sha256(Dn.tobytes()).hexdigest() == gold["D_sha256"], f"sparse={sparse}"


@pytest.mark.parametrize("dt", ["f32", "i32"])
def test_gemm_output_beyond_2_31_elements(dev, dt):
    """An output of 46 341 x 46 341 > 2^31 elements (8.6 GB): element offsets
    and tile indices need 64-bit arithmetic.  k = 16 keeps the product short;
    sampled rows at both ends and columns near the last tile are checked
    against the oracle."""
    import torch

    import paper_1701_04733_amd as btas
    n, k = 46341, 16
    A = wl.gemm_operand((n, k), dt, "min", seed=11)
    B = wl.gemm_operand((k, n), dt, "min", seed=12)
    tA, tB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    absent = float("inf") if dt == "f32" else wl.I32_INF
    tC = torch.full((n, n), absent, dtype=tA.dtype, device=dev)
    btas.tropical_gemm(tA, tB, tC, semiring="min")
    rows = [0, 1, 23170, n - 2, n - 1]
    got = tC[rows].cpu().numpy()
    C0 = wl.semiring_identity_matrix((len(rows), n), dt, "min")
    want = oracle.gemm("min", A[rows], B, C0)
    for i, r in enumerate(rows):
        assert np.array_equal(_bits(got[i]), _bits(want[i])), f"row {r}"
    cols = [0, n - 1]
    gotc = tC[:, cols].cpu().numpy()
    Cc = wl.semiring_identity_matrix((n, len(cols)), dt, "min")
    wantc = oracle.gemm("min", A, np.ascontiguousarray(B[:, cols]), Cc)
    assert np.array_equal(_bits(gotc), _bits(wantc))
    del tC
    torch.cuda.empty_cache()
