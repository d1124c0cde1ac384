"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element on the same seeded inputs.  The bar is bit equality for
both int32 and float32 (each float32 term is one rounded add and min/max are
exact, so there is nothing for a tolerance to absorb); the only
normalisation is -0 -> +0 before comparing float bits.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1701_04733_amd import workloads as wl

pytestmark = pytest.mark.gpu

SR = ["min", "max"]
DT = ["i32", "f32"]


def torch_mod():
    import torch
    return torch


@pytest.fixture(scope="module")
def btas(dev):
    import paper_1701_04733_amd as b
    b.lib()
    return b


def to_dev(x, dev):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def to_np(t):
    torch = torch_mod()
    torch.cuda.synchronize()
    return t.cpu().numpy()


def bits(x):
    x = np.ascontiguousarray(x)
    if x.dtype == np.float32:
        y = x.copy()
        y[y == 0] = 0.0                                   # -0 -> +0
        return y.view(np.uint32)
    return x.view(np.uint32)


def assert_same(got, want, what=""):
    gb, wb = bits(got), bits(want)
    if not np.array_equal(gb, wb):
        bad = np.argwhere(gb != wb)
        i = tuple(bad[0])
        raise AssertionError(f"{what}: {len(bad)} mismatches; first at {i}: got {got[i]!r} want {want[i]!r}")


def operands(m, n, k, dt, sr, seed, frac=0.1, signed=False):
    gen = wl.signed_operand if signed else wl.gemm_operand
    A = gen((m, k), dt, sr, seed=seed, inf_frac=frac)
    B = gen((k, n), dt, sr, seed=seed + 1, inf_frac=frac)
    return A, B


SHAPES = [(1, 1, 1), (2, 3, 1), (3, 7, 2), (7, 31, 65), (31, 64, 127), (64, 64, 64),
          (65, 127, 129), (127, 129, 257), (129, 257, 31), (257, 65, 1000), (300, 290, 77),
          # few output tiles, long k: split-K chunks plus a ragged last chunk
          (64, 64, 4096), (100, 37, 1000), (17, 250, 777), (256, 256, 256)]


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("shape", SHAPES)
def test_gemm_shapes(btas, dev, sr, dt, shape):
    m, n, k = shape
    A, B = operands(m, n, k, dt, sr, seed=1000 + m + n + k, signed=True)
    C = wl.signed_operand((m, n), dt, sr, seed=7 + m, inf_frac=0.3)
    want = oracle.gemm(sr, A, B, C)
    Ct = to_dev(C, dev)
    btas.tropical_gemm(to_dev(A, dev), to_dev(B, dev), Ct, semiring=sr)
    assert_same(to_np(Ct), want, f"{sr}/{dt}/{shape}")


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("frac", [0.0, 0.1, 1.0])
def test_gemm_large_tiles_ragged(btas, dev, sr, dt, frac):
    """Shape large enough for the 128x128 tiling, with ragged m, n and k."""
    m, n, k = 2945, 2890, 133
    A, B = operands(m, n, k, dt, sr, seed=77, frac=frac)
    C = wl.semiring_identity_matrix((m, n), dt, sr)
    want = oracle.gemm(sr, A, B, C)
    Ct = to_dev(C, dev)
    btas.tropical_gemm(to_dev(A, dev), to_dev(B, dev), Ct, semiring=sr)
    assert_same(to_np(Ct), want, f"{sr}/{dt}/frac={frac}")


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("frac", [0.0, 0.1, 1.0])
def test_gemm_full_tiles_direct_lds_path(btas, dev, sr, frac):
    """fp32 shapes whose 128x128 tiles are all full (the direct global->LDS
    path), signed values, a C that is partly absent, padded leading
    dimensions, and the same product through a ragged shape (the staged
    path) for comparison."""
    torch = torch_mod()
    m, n, k = 3200, 2688, 96                       # 25 x 21 = 525 >= 512 tiles of 128 x 128
    A, B = operands(m, n, k, "f32", sr, seed=91, frac=frac, signed=True)
    C = wl.signed_operand((m, n), "f32", sr, seed=92, inf_frac=0.3)
    want = oracle.gemm(sr, A, B, C)
    Ap = torch.zeros((m, k + 4), dtype=torch.float32, device=dev)
    Ap[:, :k] = to_dev(A, dev)
    Bp = torch.zeros((k, n + 8), dtype=torch.float32, device=dev)
    Bp[:, :n] = to_dev(B, dev)
    Cp = torch.zeros((m, n + 4), dtype=torch.float32, device=dev)
    Cp[:, :n] = to_dev(C, dev)
    btas.tropical_gemm(Ap[:, :k], Bp[:, :n], Cp[:, :n], semiring=sr)
    assert_same(to_np(Cp[:, :n]), want, f"{sr}/frac={frac} full tiles")
    assert (Cp[:, n:] == 0).all()
    # a ragged sub-shape of the same operands goes through the staged kernel
    mr, nr = m - 1, n - 3
    Cr = to_dev(C[:mr, :nr], dev)
    btas.tropical_gemm(to_dev(A[:mr], dev), to_dev(B[:, :nr], dev), Cr, semiring=sr)
    assert_same(to_np(Cr), want[:mr, :nr], f"{sr}/frac={frac} ragged")


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_gemm_xl_tiles(btas, dev, sr, dt):
    """Products whose full 256x256 tiles fill rounds of one per CU take the
    1024-thread XL tile (8192 x 2048: 32 x 8 = 256 tiles); a short k (80: five
    k-blocks) keeps the oracle quick.  Signed values, absent entries, a partly
    absent C; int32 operands within +-(2^23-1) (the binary32-exact direct
    path)."""
    m, n, k = 8192, 2048, 80
    A, B = operands(m, n, k, dt, sr, seed=141, frac=0.1, signed=True)
    if dt == "i32":
        lim = (1 << 23) - 1
        absent = wl.I32_INF if sr == "min" else wl.I32_NINF
        A = np.where(A == absent, A, np.clip(A, -lim, lim)).astype(np.int32)
        B = np.where(B == absent, B, np.clip(B, -lim, lim)).astype(np.int32)
    C = wl.signed_operand((m, n), dt, sr, seed=142, inf_frac=0.3)
    want = oracle.gemm(sr, A, B, C)
    Ct = to_dev(C, dev)
    btas.tropical_gemm(to_dev(A, dev), to_dev(B, dev), Ct, semiring=sr)
    assert_same(to_np(Ct), want, f"{sr}/{dt} XL")


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("shape", [(1536, 1536, 1536), (2048, 1024, 2048)])
def test_gemm_mid_size_direct_split_k(btas, dev, sr, shape):
    """fp32 products with full 128x128 tiles but fewer tiles than the device
    holds workgroups: k is split over direct-load tiles (6 and 8 chunks here)
    and the partials are combined with C; signed values, absent entries, a
    partly absent C, and the winning term of some outputs in the last chunk."""
    m, n, k = shape
    A, B = operands(m, n, k, "f32", sr, seed=131, frac=0.1, signed=True)
    A[:, -1] = (-1 if sr == "min" else 1) * 1e30                # the last chunk wins there
    C = wl.signed_operand((m, n), "f32", sr, seed=132, inf_frac=0.3)
    want = oracle.gemm(sr, A, B, C)
    Ct = to_dev(C, dev)
    btas.tropical_gemm(to_dev(A, dev), to_dev(B, dev), Ct, semiring=sr)
    assert_same(to_np(Ct), want, f"{sr} {shape}")


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_gemm_leading_dimensions_and_alignment(btas, dev, sr, dt):
    """Sub-views with padded rows, including leading dimensions that are not a
    multiple of 4 elements and base pointers only 4-byte aligned."""
    torch = torch_mod()
    m, n, k = 70, 45, 53
    bigA = wl.signed_operand((m + 3, k + 7), dt, sr, seed=5)
    bigB = wl.signed_operand((k + 2, n + 9), dt, sr, seed=6)
    bigC = wl.signed_operand((m + 1, n + 5), dt, sr, seed=8, inf_frac=0.5)
    A, B, C = bigA[1:1 + m, 3:3 + k], bigB[2:2 + k, 1:1 + n], bigC[1:1 + m, 1:1 + n]
    want = oracle.gemm(sr, A.copy(), B.copy(), C.copy())
    tA, tB, tC = to_dev(bigA, dev), to_dev(bigB, dev), to_dev(bigC, dev)
    vC = tC[1:1 + m, 1:1 + n]
    btas.tropical_gemm(tA[1:1 + m, 3:3 + k], tB[2:2 + k, 1:1 + n], vC, semiring=sr)
    got = to_np(tC)
    assert_same(got[1:1 + m, 1:1 + n], want, "view")
    # the padding around C is untouched
    mask = np.ones(got.shape, bool)
    mask[1:1 + m, 1:1 + n] = False
    assert np.array_equal(bits(got)[mask], bits(bigC)[mask])
    del torch


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_gemm_degenerate_sizes(btas, dev, sr, dt):
    torch = torch_mod()
    C = wl.signed_operand((5, 4), dt, sr, seed=3)
    Ct = to_dev(C, dev)
    A = to_dev(np.zeros((5, 0), C.dtype), dev)
    B = to_dev(np.zeros((0, 4), C.dtype), dev)
    btas.tropical_gemm(A, B, Ct, semiring=sr)                # k = 0: C unchanged
    assert_same(to_np(Ct), C, "k=0")
    E = to_dev(np.zeros((0, 4), C.dtype), dev)
    btas.tropical_gemm(to_dev(np.zeros((0, 3), C.dtype), dev),
                       to_dev(np.zeros((3, 4), C.dtype), dev), E, semiring=sr)  # m = 0
    del torch


def test_gemm_determinism_and_identity(btas, dev):
    torch = torch_mod()
    n = 515
    A = wl.signed_operand((n, n), "f32", "min", seed=9)
    I = np.full((n, n), np.inf, np.float32)
    np.fill_diagonal(I, 0)
    tA, tI = to_dev(A, dev), to_dev(I, dev)
    outs = [to_np(btas.tropical_gemm(tA, tI, semiring="min")) for _ in range(5)]
    for o in outs:
        assert_same(o, A, "A (.) I")
    outs = [to_np(btas.tropical_gemm(tI, tA, semiring="min")) for _ in range(3)]
    for o in outs:
        assert_same(o, A, "I (.) A")
    del torch


def test_gemm_errors(btas, dev):
    torch = torch_mod()
    A = torch.zeros((8, 8), dtype=torch.int32, device=dev)
    with pytest.raises(btas.BtasError, match="ALIAS"):
        btas.tropical_gemm(A, A, A)
    with pytest.raises(btas.BtasError, match="ALIAS"):
        btas.tropical_gemm(A[:4], A[:, :4], A[4:, 4:])
    h = btas.default_handle()
    L = btas.lib()
    st = L.btas_tropical_gemm(h.ptr, 0, 0, 4, 4, 4, A.data_ptr(), 3, A.data_ptr(), 8,
                              A.data_ptr() + 256, 8)
    assert st == 1 and b"lda" in L.btas_last_error(h.ptr)
    st = L.btas_tropical_gemm(h.ptr, 5, 0, 4, 4, 4, A.data_ptr(), 4, A.data_ptr(), 4, None, 4)
    assert st == 1 and b"semiring" in L.btas_last_error(h.ptr)
    st = L.btas_tropical_gemm(h.ptr, 0, 0, -1, 4, 4, None, 4, None, 4, None, 4)
    assert st == 1 and b"m=-1" in L.btas_last_error(h.ptr)


# ------------------------------------------------------- gemv / level 1 ---

@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("mn", [(1, 1), (5, 3), (64, 257), (1000, 999), (333, 4096)])
def test_gemv(btas, dev, sr, dt, mn):
    m, n = mn
    A = wl.signed_operand((m, n), dt, sr, seed=m)
    x = wl.signed_operand((n,), dt, sr, seed=n + 1)
    y = wl.signed_operand((m,), dt, sr, seed=3, inf_frac=0.3)
    want = oracle.gemv(sr, A, x, y)
    ty = to_dev(y, dev)
    btas.tropical_gemv(to_dev(A, dev), to_dev(x, dev), ty, semiring=sr)
    assert_same(to_np(ty), want, "gemv")


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_gemv_long_rows_padded(btas, dev, sr, dt):
    """Long rows with a leading dimension that is a multiple of 4 and
    n % 4 == 2 (vector loads, then the scalar tail), and a row whose winning
    term sits in that tail."""
    torch = torch_mod()
    m, n = 70, 1030
    A = wl.signed_operand((m, n + 2), dt, sr, seed=11)
    A[5, n - 1] = (-1 if sr == "min" else 1) * (2**28 if dt == "i32" else 1e30)
    x = wl.signed_operand((n,), dt, sr, seed=12)
    y = wl.signed_operand((m,), dt, sr, seed=13, inf_frac=0.3)
    want = oracle.gemv(sr, A[:, :n].copy(), x, y)
    tA, ty = to_dev(A, dev), to_dev(y, dev)
    btas.tropical_gemv(tA[:, :n], to_dev(x, dev), ty, semiring=sr)
    assert_same(to_np(ty), want, "long-row gemv")


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_dot_more_partials_than_one_pass(btas, dev, sr, dt):
    """2^24 + 5 elements: more vectors than one pass of the largest partial
    grid, so its loop and the final reduction over the full partial array
    run; the winning term near the end."""
    n = (1 << 24) + 5
    x = wl.signed_operand((n,), dt, sr, seed=21)
    y = wl.signed_operand((n,), dt, sr, seed=22)
    x[n - 7] = (-1 if sr == "min" else 1) * (2**28 if dt == "i32" else 1e30)
    d = to_np(btas.dot(to_dev(x, dev), to_dev(y, dev), semiring=sr))[0]
    assert_same(np.array([d]), np.array([oracle.dot(sr, x, y)], dtype=x.dtype), "dot 2^24+5")


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_gemv_strided(btas, dev, sr, dt):
    m, n = 77, 91
    A = wl.signed_operand((m, n + 3), dt, sr, seed=1)
    x = wl.signed_operand((2 * n,), dt, sr, seed=2)
    y = wl.signed_operand((3 * m,), dt, sr, seed=3)
    want = y.copy()
    want[::3] = oracle.gemv(sr, A[:, :n].copy(), x[::2].copy(), y[::3].copy())
    tA, tx, ty = to_dev(A, dev), to_dev(x, dev), to_dev(y, dev)
    btas.tropical_gemv(tA[:, :n], tx[::2], ty[::3], semiring=sr)
    assert_same(to_np(ty), want, "strided gemv")


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("n", [0, 1, 3, 1023, 100003])
def test_level1(btas, dev, sr, dt, n):
    torch = torch_mod()
    x = wl.signed_operand((n,), dt, sr, seed=n + 5)
    y = wl.signed_operand((n,), dt, sr, seed=n + 6)
    tx, ty = to_dev(x, dev), to_dev(y, dev)
    assert_same(to_np(btas.vadd(tx, ty, semiring=sr)), oracle.vadd(sr, x, y), "vadd")
    assert_same(to_np(btas.vmul(tx, ty, semiring=sr)), oracle.vmul(sr, x, y), "vmul")
    d = to_np(btas.dot(tx, ty, semiring=sr))[0]
    assert_same(np.array([d]), np.array([oracle.dot(sr, x, y)], dtype=x.dtype), "dot")
    alpha = 17 if dt == "i32" else 0.625
    ty2 = to_dev(y, dev)
    btas.axpy(alpha, tx, ty2, semiring=sr)
    assert_same(to_np(ty2), oracle.axpy(sr, alpha, x, y), "axpy")
    if n > 4:
        # strided views
        z = torch.empty(n // 2, dtype=tx.dtype, device=dev)
        btas.vmul(tx[::2][: n // 2], ty[1::2][: n // 2], z, semiring=sr)
        assert_same(to_np(z), oracle.vmul(sr, x[::2][: n // 2].copy(), y[1::2][: n // 2].copy()), "vmul strided")
        ty3 = to_dev(y, dev)
        m3 = n // 2
        btas.axpy(alpha, tx[::2][:m3], ty3[1::2][:m3], semiring=sr)
        want3 = y.copy()
        want3[1::2][:m3] = oracle.axpy(sr, alpha, x[::2][:m3].copy(), y[1::2][:m3].copy())
        assert_same(to_np(ty3), want3, "axpy strided")
        ds = to_np(btas.dot(tx[::2], ty[::2], semiring=sr))[0]
        assert_same(np.array([ds]), np.array([oracle.dot(sr, x[::2].copy(), y[::2].copy())], dtype=x.dtype),
                    "dot strided")
        # the winning term in the tail (n % 4 elements) and in the second vector
        # of an unrolled iteration
        for pos in (n - 1, n // 2 + 1):
            xp = x.copy()
            xp[pos] = (-1 if sr == "min" else 1) * (2**28 if dt == "i32" else 1e30)
            dp = to_np(btas.dot(to_dev(xp, dev), ty, semiring=sr))[0]
            assert_same(np.array([dp]), np.array([oracle.dot(sr, xp, y)], dtype=x.dtype), f"dot pos={pos}")


# ----------------------------------------------------------------- APSP ---

def test_apsp_small_config_golden(btas, dev):
    """n=256 ER digraph (p=0.05, weights U{1..100}, seed 1), T=8 squarings."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "apsp_er256.json")))
    W = wl.er_digraph_i32(256, 0.05, 1, 100, seed=1)
    assert hashlib.sha256(W.tobytes()).hexdigest() == gold["apsp_er256_i32_seed1"]["input_sha256"]
    D, steps, _ = btas.apsp(to_dev(W, dev))
    Dn = to_np(D)
    assert steps == 8
    assert hashlib.sha256(Dn.tobytes()).hexdigest() == gold["apsp_er256_i32_seed1"]["D_sha256"]
    want, _, _ = oracle.apsp(W)
    assert_same(Dn, want, "apsp n=256")
    D2, steps2, _ = btas.apsp(to_dev(W, dev), early_exit=True)
    assert steps2 == gold["apsp_er256_i32_seed1_early_exit"]["steps"]
    assert_same(to_np(D2), want, "apsp n=256 early exit")


@pytest.mark.parametrize("path", ["default", "per_squaring"])
@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 16, 23, 24, 32, 64, 128, 192, 193, 255, 256, 257, 512])
def test_apsp_sizes(btas, dev, dt, n, path, monkeypatch):
    """Small n take the single-launch solve by default; BTAS_SINGLE_LAUNCH=0
    keeps them on one launch per squaring.  Both equal the oracle."""
    if path == "per_squaring":
        monkeypatch.setenv("BTAS_SINGLE_LAUNCH", "0")
    Wi = wl.er_digraph_i32(n, min(1.0, 3.0 / n), 1, 1000, seed=n)
    if dt == "f32":
        g = wl.rng(n + 1)
        W = np.where(Wi == wl.I32_INF, np.inf, g.exponential(1.0, (n, n))).astype(np.float32)
        np.fill_diagonal(W, 0)
    else:
        W = Wi
    want, wsteps, _ = oracle.apsp(W)
    D, steps, _ = btas.apsp(to_dev(W, dev))
    assert steps == wsteps
    assert_same(to_np(D), want, f"apsp {dt} n={n}")
    want_e, wsteps_e, _ = oracle.apsp(W, early_exit=True)
    D, steps, _ = btas.apsp(to_dev(W, dev), early_exit=True)
    assert steps == wsteps_e
    assert_same(to_np(D), want_e, f"apsp early {dt} n={n}")
    assert_same(want_e, want, "early == fixed")


@pytest.mark.parametrize("dt", DT)
def test_apsp_in_place_and_padded(btas, dev, dt):
    torch = torch_mod()
    n = 133
    Wi = wl.er_digraph_i32(n, 0.05, 1, 50, seed=11)
    W = Wi if dt == "i32" else np.where(Wi == wl.I32_INF, np.inf, Wi * 0.3).astype(np.float32)
    want, _, _ = oracle.apsp(W)
    t = to_dev(W, dev)
    btas.apsp(t, out=t)                                    # in place, T = 8 (even)
    assert_same(to_np(t), want, "in place")
    n2 = 100                                               # T = 7 (odd)
    W2 = W[:n2, :n2].copy()
    want2, _, _ = oracle.apsp(W2)
    big = torch.full((n2, n2 + 5), 7, dtype=t.dtype, device=dev)
    big[:, :n2] = to_dev(W2, dev)
    out = torch.zeros((n2 + 1, n2 + 3), dtype=t.dtype, device=dev)
    btas.apsp(big[:, :n2], out=out[:n2, :n2])
    assert_same(to_np(out)[:n2, :n2], want2, "padded")
    in_place_pad = big[:, :n2]
    btas.apsp(in_place_pad, out=in_place_pad)
    assert_same(to_np(big)[:, :n2], want2, "padded in place")


def test_apsp_neg_cycle_and_errors(btas, dev):
    INF = wl.I32_INF
    W = np.array([[0, 1, INF], [-3, 0, INF], [INF, 2, 0]], np.int32)
    _, _, st = btas.apsp(to_dev(W, dev), check_neg_cycle=True)
    assert st == btas.WARN_NEG_CYCLE
    _, _, st = btas.apsp(to_dev(np.abs(W), dev), check_neg_cycle=True)
    assert st == btas.OK
    torch = torch_mod()
    M = torch.zeros((8, 9), dtype=torch.int32, device=dev)
    with pytest.raises(btas.BtasError, match="ALIAS"):
        btas.apsp(M[:, :8], out=M[:, 1:9])


def test_validate_mode_detects_domain(btas, dev, monkeypatch):
    """BTAS_VALIDATE=1 handles reject out-of-domain operands before writing."""
    torch = torch_mod()
    monkeypatch.setenv("BTAS_VALIDATE", "1")
    h = btas.Handle(0)
    h.bind_stream()
    A = torch.zeros((4, 4), dtype=torch.int32, device=dev)
    A[1, 2] = (1 << 29)                                     # one past the bound
    B = torch.zeros((4, 4), dtype=torch.int32, device=dev)
    C = torch.full((4, 4), 5, dtype=torch.int32, device=dev)
    with pytest.raises(btas.BtasError, match="DOMAIN"):
        btas.tropical_gemm(A, B, C, handle=h)
    assert (C == 5).all()
    A[1, 2] = btas.I32_INF
    btas.tropical_gemm(A, B, C, handle=h)
    F = torch.zeros((3, 3), dtype=torch.float32, device=dev)
    F[0, 0] = float("nan")
    with pytest.raises(btas.BtasError, match="DOMAIN"):
        btas.tropical_gemm(F, F.clone(), torch.zeros_like(F), handle=h)
    h.close()


# ------------------------------------- int32 on the binary32-exact path ---

@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("edge", [(1 << 23) - 1, 1 << 23, (1 << 29) - 1])
def test_gemm_i32_exact_range_boundary(btas, dev, sr, edge):
    """Operands whose largest finite magnitude is just inside / just outside
    the range computed on the binary32 pipeline give the oracle's bits."""
    m, n, k = 300, 260, 270
    g = wl.rng(edge % 1000 + (sr == "max"))
    A = g.integers(-edge, edge, size=(m, k), endpoint=True).astype(np.int32)
    B = g.integers(-edge, edge, size=(k, n), endpoint=True).astype(np.int32)
    A[0, 0], B[0, 0] = edge, -edge                         # hit the extremes exactly
    absent = wl.I32_INF if sr == "min" else wl.I32_NINF
    A[g.random((m, k)) < 0.1] = absent
    B[g.random((k, n)) < 0.1] = absent
    C = wl.signed_operand((m, n), "i32", sr, seed=4, inf_frac=0.5)
    want = oracle.gemm(sr, A, B, C)
    Ct = to_dev(C, dev)
    btas.tropical_gemm(to_dev(A, dev), to_dev(B, dev), Ct, semiring=sr)
    assert_same(to_np(Ct), want, f"edge={edge}")


@pytest.mark.parametrize("sr", ["min", "max"])
@pytest.mark.parametrize("edge", [1 << 28, (1 << 29) - 1])
@pytest.mark.parametrize("shape", [(300, 260, 270), (130, 1000, 4100)])
def test_gemm_i32_wide_values(btas, dev, sr, edge, shape):
    """Beyond the binary32 range the int32 product runs on clamped integer
    adds: operands up to the contract's 2^29 - 1 (finite sums reach
    +-(2^30 - 2); a sum with the absent value must never win), with absent
    rows and columns, give the oracle's bits.  The taller shape splits k."""
    m, n, k = shape
    g = wl.rng(edge % 997 + (sr == "max") + m)
    A = g.integers(-edge, edge, size=(m, k), endpoint=True).astype(np.int32)
    B = g.integers(-edge, edge, size=(k, n), endpoint=True).astype(np.int32)
    A[0, 0], B[0, 0] = edge, edge                          # the largest finite sum
    A[1, 0], B[0, 1] = -edge, -edge                        # the smallest
    absent = wl.I32_INF if sr == "min" else wl.I32_NINF
    A[g.random((m, k)) < 0.15] = absent
    B[g.random((k, n)) < 0.15] = absent
    A[2, :] = absent                                       # a row with no finite term
    B[:, 3] = absent
    A[3, :] = -edge if sr == "min" else edge               # terms that meet absent ones
    C = wl.signed_operand((m, n), "i32", sr, seed=5, inf_frac=0.5)
    want = oracle.gemm(sr, A, B, C)
    Ct = to_dev(C, dev)
    btas.tropical_gemm(to_dev(A, dev), to_dev(B, dev), Ct, semiring=sr)
    assert_same(to_np(Ct), want, f"edge={edge}")


@pytest.mark.parametrize("sr", SR)
def test_gemm_i32_full_tiles_direct_path(btas, dev, sr):
    """int32 shapes whose 128x128 tiles are all full: operands within
    +-(2^23-1) take the direct-load kernel (int32 bits converted to binary32
    in LDS, absent values included), operands beyond it the integer kernel
    launched after it; three calls in a row switch between the two on the
    device.  Extremes, absent rows and columns, a partly absent C and padded
    leading dimensions; every call gives the oracle's bits."""
    torch = torch_mod()
    m, n, k = 3200, 2688, 96                       # 525 full 128 x 128 tiles, k % 16 == 0
    absent = wl.I32_INF if sr == "min" else wl.I32_NINF
    for call, edge in enumerate([(1 << 23) - 1, 1 << 23, (1 << 23) - 1]):
        g = wl.rng(300 + call + (sr == "max"))
        A = g.integers(-edge, edge, size=(m, k), endpoint=True).astype(np.int32)
        B = g.integers(-edge, edge, size=(k, n), endpoint=True).astype(np.int32)
        A[0, 0], B[0, 0] = edge, edge                      # the largest finite sum
        A[1, 0], B[0, 1] = -edge, -edge                    # the smallest
        A[g.random((m, k)) < 0.1] = absent
        B[g.random((k, n)) < 0.1] = absent
        A[2, :] = absent                                   # a row with no finite term
        B[:, 3] = absent
        A[3, :] = -edge if sr == "min" else edge           # terms that meet absent ones
        C = wl.signed_operand((m, n), "i32", sr, seed=6 + call, inf_frac=0.3)
        want = oracle.gemm(sr, A, B, C)
        Ap = torch.zeros((m, k + 4), dtype=torch.int32, device=dev)
        Ap[:, :k] = to_dev(A, dev)
        Bp = torch.zeros((k, n + 8), dtype=torch.int32, device=dev)
        Bp[:, :n] = to_dev(B, dev)
        Cp = torch.zeros((m, n + 4), dtype=torch.int32, device=dev)
        Cp[:, :n] = to_dev(C, dev)
        btas.tropical_gemm(Ap[:, :k], Bp[:, :n], Cp[:, :n], semiring=sr)
        assert_same(to_np(Cp[:, :n]), want, f"{sr}/call {call}/edge={edge}")
        assert (Cp[:, n:] == 0).all()


def test_apsp_i32_distances_cross_exact_range(btas, dev):
    """A path graph with heavy edges: early squarings stay within +-(2^23-1),
    later ones exceed it and must switch to the integer pipeline."""
    n = 150
    W = np.full((n, n), wl.I32_INF, np.int32)
    np.fill_diagonal(W, 0)
    g = wl.rng(12)
    for i in range(n - 1):
        W[i, i + 1] = int(g.integers(1 << 19, 1 << 20))
    back = np.tril(g.random((n, n)) < 0.02, k=-1)          # backward edges only:
    W[back] = 1 << 21                                       # forward distances stay long
    np.fill_diagonal(W, 0)
    want, _, _ = oracle.apsp(W)
    assert want[0, n - 1] > (1 << 23)
    D, _, _ = btas.apsp(to_dev(W, dev))
    assert_same(to_np(D), want, "crossing")


@pytest.mark.parametrize("dt", DT)
def test_apsp_graph_mode_replays_current_inputs(btas, dev, dt):
    """The captured solve is replayed on the current contents of W."""
    for n in (5, 100, 256):
        outs = []
        t = out = None
        for seed in (1, 2, 3):
            Wi = wl.er_digraph_i32(n, min(1.0, 6.0 / n), 1, 100, seed=seed * 100 + n)
            W = Wi if dt == "i32" else np.where(Wi == wl.I32_INF, np.inf, Wi * 0.5).astype(np.float32)
            if t is None:
                t = to_dev(W, dev)
                out = torch_mod().empty_like(t)
            else:
                t.copy_(to_dev(W, dev))
            btas.apsp(t, out=out, graph=True, return_steps=False)
            want, _, _ = oracle.apsp(W)
            assert_same(to_np(out), want, f"graph n={n} seed={seed}")
            outs.append(want)
    with pytest.raises(btas.BtasError, match="INVALID_ARG"):
        btas.apsp(t, early_exit=True, graph=True)


def test_calls_follow_torch_current_stream(btas, dev):
    """The default handle launches on torch's current stream: a chain of
    products alternating between two streams (ordered with wait_stream) gives
    the oracle's bits, and after each call the handle is bound to the stream
    that was current."""
    torch = torch_mod()
    g = np.random.default_rng(5)
    A = g.random((96, 80), dtype=np.float32)
    B = g.random((80, 80), dtype=np.float32)
    want = oracle.gemm("min", A, B, np.full((96, 80), np.inf, np.float32))
    want = oracle.gemm("min", want, B, np.full((96, 80), np.inf, np.float32))
    want = oracle.gemm("min", want, B, np.full((96, 80), np.inf, np.float32))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    tA = torch.from_numpy(A).to(dev)
    tB = torch.from_numpy(B).to(dev)
    torch.cuda.synchronize()
    h = btas.default_handle(0)
    cur = tA
    for s in (s1, s2, s1):
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            s.wait_stream(s1 if s is s2 else s2)
            cur = btas.tropical_gemm(cur, tB, semiring="min")
            assert h._bound == s.cuda_stream
    torch.cuda.synchronize()
    got = cur.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    btas.default_handle(0)  # back on the default stream
    assert h._bound == torch.cuda.current_stream().cuda_stream
