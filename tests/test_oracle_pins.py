"""Pins for the CPU oracle: each test checks it against something other than
itself (IEEE binary32 arithmetic done by numpy, scipy's Dijkstra, brute-force
path enumeration, closed forms, algebraic identities of the semiring), chosen
so that a dropped term, a wrong sign or index, a swapped min/max or a
transposed operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import hand_cases
import oracle
from oracle import INF32, NINF32, FINITE_MAX
from paper_1701_04733_amd import workloads as wl

SR = ["min", "max"]
DT = ["i32", "f32"]


def _np_dtype(dt):
    return np.int32 if dt == "i32" else np.float32


def _absent(dt, sr):
    if dt == "i32":
        return INF32 if sr == "min" else NINF32
    return np.float32(np.inf if sr == "min" else -np.inf)


def _identity(n, dt, sr):
    """Tropical identity: (.)-one (0) on the diagonal, (+)-zero elsewhere."""
    I = np.full((n, n), _absent(dt, sr), dtype=_np_dtype(dt))
    np.fill_diagonal(I, 0)
    return I


def _fp32_product_numpy(sr, A, B, C):
    """Per-term IEEE binary32 adds (numpy float32 arithmetic) then min/max.

    This is the textbook definition evaluated in binary32 by a library, a
    different computation from the oracle's binary64 evaluation."""
    S = A[:, :, None] + B[None, :, :]           # float32 + float32 -> float32 (RN)
    assert S.dtype == np.float32
    red = S.min(axis=1) if sr == "min" else S.max(axis=1)
    return np.minimum(C, red) if sr == "min" else np.maximum(C, red)


def _i32_product_numpy(sr, A, B, C):
    """int64 numpy broadcast with the absent value masked in afterwards."""
    A64, B64 = A.astype(np.int64), B.astype(np.int64)
    S = A64[:, :, None] + B64[None, :, :]
    absent = INF32 if sr == "min" else NINF32
    touch = (A == absent)[:, :, None] | (B == absent)[None, :, :]
    big = np.int64(1) << 40
    S = np.where(touch, big if sr == "min" else -big, S)
    red = S.min(axis=1) if sr == "min" else S.max(axis=1)
    red = np.where(np.abs(red) >= big, absent, red)
    out = np.minimum(C.astype(np.int64), red) if sr == "min" else np.maximum(C.astype(np.int64), red)
    return out.astype(np.int32)


# ------------------------------------------------------------------ GEMM ---

@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 7), (17, 9, 33), (40, 31, 64)])
def test_gemm_f32_equals_binary32_per_term(sr, shape):
    m, n, k = shape
    A = wl.signed_operand((m, k), "f32", sr, seed=11)
    B = wl.signed_operand((k, n), "f32", sr, seed=12)
    C = wl.signed_operand((m, n), "f32", sr, seed=13, inf_frac=0.3)
    got = oracle.gemm(sr, A, B, C)
    want = _fp32_product_numpy(sr, A, B, C)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_gemm_f32_rounding_cases():
    """Sums that round in binary32 (ties-to-even, overflow to inf, subnormals)."""
    big = np.float32(3.0e38)
    tiny = np.float32(1e-45)                       # smallest subnormal
    one = np.float32(1.0)
    eps_half = np.float32(2.0 ** -24)              # exactly half an ulp of 1.0
    A = np.array([[one, big, tiny, np.float32(1.5) * eps_half]], dtype=np.float32)
    k = A.shape[1]
    for j, bval in enumerate([eps_half, big, tiny, one]):
        B = np.full((k, 1), np.inf, dtype=np.float32)
        B[j, 0] = bval
        C = np.full((1, 1), np.inf, dtype=np.float32)
        got = oracle.gemm("min", A, B, C)[0, 0]
        with np.errstate(over="ignore"):
            want = np.float32(A[0, j] + bval)      # binary32 add
        assert got.view(np.uint32) == want.view(np.uint32)
    # 1 + 2^-24 is a tie and rounds to even (1.0); 3e38+3e38 overflows to inf
    assert oracle.gemm("min", np.array([[one]], np.float32), np.array([[eps_half]], np.float32),
                       np.array([[np.inf]], np.float32))[0, 0] == one
    assert np.isinf(oracle.gemm("min", np.array([[big]], np.float32), np.array([[big]], np.float32),
                                np.array([[np.inf]], np.float32))[0, 0])


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("shape", [(1, 1, 1), (4, 6, 5), (19, 23, 29), (33, 8, 70)])
def test_gemm_i32_equals_int64_numpy(sr, shape):
    m, n, k = shape
    A = wl.signed_operand((m, k), "i32", sr, seed=21)
    B = wl.signed_operand((k, n), "i32", sr, seed=22)
    C = wl.signed_operand((m, n), "i32", sr, seed=23, inf_frac=0.3)
    assert np.array_equal(oracle.gemm(sr, A, B, C), _i32_product_numpy(sr, A, B, C))


@pytest.mark.parametrize("sr", SR)
def test_gemm_i32_sentinel_absorbs_at_domain_edge(sr):
    absent = INF32 if sr == "min" else NINF32
    far = -FINITE_MAX if sr == "min" else FINITE_MAX   # pulls hardest against absorption
    A = np.array([[absent, far]], dtype=np.int32)
    B = np.array([[far], [absent]], dtype=np.int32)
    C = np.array([[absent]], dtype=np.int32)
    assert oracle.gemm(sr, A, B, C)[0, 0] == absent
    # the extreme finite sums are exact
    A2 = np.array([[far]], dtype=np.int32)
    assert oracle.gemm(sr, A2, A2, np.array([[absent]], np.int32))[0, 0] == 2 * far


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_gemm_identity_and_absorbing(sr, dt):
    A = wl.signed_operand((13, 13), dt, sr, seed=31)
    I = _identity(13, dt, sr)
    Z = np.full((13, 13), _absent(dt, sr), dtype=_np_dtype(dt))
    same = lambda x, y: np.array_equal(x.view(np.uint32), y.view(np.uint32))
    assert same(oracle.gemm(sr, A, I, Z), A)
    assert same(oracle.gemm(sr, I, A, Z), A)
    assert same(oracle.gemm(sr, A, Z, Z), Z)
    assert same(oracle.gemm(sr, Z, A, Z), Z)


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_gemm_k1_outer_sum(sr, dt):
    a = wl.signed_operand((7, 1), dt, sr, seed=41, inf_frac=0.2)
    b = wl.signed_operand((1, 11), dt, sr, seed=42, inf_frac=0.2)
    C = wl.semiring_identity_matrix((7, 11), dt, sr)
    got = oracle.gemm(sr, a, b, C)
    absent = _absent(dt, sr)
    for i in range(7):
        for j in range(11):
            if a[i, 0] == absent or b[0, j] == absent:
                assert got[i, j] == absent
            elif dt == "i32":
                assert int(got[i, j]) == int(a[i, 0]) + int(b[0, j])
            else:
                assert got[i, j].view(np.uint32) == np.float32(a[i, 0] + b[0, j]).view(np.uint32)


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_gemm_k0_leaves_c(sr, dt):
    C = wl.signed_operand((5, 4), dt, sr, seed=51)
    A = np.zeros((5, 0), dtype=_np_dtype(dt))
    B = np.zeros((0, 4), dtype=_np_dtype(dt))
    assert np.array_equal(oracle.gemm(sr, A, B, C).view(np.uint32), C.view(np.uint32))


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_gemm_transpose_identity(sr, dt):
    A = wl.signed_operand((9, 14), dt, sr, seed=61)
    B = wl.signed_operand((14, 6), dt, sr, seed=62)
    C = wl.signed_operand((9, 6), dt, sr, seed=63, inf_frac=0.5)
    left = oracle.gemm(sr, A, B, C).T
    right = oracle.gemm(sr, np.ascontiguousarray(B.T), np.ascontiguousarray(A.T),
                        np.ascontiguousarray(C.T))
    assert np.array_equal(left.view(np.uint32), right.view(np.uint32))


@pytest.mark.parametrize("dt", DT)
def test_gemm_max_min_duality(dt):
    A = wl.signed_operand((12, 10), dt, "max", seed=71)
    B = wl.signed_operand((10, 15), dt, "max", seed=72)
    C = wl.signed_operand((12, 15), dt, "max", seed=73, inf_frac=0.4)
    # -(-0x7FFFFFFF) == 0x7FFFFFFF: the sentinels are exact negatives
    mx = oracle.gemm("max", A, B, C)
    mn = oracle.gemm("min", -A, -B, -C)
    if dt == "i32":
        assert np.array_equal(mx, -mn)
    else:
        # only the sign of an exactly-cancelled zero may differ: compare values
        assert np.array_equal(mx, -mn)


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_gemm_leading_dimensions(sr, dt):
    """Views with padded rows (lda > k etc.) give the same result."""
    A = wl.signed_operand((6, 20), dt, sr, seed=81)
    B = wl.signed_operand((20, 30), dt, sr, seed=82)
    C = wl.semiring_identity_matrix((6, 9), dt, sr)
    got = oracle.gemm(sr, A[:, 3:11], B[3:11, 5:14], C)
    want = oracle.gemm(sr, A[:, 3:11].copy(), B[3:11, 5:14].copy(), C)
    ref = (_i32_product_numpy if dt == "i32" else _fp32_product_numpy)(
        sr, A[:, 3:11].copy(), B[3:11, 5:14].copy(), C)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_gemm_domain_errors():
    ok = np.zeros((2, 2), np.int32)
    for bad in (np.iinfo(np.int32).min, FINITE_MAX + 1, -(FINITE_MAX + 1), NINF32):
        A = ok.copy()
        A[0, 1] = bad
        with pytest.raises(oracle.OracleError):
            oracle.gemm("min", A, ok, np.full((2, 2), INF32, np.int32))
    F = np.zeros((2, 2), np.float32)
    for sr, bad in (("min", -np.inf), ("max", np.inf), ("min", np.nan)):
        A = F.copy()
        A[1, 1] = bad
        with pytest.raises(oracle.OracleError):
            oracle.gemm(sr, A, F, F.copy())


# ------------------------------------------------------- gemv / level 1 ---

@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_gemv_is_one_column_gemm(sr, dt):
    A = wl.signed_operand((17, 23), dt, sr, seed=91)
    x = wl.signed_operand((23,), dt, sr, seed=92)
    y = wl.signed_operand((17,), dt, sr, seed=93, inf_frac=0.3)
    got = oracle.gemv(sr, A, x, y)
    ref = (_i32_product_numpy if dt == "i32" else _fp32_product_numpy)(
        sr, A, x.reshape(-1, 1), y.reshape(-1, 1))[:, 0]
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
def test_level1(sr, dt):
    x = wl.signed_operand((257,), dt, sr, seed=101)
    y = wl.signed_operand((257,), dt, sr, seed=102)
    absent = _absent(dt, sr)
    red = np.minimum if sr == "min" else np.maximum
    assert np.array_equal(oracle.vadd(sr, x, y), red(x, y))
    z = oracle.vmul(sr, x, y)
    d = oracle.dot(sr, x, y)
    if dt == "f32":
        want = x + y                                   # binary32 adds
        assert np.array_equal(z.view(np.uint32), want.view(np.uint32))
        wd = want.min() if sr == "min" else want.max()
        assert np.float32(d).view(np.uint32) == np.float32(wd).view(np.uint32)
    else:
        s = x.astype(np.int64) + y.astype(np.int64)
        s[(x == absent) | (y == absent)] = absent
        assert np.array_equal(z.astype(np.int64), s)
        assert int(d) == int(s.min() if sr == "min" else s.max())
    alpha = 5 if dt == "i32" else np.float32(0.375)
    ax = oracle.axpy(sr, alpha, x, y)
    t = oracle.vmul(sr, np.full_like(x, alpha), x)
    assert np.array_equal(ax.view(np.uint32), red(y, t).view(np.uint32))
    # empty dot is the (+)-identity
    e = oracle.dot(sr, x[:0], y[:0])
    assert e == absent


# ----------------------------------------------------------------- APSP ---

@pytest.mark.parametrize("n,T", [(0, 0), (1, 0), (2, 0), (3, 1), (4, 2), (5, 2), (16, 4),
                                 (17, 4), (18, 5), (256, 8), (257, 8), (258, 9), (512, 9),
                                 (16384, 14)])
def test_squaring_count(n, T):
    assert oracle.apsp_steps(n) == T
    if n > 2:
        # smallest T with 2^T >= n-1: paths of up to n-1 edges are covered
        assert 2 ** T >= n - 1 and 2 ** (T - 1) < n - 1


def _to_scipy(W):
    from scipy.sparse.csgraph import csgraph_from_dense
    Wf = W.astype(np.float64)
    if W.dtype == np.int32:
        Wf[W == INF32] = np.inf
    np.fill_diagonal(Wf, np.inf)           # self loops never help (non-negative)
    return csgraph_from_dense(Wf, null_value=np.inf)


def _dijkstra(W, indices=None):
    from scipy.sparse.csgraph import dijkstra
    return dijkstra(_to_scipy(W), directed=True, indices=indices)


@pytest.mark.parametrize("seed", range(6))
def test_apsp_tiny_bruteforce(seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(1, 8))
    W = wl.er_digraph_i32(n, 0.4, 0, 9, seed=100 + seed)      # includes zero weights
    D, steps, _ = oracle.apsp(W)
    bf = oracle.brute_force_apsp(W.tolist(), INF32)
    assert D.tolist() == bf
    assert steps == oracle.apsp_steps(n)


@pytest.mark.parametrize("n,p", [(16, 0.2), (64, 0.05), (128, 0.05), (200, 0.02)])
def test_apsp_i32_vs_fw_and_dijkstra(n, p):
    W = wl.er_digraph_i32(n, p, 1, 100, seed=n)
    D, _, _ = oracle.apsp(W)
    assert np.array_equal(D, oracle.floyd_warshall(W))
    dj = _dijkstra(W)
    want = np.where(np.isinf(dj), INF32, dj).astype(np.int64)
    assert np.array_equal(D.astype(np.int64), want)


def test_apsp_naive_products_agree():
    """The n-1 plain products D <- D (.) (I (+) W) of Sec. III give the same
    distances as repeated squaring."""
    n = 40
    W = wl.er_digraph_i32(n, 0.06, 1, 50, seed=7)
    W0 = W.copy()
    np.fill_diagonal(W0, 0)
    D = W0.copy()
    Z = np.full((n, n), INF32, np.int32)
    for _ in range(n - 2):
        D = oracle.gemm("min", D, W0, Z)
    Dsq, _, _ = oracle.apsp(W)
    assert np.array_equal(D, Dsq)


def test_apsp_one_step_short_is_wrong():
    """A directed path needs all T squarings: with T-1 it is not solved."""
    n = 18                                        # n-1 = 17 > 2^4, so T = 5
    W = np.full((n, n), INF32, np.int32)
    np.fill_diagonal(W, 0)
    for i in range(n - 1):
        W[i, i + 1] = 1
    D, steps, _ = oracle.apsp(W)
    assert steps == 5 and D[0, n - 1] == n - 1
    cur = W.copy()
    for _ in range(4):
        cur = oracle.gemm("min", cur, cur, cur)
    assert cur[0, n - 1] == INF32


@pytest.mark.parametrize("dt", DT)
def test_apsp_closed_forms(dt):
    npdt = _np_dtype(dt)
    absent = _absent(dt, "min")
    # directed cycle, unit weights: d(i,j) = (j - i) mod n
    n = 37
    W = np.full((n, n), absent, npdt)
    for i in range(n):
        W[i, (i + 1) % n] = 1
    D, _, _ = oracle.apsp(W)
    i, j = np.indices((n, n))
    assert np.array_equal(D, ((j - i) % n).astype(npdt))
    # directed path: j - i above the diagonal, absent below
    P = np.full((n, n), absent, npdt)
    for a in range(n - 1):
        P[a, a + 1] = 1
    D, _, _ = oracle.apsp(P)
    assert np.array_equal(D, np.where(j >= i, j - i, absent).astype(npdt))
    # complete graph of ones: 1 off the diagonal, one step reaches the fixpoint
    K = np.ones((n, n), npdt)
    D, steps, _ = oracle.apsp(K, early_exit=True)
    assert np.array_equal(D, np.where(i == j, 0, 1).astype(npdt)) and steps == 1
    # undirected 6x7 grid, unit weights: Manhattan distance
    r, c = 6, 7
    G = np.full((r * c, r * c), absent, npdt)
    for y in range(r):
        for x in range(c):
            u = y * c + x
            if x + 1 < c:
                G[u, u + 1] = G[u + 1, u] = 1
            if y + 1 < r:
                G[u, u + c] = G[u + c, u] = 1
    D, _, _ = oracle.apsp(G)
    yy, xx = np.divmod(np.arange(r * c), c)
    man = np.abs(yy[:, None] - yy[None, :]) + np.abs(xx[:, None] - xx[None, :])
    assert np.array_equal(D, man.astype(npdt))
    # two components: absent blocks between them
    B = np.full((10, 10), absent, npdt)
    B[:5, :5] = 2
    B[5:, 5:] = 3
    D, _, _ = oracle.apsp(B)
    assert (D[:5, 5:] == absent).all() and (D[5:, :5] == absent).all()


def test_apsp_f32_integer_weights_exact():
    n = 60
    Wi = wl.er_digraph_i32(n, 0.08, 1, 1000, seed=9)
    Wf = np.where(Wi == INF32, np.inf, Wi).astype(np.float32)
    D, _, _ = oracle.apsp(Wf)
    fw = oracle.floyd_warshall(Wf)
    assert np.array_equal(D.astype(np.float64), fw)
    Di, _, _ = oracle.apsp(Wi)
    assert np.array_equal(np.where(Di == INF32, np.inf, Di), D.astype(np.float64))


def test_apsp_f32_rounding_bound_vs_dijkstra():
    """Each distance is a depth-<=T tree of rounded adds of non-negative
    weights, so (1-u)^T d* <= d32 <= (1+u)^T d* with u = 2^-24."""
    n = 300
    r, c, w = wl.sparse_digraph_f32_exp(n, 6.0, seed=4)
    W = wl.coo_to_dense_f32(n, r, c, w)
    D, steps, _ = oracle.apsp(W, early_exit=True)
    T = oracle.apsp_steps(n)
    exact = _dijkstra(W)
    fin = np.isfinite(exact)
    assert np.array_equal(fin, np.isfinite(D))
    u = 2.0 ** -24
    d = D.astype(np.float64)[fin]
    e = exact[fin]
    assert np.all(d <= e * (1 + u) ** T + 1e-300)
    assert np.all(d >= e * (1 - u) ** T - 1e-300)
    assert 1 <= steps <= T


def test_apsp_early_exit_equals_fixed_T():
    W = wl.er_digraph_i32(150, 0.1, 1, 100, seed=3)
    Dfix, sfix, _ = oracle.apsp(W)
    Dee, see, _ = oracle.apsp(W, early_exit=True)
    assert np.array_equal(Dfix, Dee) and see <= sfix
    Wf = np.where(W == INF32, np.inf, W * np.float32(0.37)).astype(np.float32)
    Ffix, _, _ = oracle.apsp(Wf)
    Fee, _, _ = oracle.apsp(Wf, early_exit=True)
    assert np.array_equal(Ffix.view(np.uint32), Fee.view(np.uint32))


def test_apsp_invariants_small_config():
    """n=256 ER graph, p=0.05, weights in [1,100]: diagonal 0, bounded by
    I (+) W, fixpoint and triangle inequality exact, reachability = BFS."""
    from scipy.sparse.csgraph import breadth_first_order  # noqa: F401
    W = wl.er_digraph_i32(256, 0.05, 1, 100, seed=1)
    D, steps, st = oracle.apsp(W, check_neg_cycle=True)
    assert st == oracle.OK and steps == 8
    assert (np.diag(D) == 0).all()
    W0 = W.copy()
    np.fill_diagonal(W0, 0)
    assert (D.astype(np.int64) <= W0.astype(np.int64)).all()
    assert np.array_equal(oracle.gemm("min", D, D, D), D)    # fixpoint
    # reachability equals the boolean transitive closure
    R = (W0 != INF32)
    for _ in range(9):
        R = R | ((R.astype(np.int32) @ R.astype(np.int32)) > 0)
    assert np.array_equal(R, D != INF32)


def test_apsp_negative_cycle_flag():
    # a two-edge cycle of weight 1 + (-3) is seen by the first squaring
    W = np.array([[0, 1, INF32], [-3, 0, INF32], [INF32, 2, 0]], np.int32)
    _, _, st = oracle.apsp(W, check_neg_cycle=True)
    assert st == oracle.WNEGCYCLE
    _, _, st = oracle.apsp(np.abs(W), check_neg_cycle=True)
    assert st == oracle.OK


def test_generators_reproducible():
    a = wl.er_digraph_i32(64, 0.05, 1, 100, seed=1)
    b = wl.er_digraph_i32(64, 0.05, 1, 100, seed=1)
    assert np.array_equal(a, b) and (np.diag(a) == 0).all()
    g1 = wl.batched_graphs_i32(count=8)
    g2 = wl.batched_graphs_i32(count=8)
    assert all(np.array_equal(x, y) for x, y in zip(g1, g2))
    assert all(16 <= x.shape[0] <= 512 for x in g1)


def _read_hand_example():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "hand_4node.txt")
    mats, cur = {}, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line in ("W", "D"):
            cur = line
            mats[cur] = []
            continue
        mats[cur].append([INF32 if t == "INF" else int(t) for t in line.split()])
    return np.array(mats["W"], np.int32), np.array(mats["D"], np.int32)


def test_hand_worked_example():
    W, Dw = _read_hand_example()
    D, steps, _ = oracle.apsp(W)
    assert steps == 2 and np.array_equal(D, Dw)
    assert oracle.brute_force_apsp(W.tolist(), INF32) == Dw.tolist()
    # and as floats
    Wf = np.where(W == INF32, np.inf, W).astype(np.float32)
    Df, _, _ = oracle.apsp(Wf)
    assert np.array_equal(Df, Dw.astype(np.float32))


# ------------------------------------------------ blocked Floyd-Warshall ---

def _fw_f32_numpy(W):
    """Sequential Floyd-Warshall in binary32 with numpy: for each pivot z,
    D <- min(D, D[:, z] + D[z, :]) with float32 adds (a vectorised statement,
    independent of the oracle's loops)."""
    D = W.astype(np.float32).copy()
    np.fill_diagonal(D, np.minimum(np.diag(D), np.float32(0)))
    for z in range(D.shape[0]):
        S = D[:, z:z + 1] + D[z:z + 1, :]
        assert S.dtype == np.float32
        D = np.minimum(D, S)
    return D


@pytest.mark.parametrize("block", [1, 2, 3, 16, 64, 100, 500])
@pytest.mark.parametrize("n", [1, 2, 7, 64, 65, 130, 200])
def test_fw_blocked_i32_equals_fw_and_squaring(n, block):
    """Exact integers: every order of the relaxations gives the shortest
    distances, so the blocked order equals sequential Floyd-Warshall and
    repeated squaring, for every block size."""
    W = wl.er_digraph_i32(n, min(1.0, 4.0 / n), 0, 100, seed=n + block)
    Db = oracle.floyd_warshall_blocked(W, block)
    assert np.array_equal(Db, oracle.floyd_warshall(W))
    Dsq, _, _ = oracle.apsp(W)
    assert np.array_equal(Db, Dsq)


@pytest.mark.parametrize("seed", range(6))
def test_fw_blocked_tiny_bruteforce(seed):
    g = np.random.default_rng(50 + seed)
    n = int(g.integers(1, 8))
    W = wl.er_digraph_i32(n, 0.4, 0, 9, seed=300 + seed)
    for block in (1, 2, 3, 8):
        assert oracle.floyd_warshall_blocked(W, block).tolist() == oracle.brute_force_apsp(W.tolist(), INF32)


@pytest.mark.parametrize("n", [5, 64, 97])
def test_fw_blocked_f32_degenerate_blocks_are_sequential_fw(n):
    """With one pivot per block (B = 1) or a single block (B >= n) the blocked
    order is the sequential order, so the result equals a numpy binary32
    Floyd-Warshall bit for bit, for general (non-integer) weights."""
    r, c, w = wl.sparse_digraph_f32_exp(n, 5.0, seed=n)
    W = wl.coo_to_dense_f32(n, r, c, w)
    want = _fw_f32_numpy(W)
    for block in (1, n, n + 7):
        got = oracle.floyd_warshall_blocked(W, block)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), f"block={block}"


def test_fw_blocked_f32_integer_weights_exact():
    n = 150
    Wi = wl.er_digraph_i32(n, 0.05, 1, 1000, seed=21)
    Wf = np.where(Wi == INF32, np.inf, Wi).astype(np.float32)
    for block in (16, 64):
        Db = oracle.floyd_warshall_blocked(Wf, block)
        assert np.array_equal(Db.astype(np.float64), oracle.floyd_warshall(Wf))


def test_fw_blocked_f32_rounding_bound_vs_dijkstra():
    """Floyd-Warshall builds a path of h edges with at most h-1 rounded adds of
    non-negative values, so (1-u)^(n-1) d* <= d32 <= (1+u)^(n-1) d*."""
    n = 300
    r, c, w = wl.sparse_digraph_f32_exp(n, 6.0, seed=8)
    W = wl.coo_to_dense_f32(n, r, c, w)
    D = oracle.floyd_warshall_blocked(W, 64).astype(np.float64)
    exact = _dijkstra(W)
    fin = np.isfinite(exact)
    assert np.array_equal(fin, np.isfinite(D))
    u = 2.0 ** -24
    assert np.all(D[fin] <= exact[fin] * (1 + u) ** (n - 1) + 1e-300)
    assert np.all(D[fin] >= exact[fin] * (1 - u) ** (n - 1) - 1e-300)
    # and it is a different association from squaring in general: both are
    # within the bound, and they agree on the reachability pattern
    Dsq, _, _ = oracle.apsp(W)
    assert np.array_equal(np.isfinite(Dsq), fin)



# --------------------------------------- blocked FW in binary32: hand pins ---

def _fw_blocked_model(W, B, p1_desc=False, row_desc=False, col_desc=False, p2_pivot_inner=False,
                      phase3_first=False):
    """A scalar model of the blocked schedule with switches that plant the
    plausible slips (pivot order inside phase 1 or phase 2, the pivot loop
    inside the row loop in phase 2, phase 3 before phase 2); the default
    switches are the order the hand-worked fixtures follow."""
    n = W.shape[0]
    d = W.astype(np.float32).copy()
    np.fill_diagonal(d, np.minimum(np.diag(d), np.float32(0)))

    def relax(x, y, z):
        if not np.isfinite(d[x, z]):
            return
        s = np.float32(d[x, z]) + np.float32(d[z, y])
        if s < d[x, y]:
            d[x, y] = s

    def sweep(z, rows, cols):
        # pivot z over rows x cols; within one pivot no operand changes
        # (d(z,z) = 0), so the row can be relaxed as a vector
        c = np.array(cols, dtype=np.int64)
        for x in rows:
            if np.isfinite(d[x, z]):
                d[x, c] = np.minimum(d[x, c], np.float32(d[x, z]) + d[z, c])

    def panel(rows, cols, piv, desc):
        pv = piv[::-1] if desc else piv
        if p2_pivot_inner:
            for x in rows:
                for y in cols:
                    for z in pv:
                        relax(x, y, z)
        else:
            for z in pv:
                sweep(z, rows, cols)

    nb = (n + B - 1) // B
    blk = [list(range(K * B, min(n, K * B + B))) for K in range(nb)]
    for K in range(nb):
        piv = blk[K]
        others = [v for J in range(nb) if J != K for v in blk[J]]

        def phase3():  # its operands, blocks (I,K) and (K,J), do not change here
            oth = np.array(others, dtype=np.int64)
            for z in piv:
                for x in others:
                    if np.isfinite(d[x, z]):
                        s = np.float32(d[x, z]) + d[z, oth]
                        d[x, oth] = np.minimum(d[x, oth], s)
        for z in (piv[::-1] if p1_desc else piv):
            sweep(z, piv, piv)
        if phase3_first:
            phase3()
        panel(piv, others, piv, row_desc)
        panel(others, piv, piv, col_desc)
        if not phase3_first:
            phase3()
    return d


def _bits(a):
    return np.asarray(a, dtype=np.float32).view(np.uint32)


def test_fw_blocked_f32_hand_golden():
    """The oracle's binary32 blocked Floyd-Warshall at 1 < B < n equals the
    values worked out by hand in tests/golden/fw_blocked_f32_hand.txt, each
    case built so that one choice of relaxation order (blocked vs sequential,
    pivot order in phase 1, in the block-row, in the block-column) decides
    between 1 and 1 + 2^-23."""
    cases = hand_cases.fw_blocked_f32_cases()
    assert {c["name"] for c in cases} >= {"pair_order", "diagonal_block_pivots", "row_panel_pivots",
                                          "column_panel_pivots", "pivot_block_64"}
    for c in cases:
        assert 1 < c["block"] < c["n"]
        got = oracle.floyd_warshall_blocked(c["W"], c["block"])
        assert np.array_equal(_bits(got), _bits(c["D"])), c["name"]


def test_fw_blocked_f32_hand_golden_differs_from_sequential():
    """Where the fixtures say so, the blocked result is not the sequential
    one: numpy's binary32 sequential Floyd-Warshall and the oracle at B = 1
    both give 1 + 2^-23 where the blocked order gives 1."""
    for c in hand_cases.fw_blocked_f32_cases():
        if c["name"] not in ("pair_order", "pivot_block_64", "pair_update_256", "later_block_pivots_128"):
            continue
        seq = _fw_f32_numpy(c["W"])
        assert not np.array_equal(_bits(seq), _bits(c["D"])), c["name"]
        assert np.array_equal(_bits(oracle.floyd_warshall_blocked(c["W"], 1)), _bits(seq))
        diff = np.argwhere(seq != c["D"])
        assert len(diff) == 1
        i, j = diff[0]
        assert float(c["D"][i, j]) == 1.0 and float(seq[i, j]) == 1.0 + 2.0 ** -23


@pytest.mark.parametrize("slip", ["p1_desc", "row_desc", "col_desc", "p2_pivot_inner", "phase3_first",
                                  "sequential"])
def test_fw_blocked_f32_hand_golden_catches_order_slips(slip):
    """The fixtures discriminate: the scalar model in the fixtures' order
    reproduces every case, and each planted slip of the relaxation order
    changes at least one of them."""
    cases = hand_cases.fw_blocked_f32_cases()
    for c in cases:
        assert np.array_equal(_bits(_fw_blocked_model(c["W"], c["block"])), _bits(c["D"])), c["name"]
    wrong = 0
    for c in cases:
        if slip == "sequential":
            got = _fw_blocked_model(c["W"], c["n"])
        else:
            got = _fw_blocked_model(c["W"], c["block"], **{slip: True})
        wrong += not np.array_equal(_bits(got), _bits(c["D"]))
    assert wrong >= 1, slip

# ------------------------------------------------------------ witnesses ---

def _witness_numpy(sr, A, B, C, K):
    """Per-term values by numpy (binary32 adds for float32, masked int64 for
    int32) and numpy's argmin/argmax, which returns the first (smallest)
    index among equal extremes; strict improvement decides whether C and K
    change."""
    if A.dtype == np.float32:
        S = A[:, :, None] + B[None, :, :]
        assert S.dtype == np.float32
    else:
        absent = INF32 if sr == "min" else NINF32
        big = np.int64(1) << 40
        S = A.astype(np.int64)[:, :, None] + B.astype(np.int64)[None, :, :]
        touch = (A == absent)[:, :, None] | (B == absent)[None, :, :]
        S = np.where(touch, big if sr == "min" else -big, S)
    arg = S.argmin(axis=1) if sr == "min" else S.argmax(axis=1)
    red = np.take_along_axis(S, arg[:, None, :], axis=1)[:, 0, :]
    if A.dtype == np.int32:
        red = np.where(np.abs(red) >= (np.int64(1) << 40), absent, red)
    Cw = C.astype(red.dtype)
    imp = red < Cw if sr == "min" else red > Cw
    return np.where(imp, red, Cw).astype(C.dtype), np.where(imp, arg, K).astype(np.int32)


def _tie_heavy(dt, sr, shape, seed, absent_frac=0.15):
    """Few distinct values, so many terms of one output tie."""
    g = np.random.default_rng(seed)
    if dt == "i32":
        X = g.integers(-4, 5, shape).astype(np.int32)
    else:
        X = (g.integers(-8, 9, shape) * 0.25).astype(np.float32)
    X[g.random(shape) < absent_frac] = _absent(dt, sr)
    return X


@pytest.mark.parametrize("sr", SR)
@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 7, 3), (17, 9, 33), (40, 31, 64)])
def test_gemm_witness_equals_numpy_argmin(sr, dt, shape):
    m, n, k = shape
    A = _tie_heavy(dt, sr, (m, k), 1)
    B = _tie_heavy(dt, sr, (k, n), 2)
    C = _tie_heavy(dt, sr, (m, n), 3, absent_frac=0.5)
    K = np.random.default_rng(4).integers(-1, 1000, (m, n)).astype(np.int32)
    Cw, Kw = oracle.gemm_witness(sr, A, B, C, K)
    Cn, Kn = _witness_numpy(sr, A, B, C, K)
    assert np.array_equal(Cw, Cn) and np.array_equal(Kw, Kn)
    # the values are the plain product's
    assert np.array_equal(Cw, oracle.gemm(sr, A, B, C))
    # every changed witness attains its value; untouched entries keep K
    changed = Cw != C
    assert np.array_equal(Kw[~changed], K[~changed])


def test_gemm_witness_f32_ties_made_by_rounding():
    """Terms that differ exactly but round to the same binary32 value tie, so
    the smallest index wins; a term that rounds below the others wins."""
    u = np.float32(2.0 ** -24)                  # half the spacing just above 1
    A = np.array([[1.0, 1.0 + 4 * u, 1.0, 1.0]], np.float32)
    C = np.full((1, 1), np.inf, np.float32)
    K = np.full((1, 1), -1, np.int32)
    # terms RN(1 + u/2) = 1, 1 + 4u, RN(1 + u/4) = 1, RN(1 - u/2) = 1 (a tie
    # between 1 - u and 1, to even): four terms, three equal to 1 -> index 0
    B = np.array([[u / 2], [0.0], [u / 4], [-u / 2]], np.float32)
    Cw, Kw = oracle.gemm_witness("min", A, B, C, K)
    assert Cw[0, 0] == 1.0 and Kw[0, 0] == 0
    # 1 - u is representable and below 1: the last term wins
    B[3, 0] = -u
    Cw, Kw = oracle.gemm_witness("min", A, B, C, K)
    assert Cw[0, 0] == np.float32(1.0) - u and Kw[0, 0] == 3
    # max-plus: RN(1 + 4u) is the largest
    Cm = np.full((1, 1), -np.inf, np.float32)
    Cw, Kw = oracle.gemm_witness("max", A, B, Cm, K)
    assert Cw[0, 0] == np.float32(1.0) + 4 * u and Kw[0, 0] == 1


@pytest.mark.parametrize("sr", SR)
def test_gemm_witness_no_change_keeps_k_and_absent_terms_never_win(sr):
    dt = "i32"
    A = np.full((3, 4), _absent(dt, sr), np.int32)
    B = np.zeros((4, 2), np.int32)
    C = np.array([[5, _absent(dt, sr)]] * 3, np.int32)
    K = np.array([[7, 8]] * 3, np.int32)
    Cw, Kw = oracle.gemm_witness(sr, A, B, C, K)
    assert np.array_equal(Cw, C) and np.array_equal(Kw, K)
    # k = 0: nothing changes
    Cw, Kw = oracle.gemm_witness(sr, A[:, :0], B[:0], C, K)
    assert np.array_equal(Cw, C) and np.array_equal(Kw, K)


def _walk(S, i, j, limit):
    path = [i]
    while path[-1] != j and len(path) <= limit:
        nxt = int(S[path[-1], j])
        if nxt < 0:
            return None
        path.append(nxt)
    return path if path[-1] == j else None


@pytest.mark.parametrize("seed", range(8))
def test_successors_tiny_bruteforce(seed):
    """Positive weights: S_ij is the smallest neighbour u with
    w(i,u) + d(u,j) = d(i,j), d by simple-path enumeration."""
    g = np.random.default_rng(seed)
    n = int(g.integers(1, 8))
    W = wl.er_digraph_i32(n, 0.45, 1, 6, seed=300 + seed)
    D, _, _ = oracle.apsp(W)
    S = oracle.successors(W, D)
    d = oracle.brute_force_apsp(W.tolist(), INF32)
    for i in range(n):
        assert S[i, i] == i
        for j in range(n):
            if i == j:
                continue
            cands = [u for u in range(n) if u != i and W[i, u] != INF32 and d[u][j] != INF32
                     and W[i, u] + d[u][j] == d[i][j]]
            assert S[i, j] == (min(cands) if d[i][j] != INF32 else -1), (i, j)


@pytest.mark.parametrize("n,p", [(50, 0.1), (200, 0.03)])
def test_successors_i32_paths_are_shortest(n, p):
    """Following S from i reaches j in < n hops, the weights along the walk
    sum exactly to d(i,j) (scipy Dijkstra), and S_ij = -1 exactly where j is
    unreachable; S also equals numpy's first argmin of W' + D."""
    W = wl.er_digraph_i32(n, p, 1, 1000, seed=n)
    D, _, _ = oracle.apsp(W)
    S = oracle.successors(W, D)
    ref = _dijkstra(W)
    for i in range(n):
        for j in range(n):
            if not np.isfinite(ref[i, j]):
                assert S[i, j] == -1
                continue
            path = _walk(S, i, j, n)
            assert path is not None, (i, j)
            assert sum(int(W[a, b]) for a, b in zip(path, path[1:])) == ref[i, j]
    Wp = W.copy()
    np.fill_diagonal(Wp, INF32)
    _, Kn = _witness_numpy("min", Wp, D, np.full((n, n), INF32, np.int32),
                           np.full((n, n), -1, np.int32))
    np.fill_diagonal(Kn, np.arange(n))
    assert np.array_equal(S, Kn)


def test_successors_f32_integer_weights_match_int32():
    """Integer-valued binary32 weights: every sum is exact, so the float
    successors equal the integer ones."""
    n = 120
    Wi = wl.er_digraph_i32(n, 0.05, 1, 100, seed=12)
    Wf = np.where(Wi == INF32, np.inf, Wi).astype(np.float32)
    Si = oracle.successors(Wi, oracle.apsp(Wi)[0])
    Sf = oracle.successors(Wf, oracle.apsp(Wf)[0])
    assert np.array_equal(Si, Sf)


def test_successors_f32_general_weights_walks_reach_target():
    """Exponential weights: every walk reaches its target, and its fp64 length
    is within the rounding bound of the fp64 Dijkstra distance."""
    n = 160
    r, c, w = wl.sparse_digraph_f32_exp(n, 5.0, seed=21)
    W = wl.coo_to_dense_f32(n, r, c, w)
    D, steps, _ = oracle.apsp(W)
    S = oracle.successors(W, D)
    ref = _dijkstra(W)
    u = 2.0 ** -24
    for i in range(n):
        for j in range(n):
            if i == j or not np.isfinite(ref[i, j]):
                assert S[i, j] == (i if i == j else -1)
                continue
            path = _walk(S, i, j, n)
            assert path is not None, (i, j)
            length = sum(float(W[a, b]) for a, b in zip(path, path[1:]))
            assert ref[i, j] <= length <= ref[i, j] * (1 + u) ** (2 * steps + 2) * (1 + u) ** len(path)


# ------------------------------------------------- max-plus applications ---

def _random_dag_i32(n, p, lo, hi, seed):
    """Edges only from lower to higher index (acyclic); absent = NINF32."""
    g = np.random.default_rng(seed)
    W = np.full((n, n), NINF32, np.int32)
    mask = np.triu(g.random((n, n)) < p, 1)
    W[mask] = g.integers(lo, hi + 1, mask.sum())
    return W


def _dag_longest_dp(W):
    """Longest paths of a DAG with edges i < j by dynamic programming in
    reverse topological order (a textbook method, exact in Python ints)."""
    n = W.shape[0]
    L = [[None] * n for _ in range(n)]
    for i in range(n - 1, -1, -1):
        L[i][i] = 0
        for k in range(i + 1, n):
            if W[i, k] == NINF32:
                continue
            for j in range(k, n):
                if L[k][j] is not None:
                    cand = int(W[i, k]) + L[k][j]
                    if L[i][j] is None or cand > L[i][j]:
                        L[i][j] = cand
    return np.array([[NINF32 if x is None else x for x in row] for row in L], np.int64)


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("n", [1, 2, 17, 64])
def test_closure_min_plus_is_apsp(dt, n):
    W = wl.er_digraph_i32(n, min(1.0, 4.0 / n), 1, 100, seed=n)
    if dt == "f32":
        W = np.where(W == INF32, np.inf, W * 0.37).astype(np.float32)
        np.fill_diagonal(W, 0)
    for ee in (False, True):
        D, s, _ = oracle.closure("min", W, early_exit=ee)
        D2, s2, _ = oracle.apsp(W, early_exit=ee)
        assert s == s2 and np.array_equal(D.view(np.uint32), D2.view(np.uint32))


@pytest.mark.parametrize("n,p", [(12, 0.4), (60, 0.1), (150, 0.05)])
def test_closure_max_plus_dag_equals_dp(n, p):
    W = _random_dag_i32(n, p, -20, 100, seed=n)
    D, steps, st = oracle.closure("max", W, check=True)
    assert st == oracle.OK and steps == oracle.apsp_steps(n)
    assert np.array_equal(D.astype(np.int64), _dag_longest_dp(W))


@pytest.mark.parametrize("seed", range(5))
def test_closure_max_plus_tiny_bruteforce(seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(1, 7))
    W = _random_dag_i32(n, 0.5, -5, 9, seed=40 + seed)
    D, _, _ = oracle.closure("max", W)
    for i in range(n):
        for j in range(n):
            best = None

            def walk(v, acc, seen):
                nonlocal best
                if v == j and (best is None or acc > best):
                    best = acc
                for u in range(n):
                    if u not in seen and W[v, u] != NINF32:
                        walk(u, acc + int(W[v, u]), seen | {u})
            walk(i, 0, {i})
            assert D[i, j] == (NINF32 if best is None else best), (i, j)


@pytest.mark.parametrize("dt", DT)
def test_closure_max_min_duality(dt):
    """max-plus closure of W = -(min-plus closure of -W), absent values
    swapped: negation is exact and commutes with rounding to nearest."""
    n = 90
    Wi = _random_dag_i32(n, 0.08, -50, 200, seed=3)
    if dt == "i32":
        W = Wi
        neg = np.where(W == NINF32, INF32, -W.astype(np.int64)).astype(np.int32)
        Dmax, s1, _ = oracle.closure("max", W, early_exit=True)
        Dmin, s2, _ = oracle.closure("min", neg, early_exit=True)
        back = np.where(Dmin == INF32, NINF32, -Dmin.astype(np.int64)).astype(np.int32)
    else:
        g = np.random.default_rng(4)
        W = np.where(Wi == NINF32, -np.inf, Wi * g.random((n, n))).astype(np.float32)
        Dmax, s1, _ = oracle.closure("max", W, early_exit=True)
        Dmin, s2, _ = oracle.closure("min", -W, early_exit=True)
        back = -Dmin
    assert s1 == s2
    assert np.array_equal(Dmax, back)


def test_closure_max_plus_positive_cycle_flag_and_critical_path():
    # chain 0 -> 1 -> ... -> 5 with durations: the critical path is the sum
    n = 6
    W = np.full((n, n), NINF32, np.int32)
    dur = [3, 1, 4, 1, 5]
    for i, d in enumerate(dur):
        W[i, i + 1] = d
    W[0, 5] = 10                              # a shortcut shorter than the chain
    D, _, st = oracle.closure("max", W, check=True)
    assert st == oracle.OK and D[0, 5] == sum(dur) and D[5, 0] == NINF32
    W[5, 0] = 1                               # closes a positive cycle
    _, _, st = oracle.closure("max", W, check=True)
    assert st == oracle.WNEGCYCLE


def _cycle_mean_bruteforce(A):
    from fractions import Fraction
    n = A.shape[0]
    best = None
    def walk(start, v, acc, length, seen):
        nonlocal best
        for u in range(n):
            if A[v, u] == NINF32:
                continue
            if u == start:
                m = Fraction(acc + int(A[v, u]), length + 1)
                best = m if best is None or m > best else best
            elif u > start and u not in seen:
                walk(start, u, acc + int(A[v, u]), length + 1, seen | {u})
    for s in range(n):
        walk(s, s, 0, 0, {s})
    return best


@pytest.mark.parametrize("seed", range(8))
def test_cycle_mean_tiny_bruteforce(seed):
    """Karp's value equals the best mean over all simple cycles (each cycle
    enumerated once from its smallest vertex), as an exact fraction."""
    from fractions import Fraction
    g = np.random.default_rng(seed)
    n = int(g.integers(1, 7))
    A = np.full((n, n), NINF32, np.int32)
    mask = g.random((n, n)) < 0.45
    A[mask] = g.integers(-9, 10, mask.sum())
    num, den = oracle.cycle_mean(A)
    best = _cycle_mean_bruteforce(A)
    if best is None:
        assert den == 0
    else:
        assert den > 0 and Fraction(num, den) == best and math.gcd(num, den) == 1


def test_cycle_mean_closed_forms_and_f32():
    from fractions import Fraction
    n = 7
    A = np.full((n, n), NINF32, np.int32)
    w = [2, 9, -4, 6, 1, 3, 5]
    for i in range(n):
        A[i, (i + 1) % n] = w[i]             # one cycle through every vertex
    num, den = oracle.cycle_mean(A)
    assert Fraction(num, den) == Fraction(sum(w), n)
    A[3, 3] = 7                               # a self loop with a larger mean
    assert oracle.cycle_mean(A) == (7, 1)
    dag = _random_dag_i32(20, 0.3, -5, 5, seed=1)
    assert oracle.cycle_mean(dag)[1] == 0     # acyclic: no cycle
    full = np.full((5, 5), 4, np.int32)
    assert Fraction(*oracle.cycle_mean(full)) == 4
    # float32 with integer weights: the same value, rounded once to binary64
    g = np.random.default_rng(9)
    Ai = np.full((40, 40), NINF32, np.int32)
    mask = g.random((40, 40)) < 0.08
    Ai[mask] = g.integers(-100, 100, mask.sum())
    num, den = oracle.cycle_mean(Ai)
    Af = np.where(Ai == NINF32, -np.inf, Ai).astype(np.float32)
    lam = oracle.cycle_mean(Af)
    assert (den == 0 and lam == -np.inf) or lam == num / den
