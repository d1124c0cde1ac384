"""CPU oracle for tropical linear algebra and APSP by repeated squaring.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the library.  It wraps the plain C
implementation in ``oracle.c`` (exact int64 arithmetic for int32 data, binary64
arithmetic rounded once to binary32 for float32 data) and adds the pure-Python
brute-force path enumeration used to pin it on tiny graphs.

Semirings follow Sec. I, eqs. (1)-(4); the product follows the min-plus form
of the matrix-product listing in Sec. IV; repeated squaring follows Sec. III;
Floyd-Warshall follows Algorithm 2 of Sec. IV.

Sentinels are this module's own: ``INF32 = 0x7FFFFFFF`` (min-plus absent value)
and ``NINF32 = -0x7FFFFFFF`` (max-plus absent value).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

INF32 = 0x7FFFFFFF
NINF32 = -0x7FFFFFFF
FINITE_MAX = (1 << 29) - 1

OK, EARG, EDOMAIN, WNEGCYCLE = 0, 1, 2, 3
SEMIRINGS = {"min": 0, "max": 1}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class OracleError(RuntimeError):
    pass


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: F401  (build script lives beside)
            _b.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L = ctypes.c_long
        I = ctypes.c_int
        for name in ("or_gemm_i32", "or_gemm_f32"):
            getattr(lib, name).argtypes = [I, L, L, L, P, L, P, L, P, L]
        for name in ("or_gemv_i32", "or_gemv_f32"):
            getattr(lib, name).argtypes = [I, L, L, P, L, P, L, P, L]
        for name in ("or_vadd_i32", "or_vadd_f32", "or_vmul_i32", "or_vmul_f32"):
            getattr(lib, name).argtypes = [I, L, P, L, P, L, P, L]
        for name in ("or_dot_i32", "or_dot_f32"):
            getattr(lib, name).argtypes = [I, L, P, L, P, L, P]
        lib.or_axpy_i32.argtypes = [I, L, ctypes.c_int32, P, L, P, L]
        lib.or_axpy_f32.argtypes = [I, L, ctypes.c_float, P, L, P, L]
        for name in ("or_apsp_i32", "or_apsp_f32"):
            getattr(lib, name).argtypes = [L, P, L, P, L, I, I, ctypes.POINTER(I)]
        lib.or_fw_i32.argtypes = [L, P, L, P, L]
        lib.or_fw_f64.argtypes = [L, P, L, P, L]
        lib.or_fw_blocked_i32.argtypes = [L, P, L, P, L, L]
        lib.or_fw_blocked_f32.argtypes = [L, P, L, P, L, L]
        for name in ("or_gemm_witness_i32", "or_gemm_witness_f32"):
            getattr(lib, name).argtypes = [I, L, L, L, P, L, P, L, P, L, P, L]
        for name in ("or_successors_i32", "or_successors_f32"):
            getattr(lib, name).argtypes = [L, P, L, P, L, P, L]
        for name in ("or_closure_i32", "or_closure_f32"):
            getattr(lib, name).argtypes = [I, L, P, L, P, L, I, I, ctypes.POINTER(I)]
        lib.or_cycle_mean_i32.argtypes = [L, P, L, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int64)]
        lib.or_cycle_mean_f32.argtypes = [L, P, L, ctypes.POINTER(ctypes.c_double)]
        lib.or_apsp_steps.argtypes = [L]
        lib.or_num_threads.restype = I
        lib.or_set_num_threads.argtypes = [I]
        _LIB = lib
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(status: int, what: str, allow=(OK,)) -> int:
    if status not in allow:
        raise OracleError(f"{what}: oracle status {status}")
    return status


def _sfx(dtype) -> str:
    dt = np.dtype(dtype)
    if dt == np.int32:
        return "i32"
    if dt == np.float32:
        return "f32"
    raise TypeError(f"oracle supports int32 and float32, not {dt}")


def _mat(x: np.ndarray) -> np.ndarray:
    """A row-major view with unit column stride (leading dimension = strides[0])."""
    if x.ndim != 2:
        raise ValueError("expected a matrix")
    if x.strides[1] != x.itemsize or x.strides[0] % x.itemsize or x.strides[0] < 0:
        x = np.ascontiguousarray(x)
    return x


def _ld(x: np.ndarray) -> int:
    return max(1, x.strides[0] // x.itemsize) if x.shape[0] > 0 else max(1, x.shape[1])


def num_threads() -> int:
    return _lib().or_num_threads()


def set_num_threads(t: int) -> None:
    _lib().or_set_num_threads(int(t))


def apsp_steps(n: int) -> int:
    """T = ceil(log2(n-1)) computed in integers; 0 for n <= 2 (Sec. III)."""
    return _lib().or_apsp_steps(int(n))


def gemm(semiring: str, A: np.ndarray, B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Return C (+) A (.) B (C is not modified)."""
    A, B = _mat(A), _mat(B)
    if A.dtype != B.dtype or A.dtype != C.dtype:
        raise TypeError("dtype mismatch")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or C.shape != (m, n):
        raise ValueError("shape mismatch")
    out = np.array(C, dtype=C.dtype, order="C", copy=True)
    fn = getattr(_lib(), "or_gemm_" + _sfx(A.dtype))
    _check(fn(SEMIRINGS[semiring], m, n, k, _ptr(A), _ld(A), _ptr(B), _ld(B),
              _ptr(out), max(1, n)), "gemm")
    return out


def gemm_witness(semiring: str, A: np.ndarray, B: np.ndarray, C: np.ndarray,
                 K: np.ndarray):
    """Return (C', K') for C' = C (+) A (.) B: where C'_ij strictly improves on
    C_ij, K'_ij is the smallest p with A_ip (.) B_pj = C'_ij; elsewhere C and K
    are kept (neither input is modified)."""
    A, B = _mat(A), _mat(B)
    if A.dtype != B.dtype or A.dtype != C.dtype:
        raise TypeError("dtype mismatch")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or C.shape != (m, n) or K.shape != (m, n):
        raise ValueError("shape mismatch")
    out = np.array(C, dtype=C.dtype, order="C", copy=True)
    kout = np.array(K, dtype=np.int32, order="C", copy=True)
    fn = getattr(_lib(), "or_gemm_witness_" + _sfx(A.dtype))
    _check(fn(SEMIRINGS[semiring], m, n, k, _ptr(A), _ld(A), _ptr(B), _ld(B),
              _ptr(out), max(1, n), _ptr(kout), max(1, n)), "gemm_witness")
    return out, kout


def successors(W: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Successor matrix: S_ii = i; for i != j the smallest u != i minimising
    W_iu (.) D_uj (min-plus), -1 if every such term is absent."""
    W, D = _mat(W), _mat(D)
    n = W.shape[0]
    if W.shape != (n, n) or D.shape != (n, n) or W.dtype != D.dtype:
        raise ValueError("W and D must be square, same shape and dtype")
    S = np.empty((n, n), dtype=np.int32)
    fn = getattr(_lib(), "or_successors_" + _sfx(W.dtype))
    _check(fn(n, _ptr(W), max(1, _ld(W)), _ptr(D), max(1, _ld(D)), _ptr(S), max(1, n)),
           "successors")
    return S


def gemv(semiring: str, A: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Return y (+) A (.) x for contiguous vectors."""
    A = _mat(A)
    x = np.ascontiguousarray(x)
    out = np.array(y, copy=True)
    m, n = A.shape
    fn = getattr(_lib(), "or_gemv_" + _sfx(A.dtype))
    _check(fn(SEMIRINGS[semiring], m, n, _ptr(A), _ld(A), _ptr(x), 1, _ptr(out), 1), "gemv")
    return out


def vadd(semiring: str, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    x, y = np.ascontiguousarray(x), np.ascontiguousarray(y)
    z = np.empty_like(x)
    fn = getattr(_lib(), "or_vadd_" + _sfx(x.dtype))
    _check(fn(SEMIRINGS[semiring], x.size, _ptr(x), 1, _ptr(y), 1, _ptr(z), 1), "vadd")
    return z


def vmul(semiring: str, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    x, y = np.ascontiguousarray(x), np.ascontiguousarray(y)
    z = np.empty_like(x)
    fn = getattr(_lib(), "or_vmul_" + _sfx(x.dtype))
    _check(fn(SEMIRINGS[semiring], x.size, _ptr(x), 1, _ptr(y), 1, _ptr(z), 1), "vmul")
    return z


def dot(semiring: str, x: np.ndarray, y: np.ndarray):
    x, y = np.ascontiguousarray(x), np.ascontiguousarray(y)
    r = np.zeros(1, dtype=x.dtype)
    fn = getattr(_lib(), "or_dot_" + _sfx(x.dtype))
    _check(fn(SEMIRINGS[semiring], x.size, _ptr(x), 1, _ptr(y), 1, _ptr(r)), "dot")
    return r[0]


def axpy(semiring: str, alpha, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Return y (+) alpha (.) x."""
    x = np.ascontiguousarray(x)
    out = np.array(y, copy=True)
    sfx = _sfx(x.dtype)
    fn = getattr(_lib(), "or_axpy_" + sfx)
    a = int(alpha) if sfx == "i32" else float(alpha)
    _check(fn(SEMIRINGS[semiring], x.size, a, _ptr(x), 1, _ptr(out), 1), "axpy")
    return out


def apsp(W: np.ndarray, early_exit: bool = False, check_neg_cycle: bool = False):
    """Repeated min-plus squaring of I (+) W.  Returns (D, steps, status)."""
    W = _mat(W)
    n = W.shape[0]
    if W.shape != (n, n):
        raise ValueError("W must be square")
    D = np.empty((n, n), dtype=W.dtype)
    steps = ctypes.c_int(0)
    fn = getattr(_lib(), "or_apsp_" + _sfx(W.dtype))
    st = fn(n, _ptr(W), max(1, _ld(W)), _ptr(D), max(1, n), int(early_exit),
            int(check_neg_cycle), ctypes.byref(steps))
    _check(st, "apsp", allow=(OK, WNEGCYCLE))
    return D, steps.value, st


def closure(semiring: str, W: np.ndarray, early_exit: bool = False, check: bool = False):
    """(I (+) W)^(2^s) by repeated squaring over the given semiring (min-plus:
    shortest distances; max-plus: heaviest walks, the longest paths of a
    graph without positive cycles).  Returns (D, steps, status)."""
    W = _mat(W)
    n = W.shape[0]
    if W.shape != (n, n):
        raise ValueError("W must be square")
    D = np.empty((n, n), dtype=W.dtype)
    steps = ctypes.c_int(0)
    fn = getattr(_lib(), "or_closure_" + _sfx(W.dtype))
    st = fn(SEMIRINGS[semiring], n, _ptr(W), max(1, _ld(W)), _ptr(D), max(1, n), int(early_exit),
            int(check), ctypes.byref(steps))
    _check(st, "closure", allow=(OK, WNEGCYCLE))
    return D, steps.value, st


def cycle_mean(A: np.ndarray):
    """Maximum cycle mean of a max-plus matrix (Karp).  int32: (num, den)
    exactly, den = 0 when there is no cycle; float32: a float (-inf: none)."""
    A = _mat(A)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("A must be square")
    if A.dtype == np.int32:
        num, den = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(_lib().or_cycle_mean_i32(n, _ptr(A), max(1, _ld(A)), ctypes.byref(num),
                                        ctypes.byref(den)), "cycle_mean")
        return num.value, den.value
    lam = ctypes.c_double(0.0)
    _check(_lib().or_cycle_mean_f32(n, _ptr(A), max(1, _ld(A)), ctypes.byref(lam)), "cycle_mean")
    return lam.value


def floyd_warshall(W: np.ndarray) -> np.ndarray:
    """Sequential Floyd-Warshall (Algorithm 2) on I (+) W.

    int32 input: exact int64 arithmetic.  float input: binary64 arithmetic,
    returned as float64 (exact for integer-valued weights whose path sums stay
    below 2^53).
    """
    W = _mat(W)
    n = W.shape[0]
    if W.dtype == np.int32:
        D = np.empty((n, n), dtype=np.int32)
        _check(_lib().or_fw_i32(n, _ptr(W), max(1, _ld(W)), _ptr(D), max(1, n)), "fw")
        return D
    W64 = np.ascontiguousarray(W, dtype=np.float64)
    D = np.empty((n, n), dtype=np.float64)
    _check(_lib().or_fw_f64(n, _ptr(W64), max(1, n), _ptr(D), max(1, n)), "fw")
    return D


def floyd_warshall_blocked(W: np.ndarray, block: int = 64) -> np.ndarray:
    """Three-phase blocked Floyd-Warshall on I (+) W with pivot blocks of
    `block` vertices, in the input's dtype (int32 exact; fp32 one rounding per
    relaxation).  The fp32 result is defined by this order and block size."""
    W = _mat(W)
    n = W.shape[0]
    if W.shape != (n, n):
        raise ValueError("W must be square")
    D = np.empty((n, n), dtype=W.dtype)
    fn = getattr(_lib(), "or_fw_blocked_" + _sfx(W.dtype))
    _check(fn(n, _ptr(W), max(1, _ld(W)), _ptr(D), max(1, n), int(block)), "fw_blocked")
    return D


from .brute import brute_force_apsp  # noqa: E402,F401
