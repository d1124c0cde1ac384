"""Python binding of libbtas: tropical GEMM / gemv / level-1 and APSP on MI355X.

Thin ctypes marshalling over the C ABI declared in ``include/btas.h``: torch
tensors supply device pointers, leading dimensions and the current HIP
stream; every step of the computation runs in the HIP kernels of libbtas.
There is no CPU fallback: if ``libbtas.so`` is missing or no GPU is present,
calls raise.

Semirings (Sec. I, eqs. (1)-(4)): ``"min"`` (min-plus) and ``"max"``
(max-plus).  Element types: ``torch.int32`` (saturating +-INF sentinels
``I32_INF`` / ``I32_NEG_INF``) and ``torch.float32`` (IEEE +-inf).
"""
from __future__ import annotations

import atexit
import ctypes
import os
import threading
import weakref

__all__ = [
    "I32_INF", "I32_NEG_INF", "I32_FINITE_MAX", "BtasError", "lib", "library_path",
    "Handle", "default_handle", "tropical_gemm", "tropical_gemv", "vadd", "vmul", "dot",
    "axpy", "apsp", "apsp_num_steps", "version", "apsp_batched", "BatchedAPSP", "Server",
    "close_all", "apsp_noalloc", "NOALLOC_MAX_N",
]

I32_INF = 0x7FFFFFFF
I32_NEG_INF = -0x7FFFFFFF
I32_FINITE_MAX = (1 << 29) - 1

MIN_PLUS, MAX_PLUS = 0, 1
INT32, FLOAT32 = 0, 1
APSP_EARLY_EXIT, APSP_CHECK_NEG_CYCLE, APSP_GRAPH, APSP_SINGLE_LAUNCH = 1, 2, 4, 8

STATUS = {0: "BTAS_OK", 1: "BTAS_ERR_INVALID_ARG", 2: "BTAS_ERR_ALIAS", 3: "BTAS_ERR_DOMAIN",
          4: "BTAS_ERR_OOM", 5: "BTAS_ERR_DEVICE", 6: "BTAS_ERR_UNSUPPORTED",
          7: "BTAS_WARN_NEG_CYCLE", 8: "BTAS_WARN_POS_CYCLE"}
OK, WARN_NEG_CYCLE, WARN_POS_CYCLE = 0, 7, 8

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libbtas.so")
_LIB = None
_LOCK = threading.Lock()

# Handles and servers still open at interpreter exit are closed by an atexit
# hook, servers first (each owns a handle and a worker thread), while torch
# and the HIP runtime are still up: destroying them later, from __del__
# during module teardown, would synchronise streams and free graphs and
# device memory after the runtime (or a profiler attached to it) has begun
# its own shutdown.  The hook is registered on the first open, after torch
# has been imported, so that it runs before torch's own exit hooks.
_LIVE = weakref.WeakSet()
_ATEXIT_DONE = False


def _track(obj):
    global _ATEXIT_DONE
    with _LOCK:
        _LIVE.add(obj)
        if not _ATEXIT_DONE:
            atexit.register(close_all)
            _ATEXIT_DONE = True


def close_all():
    """Close every open Server, then every open Handle (idempotent)."""
    objs = list(_LIVE)
    for o in objs:
        if isinstance(o, Server):
            o.close()
    for o in objs:
        if isinstance(o, Handle):
            o.close()
    _HANDLES.clear()


class ServerStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_long), ("launches", ctypes.c_long),
                ("busy_seconds", ctypes.c_double), ("pool_bytes", ctypes.c_size_t),
                ("pool_used_bytes", ctypes.c_size_t), ("pool_peak_bytes", ctypes.c_size_t),
                ("active", ctypes.c_int), ("pending", ctypes.c_int)]


class BtasError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def lib():
    """Load libbtas.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    with _LOCK:
        if _LIB is not None:
            return _LIB
        if not os.path.exists(library_path):
            raise RuntimeError(f"libbtas.so not found at {library_path}; run "
                               "python -m paper_1701_04733_amd.build")
        L = ctypes.CDLL(library_path)
        P, I, U = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint
        L.btas_create.argtypes = [ctypes.POINTER(P), I]
        L.btas_destroy.argtypes = [P]
        L.btas_set_stream.argtypes = [P, P]
        L.btas_synchronize.argtypes = [P]
        L.btas_status_string.argtypes = [I]
        L.btas_status_string.restype = ctypes.c_char_p
        L.btas_last_error.argtypes = [P]
        L.btas_last_error.restype = ctypes.c_char_p
        L.btas_version.restype = ctypes.c_char_p
        L.btas_tropical_gemm.argtypes = [P, I, I, I, I, I, P, I, P, I, P, I]
        L.btas_tropical_gemv.argtypes = [P, I, I, I, I, P, I, P, I, P, I]
        for name in ("btas_tropical_vadd", "btas_tropical_vmul"):
            getattr(L, name).argtypes = [P, I, I, I, P, I, P, I, P, I]
        L.btas_tropical_dot.argtypes = [P, I, I, I, P, I, P, I, P]
        L.btas_tropical_axpy.argtypes = [P, I, I, I, P, P, I, P, I]
        L.btas_apsp_squaring.argtypes = [P, I, I, P, I, P, I, U, ctypes.POINTER(I)]
        L.btas_apsp_num_steps.argtypes = [I]
        L.btas_apsp_squaring_noalloc.argtypes = [P, I, I, P, I, P, I, U, ctypes.POINTER(I)]
        L.btas_apsp_last_packed16.argtypes = [P]
        IP = ctypes.POINTER(I)
        PP = ctypes.POINTER(P)
        L.btas_apsp_squaring_batched.argtypes = [P, I, I, IP, PP, IP, PP, IP, U]
        L.btas_batched_plan_info.argtypes = [P, IP, ctypes.POINTER(ctypes.c_double)]
        L.btas_batched_tile_choice.argtypes = [P, I, I]
        L.btas_apsp_floyd_warshall.argtypes = [P, I, I, P, I, P, I, U]
        L.btas_tropical_gemm_witness.argtypes = [P, I, I, I, I, I, P, I, P, I, P, I, P, I]
        L.btas_apsp_successors.argtypes = [P, I, I, P, I, P, I, P, I]
        L.btas_tropical_closure.argtypes = [P, I, I, I, P, I, P, I, U, ctypes.POINTER(I)]
        L.btas_apsp_floyd_warshall_batched.argtypes = [P, I, I, IP, PP, IP, PP, IP, U]
        I64P = ctypes.POINTER(ctypes.c_int64)
        L.btas_maxplus_cycle_mean.argtypes = [P, I, I, P, I, I64P, I64P, ctypes.POINTER(ctypes.c_double)]
        L.btas_server_create.argtypes = [ctypes.POINTER(P), I, I, ctypes.c_size_t, I, ctypes.c_double]
        L.btas_server_destroy.argtypes = [P]
        L.btas_server_now.argtypes = [P]
        L.btas_server_now.restype = ctypes.c_double
        I64 = ctypes.c_int64
        L.btas_server_submit.argtypes = [P, I, I, P, P, P, U, ctypes.c_double, ctypes.POINTER(I64)]
        L.btas_server_wait.argtypes = [P, I64, ctypes.c_double, IP]
        L.btas_server_result.argtypes = [P, I64, ctypes.POINTER(P), IP, IP]
        L.btas_server_copy_result.argtypes = [P, I64, P, I]
        D = ctypes.c_double
        L.btas_server_times.argtypes = [P, I64, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)]
        L.btas_server_release.argtypes = [P, I64]
        L.btas_server_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
        _LIB = L
    return _LIB


def version() -> str:
    return lib().btas_version().decode()


def apsp_num_steps(n: int) -> int:
    """T = ceil(log2(n-1)) for n > 2, else 0 (Sec. III)."""
    return lib().btas_apsp_num_steps(int(n))


class Handle:
    """One libbtas handle bound to a device; follows torch's current stream."""

    def __init__(self, device: int = 0):
        self.device = int(device)
        h = ctypes.c_void_p()
        st = lib().btas_create(ctypes.byref(h), self.device)
        if st != OK:
            raise BtasError(st, f"btas_create(device={device}) failed")
        self._h = h
        self._bound = None  # the stream last handed to btas_set_stream
        _track(self)

    @property
    def ptr(self):
        return self._h

    def bind_stream(self, stream=None):
        """Make the handle launch on ``stream`` (torch's current stream of the
        handle's device if None); skips the library call when unchanged."""
        raw = stream.cuda_stream if stream is not None else _current_raw_stream(self.device)
        if raw != self._bound:
            lib().btas_set_stream(self._h, ctypes.c_void_p(raw))
            self._bound = raw

    def check(self, st: int, allow=(OK,)) -> int:
        if st not in allow:
            msg = lib().btas_last_error(self._h).decode()
            raise BtasError(st, msg)
        return st

    def synchronize(self):
        """Wait for the handle's stream; raises BTAS_ERR_DEVICE if an earlier
        asynchronous single-launch solve on this handle timed out waiting on
        other workgroups."""
        self.check(lib().btas_synchronize(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().btas_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_HANDLES: dict = {}
_RAW_STREAM = None


def _current_raw_stream(device: int) -> int:
    """torch's current stream on ``device`` as a raw pointer value."""
    global _RAW_STREAM
    if _RAW_STREAM is None:
        import torch
        fast = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        _RAW_STREAM = fast if fast is not None else (lambda d: torch.cuda.current_stream(d).cuda_stream)
    return _RAW_STREAM(device)


def default_handle(device: int | None = None) -> Handle:
    import torch
    if device is None:
        device = torch.cuda.current_device()
    h = _HANDLES.get(device)
    if h is None:
        h = _HANDLES[device] = Handle(device)
    h.bind_stream()
    return h


# ------------------------------------------------------------ marshalling ---

def _sr(semiring) -> int:
    if semiring in ("min", MIN_PLUS):
        return MIN_PLUS
    if semiring in ("max", MAX_PLUS):
        return MAX_PLUS
    raise ValueError(f"semiring must be 'min' or 'max', not {semiring!r}")


def _dt(t) -> int:
    import torch
    if t.dtype == torch.int32:
        return INT32
    if t.dtype == torch.float32:
        return FLOAT32
    raise TypeError(f"btas supports int32 and float32 tensors, not {t.dtype}")


def _mat(t, name):
    if t.dim() != 2:
        raise ValueError(f"{name} must be a matrix")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    rows, cols = t.shape
    if rows == 0 or cols == 0:
        return ctypes.c_void_p(t.data_ptr() or None), max(1, cols)
    s0, s1 = t.stride()
    if cols > 1 and s1 != 1:
        raise ValueError(f"{name} must have unit column stride (row-major with leading dimension)")
    ld = s0 if rows > 1 else max(1, cols)
    return ctypes.c_void_p(t.data_ptr()), max(1, ld)


def _vec(t, name):
    if t.dim() != 1:
        raise ValueError(f"{name} must be a vector")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.numel() == 0:
        return ctypes.c_void_p(t.data_ptr() or None), 1
    return ctypes.c_void_p(t.data_ptr()), max(1, t.stride(0))


def _handle_for(t, handle):
    return handle if handle is not None else default_handle(max(t.get_device(), 0))


def tropical_gemm(A, B, C=None, semiring="min", handle=None):
    """C <- C (+) A (.) B on the device (C allocated as the (+)-identity if None)."""
    import torch
    sr = _sr(semiring)
    if C is None:
        fill = (I32_INF if sr == MIN_PLUS else I32_NEG_INF) if A.dtype == torch.int32 else \
            (float("inf") if sr == MIN_PLUS else float("-inf"))
        C = torch.full((A.size(0), B.size(1)), fill, dtype=A.dtype, device=A.device)
    if A.dtype != B.dtype or A.dtype != C.dtype:
        raise TypeError("A, B and C must share a dtype")
    h = _handle_for(C, handle)
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pc, ldc = _mat(C, "C")
    m, k = A.shape
    if B.size(0) != k or C.shape != (m, B.size(1)):
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}")
    h.check(lib().btas_tropical_gemm(h.ptr, sr, _dt(A), m, B.size(1), k, pa, lda, pb, ldb, pc, ldc))
    return C


def tropical_gemm_witness(A, B, C=None, K=None, semiring="min", handle=None):
    """C <- C (+) A (.) B and, where an entry strictly improves, K <- the
    smallest p attaining it (C starts as the (+)-identity and K as -1 when
    None).  Returns (C, K)."""
    import torch
    sr = _sr(semiring)
    m, n = A.size(0), B.size(1)
    if C is None:
        fill = (I32_INF if sr == MIN_PLUS else I32_NEG_INF) if A.dtype == torch.int32 else \
            (float("inf") if sr == MIN_PLUS else float("-inf"))
        C = torch.full((m, n), fill, dtype=A.dtype, device=A.device)
    if K is None:
        K = torch.full((m, n), -1, dtype=torch.int32, device=A.device)
    if A.dtype != B.dtype or A.dtype != C.dtype or K.dtype != torch.int32:
        raise TypeError("A, B and C must share a dtype and K must be int32")
    h = _handle_for(C, handle)
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pc, ldc = _mat(C, "C")
    pk, ldk = _mat(K, "K")
    k = A.size(1)
    if B.size(0) != k or C.shape != (m, n) or K.shape != (m, n):
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, "
                         f"C {tuple(C.shape)}, K {tuple(K.shape)}")
    h.check(lib().btas_tropical_gemm_witness(h.ptr, sr, _dt(A), m, n, k, pa, lda, pb, ldb,
                                             pc, ldc, pk, ldk))
    return C, K


def apsp_successors(W, D, out=None, handle=None):
    """Successor matrix S of a solved distance matrix D of W (min-plus):
    S_ii = i; S_ij = the smallest u != i minimising W_iu (.) D_uj, -1 if
    every term is absent."""
    import torch
    n = W.size(0)
    if W.shape != (n, n) or D.shape != (n, n) or W.dtype != D.dtype:
        raise ValueError("W and D must be square, of one shape and dtype")
    if out is None:
        out = torch.empty((n, n), dtype=torch.int32, device=W.device)
    if out.dtype != torch.int32 or out.shape != (n, n):
        raise TypeError("out must be an n x n int32 tensor")
    h = _handle_for(W, handle)
    pw, ldw = _mat(W, "W")
    pd, ldd = _mat(D, "D")
    ps, lds = _mat(out, "S")
    h.check(lib().btas_apsp_successors(h.ptr, _dt(W), n, pw, ldw, pd, ldd, ps, lds))
    return out


def tropical_closure(W, semiring="max", out=None, early_exit=False, check_cycle=False,
                     handle=None):
    """(I (+) W)^(2^s) by repeated squaring over the semiring (min: shortest
    distances; max: heaviest walks, the longest paths of a graph without
    positive cycles).  Returns (D, steps, status)."""
    import torch
    n = W.size(0)
    if W.shape != (n, n):
        raise ValueError("W must be square")
    if out is None:
        out = torch.empty_like(W)
    h = _handle_for(W, handle)
    pw, ldw = _mat(W, "W")
    pd, ldd = _mat(out, "D")
    steps = ctypes.c_int(0)
    flags = (APSP_EARLY_EXIT if early_exit else 0) | (APSP_CHECK_NEG_CYCLE if check_cycle else 0)
    st = h.check(lib().btas_tropical_closure(h.ptr, _sr(semiring), _dt(W), n, pw, ldw, pd, ldd, flags,
                                             ctypes.byref(steps)),
                 allow=(OK, WARN_NEG_CYCLE, WARN_POS_CYCLE))
    return out, steps.value, st


def maxplus_cycle_mean(A, handle=None):
    """Maximum cycle mean of a max-plus matrix (Karp).  int32: the exact
    fraction (num, den) in lowest terms, den = 0 when acyclic; float32: a
    float, -inf when acyclic."""
    import torch
    n = A.size(0)
    if A.shape != (n, n):
        raise ValueError("A must be square")
    h = _handle_for(A, handle)
    pa, lda = _mat(A, "A")
    num, den, lam = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_double(0.0)
    h.check(lib().btas_maxplus_cycle_mean(h.ptr, _dt(A), n, pa, lda, ctypes.byref(num),
                                          ctypes.byref(den), ctypes.byref(lam)))
    if A.dtype == torch.int32:
        return num.value, den.value
    return lam.value


def shortest_path(S, i, j):
    """The vertices of the path from i to j read off a successor matrix (a
    host copy, numpy or nested lists); None if j is unreachable."""
    path = [int(i)]
    n = len(S)
    while path[-1] != j:
        nxt = int(S[path[-1]][j])
        if nxt < 0 or len(path) > n:
            return None
        path.append(nxt)
    return path


def tropical_gemv(A, x, y, semiring="min", handle=None):
    """y <- y (+) A (.) x on the device."""
    h = _handle_for(y, handle)
    pa, lda = _mat(A, "A")
    px, incx = _vec(x, "x")
    py, incy = _vec(y, "y")
    m, n = A.shape
    if x.numel() != n or y.numel() != m:
        raise ValueError("shape mismatch")
    h.check(lib().btas_tropical_gemv(h.ptr, _sr(semiring), _dt(A), m, n, pa, lda, px, incx, py, incy))
    return y


def _binary(name, x, y, z, semiring, handle):
    import torch
    if z is None:
        z = torch.empty_like(x)
    h = _handle_for(z, handle)
    px, ix = _vec(x, "x")
    py, iy = _vec(y, "y")
    pz, iz = _vec(z, "z")
    if not (x.numel() == y.numel() == z.numel()):
        raise ValueError("length mismatch")
    h.check(getattr(lib(), name)(h.ptr, _sr(semiring), _dt(x), x.numel(), px, ix, py, iy, pz, iz))
    return z


def vadd(x, y, z=None, semiring="min", handle=None):
    """z = x (+) y."""
    return _binary("btas_tropical_vadd", x, y, z, semiring, handle)


def vmul(x, y, z=None, semiring="min", handle=None):
    """z = x (.) y."""
    return _binary("btas_tropical_vmul", x, y, z, semiring, handle)


def dot(x, y, semiring="min", out=None, handle=None):
    """(+)_i x_i (.) y_i, returned as a one-element device tensor."""
    import torch
    if out is None:
        out = torch.empty(1, dtype=x.dtype, device=x.device)
    h = _handle_for(x, handle)
    px, ix = _vec(x, "x")
    py, iy = _vec(y, "y")
    if x.numel() != y.numel():
        raise ValueError("length mismatch")
    h.check(lib().btas_tropical_dot(h.ptr, _sr(semiring), _dt(x), x.numel(), px, ix, py, iy,
                                    ctypes.c_void_p(out.data_ptr())))
    return out


def axpy(alpha, x, y, semiring="min", handle=None):
    """y <- y (+) alpha (.) x (alpha is a host scalar)."""
    import torch
    h = _handle_for(y, handle)
    if x.dtype == torch.int32:
        a = ctypes.c_int32(int(alpha))
    else:
        a = ctypes.c_float(float(alpha))
    px, ix = _vec(x, "x")
    py, iy = _vec(y, "y")
    if x.numel() != y.numel():
        raise ValueError("length mismatch")
    h.check(lib().btas_tropical_axpy(h.ptr, _sr(semiring), _dt(x), x.numel(),
                                     ctypes.cast(ctypes.byref(a), ctypes.c_void_p), px, ix, py, iy))
    return y


def apsp(W, out=None, early_exit=False, check_neg_cycle=False, return_steps=True, graph=False,
         single_launch=False, handle=None):
    """All-pairs shortest paths by repeated min-plus squaring of I (+) W.

    Returns (D, steps, status); status is OK or WARN_NEG_CYCLE.  With
    ``return_steps=False`` steps is None and the call stays asynchronous unless
    a flag needs the host (early exit on the per-squaring path, the
    negative-cycle check); a device-side failure of such a call (a wait
    timeout of the single-launch solve) is raised by the handle's next call
    or ``synchronize()``.  ``graph`` replays a captured hipGraph of the
    fixed-T solve; ``single_launch`` runs the whole solve as one cooperative
    kernel (n <= 500).  ``out`` may be W itself (in place).
    """
    import torch
    n = W.size(0)
    if W.shape != (n, n):
        raise ValueError("W must be square")
    if out is None:
        out = torch.empty_like(W)
    h = _handle_for(W, handle)
    pw, ldw = _mat(W, "W")
    pd, ldd = _mat(out, "D")
    flags = (APSP_EARLY_EXIT if early_exit else 0) | (APSP_CHECK_NEG_CYCLE if check_neg_cycle else 0) \
        | (APSP_GRAPH if graph else 0) | (APSP_SINGLE_LAUNCH if single_launch else 0)
    steps = ctypes.c_int(0)
    sp = ctypes.byref(steps) if return_steps else None
    st = h.check(lib().btas_apsp_squaring(h.ptr, _dt(W), n, pw, ldw, pd, ldd, flags, sp),
                 allow=(OK, WARN_NEG_CYCLE))
    return out, (steps.value if sp is not None else None), st


NOALLOC_MAX_N = 2896


def apsp_noalloc(W, out, early_exit=False, check_neg_cycle=False, return_steps=True,
                 single_launch=False, handle=None):
    """``apsp`` through the entry point that allocates nothing during the call
    (its workspace is a fixed per-GPU array, n <= NOALLOC_MAX_N); ``out`` must
    be given.  Calls that may overlap in time on one GPU race on that array.
    Returns (D, steps, status) with the same bits as ``apsp``."""
    n = W.size(0)
    if W.shape != (n, n) or out.shape != (n, n) or out.dtype != W.dtype:
        raise ValueError("W and out must be square, of one shape and dtype")
    h = _handle_for(W, handle)
    pw, ldw = _mat(W, "W")
    pd, ldd = _mat(out, "D")
    flags = (APSP_EARLY_EXIT if early_exit else 0) | (APSP_CHECK_NEG_CYCLE if check_neg_cycle else 0) \
        | (APSP_SINGLE_LAUNCH if single_launch else 0)
    steps = ctypes.c_int(0)
    sp = ctypes.byref(steps) if return_steps else None
    st = h.check(lib().btas_apsp_squaring_noalloc(h.ptr, _dt(W), n, pw, ldw, pd, ldd, flags, sp),
                 allow=(OK, WARN_NEG_CYCLE))
    return out, (steps.value if sp is not None else None), st


def apsp_last_packed16(handle=None) -> bool:
    """Whether the handle's last APSP call that returned its step count ran
    the single-launch solve on packed 16-bit distances."""
    import torch
    h = handle if handle is not None else default_handle(torch.cuda.current_device())
    return bool(lib().btas_apsp_last_packed16(h.ptr))


def floyd_warshall(W, out=None, check_neg_cycle=False, handle=None):
    """All-pairs shortest paths of I (+) W by blocked Floyd-Warshall (pivot
    blocks of 64 vertices).  Returns (D, status); ``out`` may be W itself."""
    import torch
    n = W.size(0)
    if W.shape != (n, n):
        raise ValueError("W must be square")
    if out is None:
        out = torch.empty_like(W)
    h = _handle_for(W, handle)
    pw, ldw = _mat(W, "W")
    pd, ldd = _mat(out, "D")
    st = h.check(lib().btas_apsp_floyd_warshall(h.ptr, _dt(W), n, pw, ldw, pd, ldd,
                                                APSP_CHECK_NEG_CYCLE if check_neg_cycle else 0),
                 allow=(OK, WARN_NEG_CYCLE))
    return out, st


class BatchedAPSP:
    """Repeated solves of one fixed set of graphs (same tensors every call).

    The first ``run()`` plans and captures the hipGraph; later calls replay it.
    ``Ws`` and ``Ds`` are lists of square device tensors of one dtype; D[i]
    may be W[i] itself.  ``early_exit``: a graph's later squarings are skipped
    on the device once one leaves it unchanged (same results).
    """

    def __init__(self, Ws, Ds=None, handle=None, early_exit=False):
        import torch
        if not Ws:
            raise ValueError("need at least one graph")
        self.Ws = list(Ws)
        self.Ds = list(Ds) if Ds is not None else [torch.empty_like(w) for w in self.Ws]
        dts = {_dt(w) for w in self.Ws} | {_dt(d) for d in self.Ds}
        if len(dts) != 1:
            raise TypeError("all graphs must share one dtype")
        self.dt = dts.pop()
        self.h = handle if handle is not None else default_handle(self.Ws[0].device.index or 0)
        cnt = len(self.Ws)
        if len(self.Ds) != cnt:
            raise ValueError("Ws and Ds differ in length")
        IA = ctypes.c_int * cnt
        PA = ctypes.c_void_p * cnt
        ns, pw, lw, pd, ld = [], [], [], [], []
        for w, d in zip(self.Ws, self.Ds):
            n = w.size(0)
            if w.shape != (n, n) or d.shape != (n, n):
                raise ValueError("graphs must be square and D must match W")
            a, b = _mat(w, "W")
            c, e = _mat(d, "D")
            ns.append(n); pw.append(a.value); lw.append(b); pd.append(c.value); ld.append(e)
        self._args = (IA(*ns), PA(*pw), IA(*lw), PA(*pd), IA(*ld))
        self.flags = APSP_EARLY_EXIT if early_exit else 0

    def run(self):
        n, pw, lw, pd, ld = self._args
        self.h.check(lib().btas_apsp_squaring_batched(self.h.ptr, self.dt, len(self.Ws), n, pw, lw,
                                                      pd, ld, self.flags))
        return self.Ds

    def plan_info(self):
        launches = ctypes.c_int(0)
        terms = ctypes.c_double(0)
        self.h.check(lib().btas_batched_plan_info(self.h.ptr, ctypes.byref(launches),
                                                  ctypes.byref(terms)))
        return {"launches": launches.value, "terms": terms.value}

    def tile_choice(self, n: int) -> int:
        return lib().btas_batched_tile_choice(self.h.ptr, self.dt, int(n))


def apsp_batched(Ws, Ds=None, handle=None, early_exit=False):
    """Solve every graph in ``Ws`` by repeated squaring in one graph launch."""
    return BatchedAPSP(Ws, Ds, handle, early_exit=early_exit).run()


class FloydWarshallBatched:
    """Repeated blocked Floyd-Warshall solves of one fixed set of graphs
    (square device tensors of one dtype; ``Ds[i]`` may be ``Ws[i]``).  The
    argument arrays are prepared once; the first ``run()`` plans and captures
    the launch sequence, later calls replay it.  int32 results equal the
    squaring's; float32 results equal ``floyd_warshall`` graph by graph.
    Outputs allocated here are, with ``aligned_outputs`` (the default),
    n x n views of n x round_up(n, 4) buffers: rows that start on 16-byte
    boundaries let every update tile use vector loads (the 4096-graph
    workload: 5.6 against 6.0 ms)."""

    def __init__(self, Ws, Ds=None, handle=None, aligned_outputs=True):
        import torch
        if not Ws:
            raise ValueError("need at least one graph")
        self.Ws = list(Ws)
        if Ds is not None:
            self.Ds = list(Ds)
        elif aligned_outputs:
            self.Ds = [torch.empty((w.size(0), (w.size(0) + 3) // 4 * 4), dtype=w.dtype,
                                   device=w.device)[:, :w.size(0)] if w.dim() == 2 else torch.empty_like(w)
                       for w in self.Ws]
        else:
            self.Ds = [torch.empty_like(w) for w in self.Ws]
        dts = {_dt(w) for w in self.Ws} | {_dt(d) for d in self.Ds}
        if len(dts) != 1 or len(self.Ds) != len(self.Ws):
            raise ValueError("one dtype for all graphs, and as many outputs as inputs")
        self.dt = dts.pop()
        self.h = handle if handle is not None else default_handle(self.Ws[0].device.index or 0)
        cnt = len(self.Ws)
        ns, pw, lw, pd, ld = [], [], [], [], []
        for w, d in zip(self.Ws, self.Ds):
            m = w.size(0)
            if w.shape != (m, m) or d.shape != (m, m):
                raise ValueError("graphs must be square and D must match W")
            a, b = _mat(w, "W")
            c, e = _mat(d, "D")
            ns.append(m); pw.append(a.value); lw.append(b); pd.append(c.value); ld.append(e)
        IA = ctypes.c_int * cnt
        PA = ctypes.c_void_p * cnt
        self._args = (IA(*ns), PA(*pw), IA(*lw), PA(*pd), IA(*ld))

    def run(self):
        n, pw, lw, pd, ld = self._args
        self.h.check(lib().btas_apsp_floyd_warshall_batched(self.h.ptr, self.dt, len(self.Ws), n, pw,
                                                            lw, pd, ld, 0))
        return self.Ds


def floyd_warshall_batched(Ws, Ds=None, handle=None):
    """Blocked Floyd-Warshall of every graph in ``Ws`` in one captured launch
    sequence (see FloydWarshallBatched).  Returns Ds."""
    if not Ws:
        return []
    return FloydWarshallBatched(Ws, Ds, handle).run()


class Server:
    """APSP request server (continuous batching or the FIFO baseline).

    Requests are COO edge lists (host numpy arrays); distance matrices stay on
    the device until ``release``.  Thread-safe: a client thread may submit
    while another waits and releases.
    """

    def __init__(self, dtype="f32", budget_bytes=64 << 30, mode="continuous",
                 quantum_terms=0.0, device=0):
        self.dt = FLOAT32 if dtype in ("f32", "float32") else INT32
        self.np_dtype = "float32" if self.dt == FLOAT32 else "int32"
        m = {"continuous": 0, "fifo": 1}[mode]
        p = ctypes.c_void_p()
        st = lib().btas_server_create(ctypes.byref(p), int(device), self.dt, int(budget_bytes), m,
                                      float(quantum_terms))
        if st != OK:
            raise BtasError(st, "btas_server_create failed")
        self._s = p
        _track(self)

    def now(self) -> float:
        return lib().btas_server_now(self._s)

    def submit(self, n, rows, cols, w, early_exit=False, arrival=-1.0) -> int:
        import numpy as np
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        w = np.ascontiguousarray(w, dtype=self.np_dtype)
        if not (rows.size == cols.size == w.size):
            raise ValueError("rows, cols and w differ in length")
        rid = ctypes.c_int64(0)
        st = lib().btas_server_submit(self._s, int(n), rows.size, rows.ctypes.data, cols.ctypes.data,
                                      w.ctypes.data, APSP_EARLY_EXIT if early_exit else 0,
                                      float(arrival), ctypes.byref(rid))
        if st != OK:
            raise BtasError(st, f"btas_server_submit(n={n}) failed")
        return rid.value

    def wait(self, rid, timeout=-1.0) -> bool:
        done = ctypes.c_int(0)
        st = lib().btas_server_wait(self._s, int(rid), float(timeout), ctypes.byref(done))
        if st != OK:
            raise BtasError(st, f"request {rid} failed")
        return bool(done.value)

    def steps(self, rid) -> int:
        s = ctypes.c_int(0)
        st = lib().btas_server_result(self._s, int(rid), None, None, ctypes.byref(s))
        if st != OK:
            raise BtasError(st, f"request {rid} has no result")
        return s.value

    def result_into(self, rid, out):
        """Copy request rid's distance matrix into the device matrix ``out``."""
        p, ld = _mat(out, "out")
        st = lib().btas_server_copy_result(self._s, int(rid), p, ld)
        if st != OK:
            raise BtasError(st, f"request {rid} has no result")
        return out

    def times(self, rid):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = lib().btas_server_times(self._s, int(rid), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        if st != OK:
            raise BtasError(st, f"unknown request {rid}")
        return a.value, b.value, c.value

    def release(self, rid):
        st = lib().btas_server_release(self._s, int(rid))
        if st != OK:
            raise BtasError(st, f"cannot release request {rid}")

    def stats(self) -> dict:
        s = ServerStats()
        lib().btas_server_stats(self._s, ctypes.byref(s))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_s", None) is not None and self._s.value:
            lib().btas_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
