"""Degenerate sizes of the entry points added beside the product and the
squaring: empty matrices, one vertex, k = 0 products, and their argument
errors, each against the oracle or the definition."""
import numpy as np
import pytest

import oracle
from oracle import INF32, NINF32

pytestmark = pytest.mark.gpu


def _dev(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


@pytest.mark.parametrize("dt", ["i32", "f32"])
def test_witness_degenerate(dev, dt):
    import torch

    import paper_1701_04733_amd as btas
    npdt = np.int32 if dt == "i32" else np.float32
    absent = INF32 if dt == "i32" else np.inf
    # k = 0: nothing improves, C and K keep their values
    A = np.zeros((3, 0), npdt)
    B = np.zeros((0, 4), npdt)
    C = np.full((3, 4), 7, npdt)
    K = np.full((3, 4), 5, np.int32)
    Cg, Kg = btas.tropical_gemm_witness(_dev(A, dev), _dev(B, dev), _dev(C, dev), _dev(K, dev))
    assert (Cg.cpu().numpy() == 7).all() and (Kg.cpu().numpy() == 5).all()
    # m = 0 and n = 0 are no-ops
    btas.tropical_gemm_witness(torch.zeros((0, 3), dtype=Cg.dtype, device=dev),
                               torch.zeros((3, 2), dtype=Cg.dtype, device=dev))
    btas.tropical_gemm_witness(torch.zeros((2, 3), dtype=Cg.dtype, device=dev),
                               torch.zeros((3, 0), dtype=Cg.dtype, device=dev))
    # 1 x 1 x 1 against the oracle, both semirings
    for sr in ("min", "max"):
        A = np.array([[2]], npdt)
        B = np.array([[3]], npdt)
        C = np.full((1, 1), absent if sr == "min" else (NINF32 if dt == "i32" else -np.inf), npdt)
        K = np.full((1, 1), -1, np.int32)
        want_c, want_k = oracle.gemm_witness(sr, A, B, C, K)
        Cg, Kg = btas.tropical_gemm_witness(_dev(A, dev), _dev(B, dev), _dev(C, dev), _dev(K, dev),
                                            semiring=sr)
        assert Cg.cpu().numpy()[0, 0] == want_c[0, 0] and Kg.cpu().numpy()[0, 0] == want_k[0, 0]


@pytest.mark.parametrize("dt", ["i32", "f32"])
def test_graph_calls_on_empty_and_one_vertex(dev, dt):
    import torch

    import paper_1701_04733_amd as btas
    npdt = np.int32 if dt == "i32" else np.float32
    tdt = torch.int32 if dt == "i32" else torch.float32
    E = torch.zeros((0, 0), dtype=tdt, device=dev)
    D, st = btas.floyd_warshall(E)
    assert st == btas.OK and D.shape == (0, 0)
    assert btas.apsp_successors(E, E).shape == (0, 0)
    D, steps, st = btas.tropical_closure(E, "max")
    assert steps == 0 and st == btas.OK
    cm = btas.maxplus_cycle_mean(E)
    assert cm == ((0, 0) if dt == "i32" else -np.inf)
    # one vertex: FW as the oracle's blocked order (a negative self loop is a
    # negative cycle and relaxes through itself); closure [[max(w, 0)]] with
    # no squaring; successor [[0]]
    for w in (5, -5):
        W = np.array([[w]], npdt)
        D, _ = btas.floyd_warshall(_dev(W, dev))
        assert D.cpu().numpy()[0, 0] == oracle.floyd_warshall_blocked(W, 64)[0, 0]
        D, steps, _ = btas.tropical_closure(_dev(W, dev), "max")
        assert steps == 0 and D.cpu().numpy()[0, 0] == max(w, 0)
        assert btas.apsp_successors(_dev(W, dev), _dev(np.minimum(W, 0), dev)).cpu().numpy()[0, 0] == 0
        # a single self loop is the only cycle: its weight is the mean
        cm = btas.maxplus_cycle_mean(_dev(W, dev))
        assert cm == ((w, 1) if dt == "i32" else float(w))


def test_argument_errors(dev):
    import torch

    import paper_1701_04733_amd as btas
    L = btas.lib()
    h = btas.default_handle(0)
    code = {name: v for v, name in btas.STATUS.items()}
    A = torch.zeros((4, 4), dtype=torch.int32, device=dev)
    p = A.data_ptr()
    # closure: unknown semiring, unknown flag bits, ld below n
    assert L.btas_tropical_closure(h.ptr, 7, btas.INT32, 4, p, 4, p, 4, 0, None) == code["BTAS_ERR_INVALID_ARG"]
    assert L.btas_tropical_closure(h.ptr, 1, btas.INT32, 4, p, 4, p, 4, 0x10, None) == code["BTAS_ERR_INVALID_ARG"]
    assert L.btas_tropical_closure(h.ptr, 1, btas.INT32, 4, p, 3, p, 4, 0, None) == code["BTAS_ERR_INVALID_ARG"]
    # cycle mean: negative n, null A
    assert L.btas_maxplus_cycle_mean(h.ptr, btas.INT32, -1, p, 4, None, None, None) == code["BTAS_ERR_INVALID_ARG"]
    assert L.btas_maxplus_cycle_mean(h.ptr, btas.INT32, 4, None, 4, None, None, None) == code["BTAS_ERR_INVALID_ARG"]
    # successors: S over D
    assert L.btas_apsp_successors(h.ptr, btas.INT32, 4, p, 4, p, 4, p, 4) == code["BTAS_ERR_ALIAS"]
