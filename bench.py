#!/usr/bin/env python3
"""Benchmark: tropical GEMM at m=n=k=8192 on one MI355X.

One step = the four 8192^3 products C <- C (+) A (.) B of the GEMM workload:
{min-plus, max-plus} x {float32, int32}; float32 entries uniform [0,1), int32
entries uniform [0, 10^6], 10% of entries set to the semiring's absent value,
C initialised to the (+)-identity.  Inputs are generated once on the host
(seeded), copied to HBM before timing, and every timed product rewrites its
own C (re-initialised outside the timed region is not needed: C (+) X is
idempotent in value, and each launch reads and writes all of C).

Prints ONE JSON line with the throughput in tropical Gop/s (2 ops per term:
one (.) and one (+)), the roofline of the dominant kernel (min-plus float32)
against the VALU issue peak, and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--extras]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 8192
VARIANTS = [("min", "f32"), ("max", "f32"), ("min", "i32"), ("max", "i32")]

# MI355X VALU issue peak from unit counts: fp32 vector 157.3 TFLOP/s =
# 256 CUs x 128 fp32 lanes x 2 (an FMA counts twice) x 2.4 GHz, i.e. 78.64e12
# lane-slots per second.  A tropical term (one (.) and one (+)) needs at least
# 1.5 slots with the instructions this build uses: one add, plus half of a
# three-input min/max that folds two terms.  Two tropical ops per term.
CUS, FP32_LANES, CLOCK_HZ = 256, 128, 2.4e9
SLOTS_PER_S = CUS * FP32_LANES * CLOCK_HZ             # 78.64e12
SLOTS_PER_TERM = 1.5
PEAK_TOPS = SLOTS_PER_S / SLOTS_PER_TERM * 2 / 1e12   # 104.86 tropical Top/s


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-rows", type=int, default=160,
                   help="rows of the 8192^3 min-plus fp32 product timed on the oracle")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the APSP workloads (small, large, batched, served)")
    p.add_argument("--extras", default="level12,int32_wide,apsp_small,apsp_large,witness,maxplus,batched,served",
                   help="comma-separated subset of the extra workloads to run")
    p.add_argument("--served-count", type=int, default=500,
                   help="requests per arrival rate in the served workload (the stated "
                        "configuration is 2000)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="run one plain 256 MiB device copy first (reference for HBM counters)")
    p.add_argument("--served-rates", default="100,300,1000,3000,10000",
                   help="comma-separated Poisson arrival rates (req/s) for the served workload")
    return p.parse_args()


GEMM_SOURCES = ["paper_1701_04733_amd/csrc/gemm.hip", "paper_1701_04733_amd/csrc/gemm_tile.h",
                "paper_1701_04733_amd/csrc/semiring.h"]
COUNTERS = "profiles/tropical_gemm_8192_hbm_counters.txt"


def measured_traffic(tag="min-plus/f32"):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None if the GEMM sources changed since it was taken."""
    import hashlib
    try:
        h = hashlib.sha256()
        for p in GEMM_SOURCES:
            with open(os.path.join(ROOT, p), "rb") as f:
                h.update(f.read())
        fields = {}
        with open(os.path.join(ROOT, COUNTERS)) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
        if fields.get("sources_sha256") != h.hexdigest():
            return None
        return float(fields[f"traffic_bytes_per_launch[{tag}]"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(A, B, C, rows):
    """The oracle as it stands, on a bounded slab of the min-plus fp32 product."""
    import oracle
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    oracle.gemm("min", A[:rows], B, C[:rows])
    dt = time.perf_counter() - t0
    ops = 2.0 * rows * N * N
    return {"value": ops / dt / 1e9, "unit": "Gop/s", "cores": threads, "kind": "oracle",
            "sample": f"min-plus fp32 rows 0..{rows - 1} of the 8192^3 product "
                      f"({rows}x{N}x{N} terms), {dt:.2f} s",
            "cpu": platform.processor() or platform.machine(), "nproc": os.cpu_count()}


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def bench_apsp_small(dev, reps=200):
    """One APSP on an ER digraph, n=256, p=0.05, int32 weights U{1..100}, T=8:
    per-solve latency of one launch per squaring (init + 8 split-K squarings),
    of the same sequence captured as one hipGraph launch, of the whole solve
    as one cooperative kernel (fixed T, the default at this size; with the
    early-exit test on the device; and on packed 16-bit distances, which
    these weights allow), and of the batched path with a single graph."""
    import numpy as np
    import torch

    import paper_1701_04733_amd as btas
    from paper_1701_04733_amd import workloads as wl
    W = torch.from_numpy(wl.er_digraph_i32(256, 0.05, 1, 100, seed=1)).to(dev)
    D = torch.empty_like(W)
    g = btas.BatchedAPSP([W], [D])
    out = {"workload": "APSP n=256 ER p=0.05 int32 U{1..100}, T=8 squarings"}
    def with_env(var, val, fn):
        prev = os.environ.get(var)
        os.environ[var] = val
        try:
            fn()
        finally:
            if prev is None:
                del os.environ[var]
            else:
                os.environ[var] = prev

    def per_squaring():
        with_env("BTAS_SINGLE_LAUNCH", "0", lambda: btas.apsp(W, out=D, return_steps=False))

    def single_packed16():
        # the same single launch on packed 16-bit distances (opt-in)
        with_env("BTAS_U16", "1", lambda: btas.apsp(W, out=D, return_steps=False, single_launch=True))

    with_env("BTAS_U16", "1", lambda: btas.apsp(W, out=D, single_launch=True))
    out["packed16_gate_passed"] = btas.apsp_last_packed16()
    for name, fn in (("per_squaring", per_squaring),
                     ("graph", lambda: btas.apsp(W, out=D, return_steps=False, graph=True)),
                     ("single_launch", lambda: btas.apsp(W, out=D, return_steps=False, single_launch=True)),
                     ("single_launch_early_exit",
                      lambda: btas.apsp(W, out=D, return_steps=False, single_launch=True, early_exit=True)),
                     ("single_launch_packed16", single_packed16),
                     ("batched_one_graph", g.run)):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        lat = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        thr = reps / (time.perf_counter() - t0)
        out[name] = {"latency_us_p50": round(float(np.percentile(lat, 50)) * 1e6, 1),
                     "latency_us_p99": round(float(np.percentile(lat, 99)) * 1e6, 1),
                     "solves_per_s": round(thr, 1)}
    return out


def bench_apsp_large(dev):
    """One APSP, n=16384 fp32, mean out-degree 16, exponential(1) weights,
    early exit (capped at T=14): the default solve (its first squarings run
    as sparse products), the same with dense squarings only, and the same
    graph by blocked Floyd-Warshall."""
    import torch

    import paper_1701_04733_amd as btas
    from paper_1701_04733_amd import workloads as wl
    n = 16384
    W = torch.from_numpy(wl.apsp_large_f32(n, 16.0, seed=4)).to(dev)
    D = torch.empty_like(W)
    btas.apsp(W[:4096, :4096].contiguous(), early_exit=True)  # warm the kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, steps, _ = btas.apsp(W, out=D, early_exit=True)       # sparse first squarings
    torch.cuda.synchronize()
    sec_default = time.perf_counter() - t0
    # dense squarings only: every step is an n^3 product, so Gop/s is the
    # product kernels' real rate
    os.environ["BTAS_SPARSE_STEPS"] = "0"
    try:
        t0 = time.perf_counter()
        _, steps, _ = btas.apsp(W, out=D, early_exit=True)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
    finally:
        del os.environ["BTAS_SPARSE_STEPS"]
    ops = 2.0 * n ** 3 * steps
    # the same graph by blocked Floyd-Warshall: n^3 relaxations in one pass
    # (a warm-up call at full size, then the median of three)
    F = torch.empty_like(W)
    btas.floyd_warshall(W, out=F)
    torch.cuda.synchronize()
    fw_ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        btas.floyd_warshall(W, out=F)
        torch.cuda.synchronize()
        fw_ts.append(time.perf_counter() - t0)
    fw_sec = sorted(fw_ts)[1]
    fw_ops = 2.0 * n ** 3
    fin = torch.isfinite(D)
    rel = ((F - D).abs() / D.abs().clamp_min(1e-30))[fin & (D > 0)].max().item()
    return {"workload": "APSP n=16384 fp32, out-degree 16, exp(1) weights, early exit",
            "seconds": round(sec_default, 4), "steps": steps, "T": btas.apsp_num_steps(n),
            "dense_steps_only": {"seconds": round(sec, 4), "Gop/s": round(ops / sec / 1e9, 1),
                                 "frac_valu_peak": round(ops / sec / 1e12 / PEAK_TOPS, 4)},
            "floyd_warshall": {"seconds": round(fw_sec, 4), "Gop/s": round(fw_ops / fw_sec / 1e9, 1),
                               "frac_valu_peak": round(fw_ops / fw_sec / 1e12 / PEAK_TOPS, 4),
                               "speedup_vs_squaring": round(sec_default / fw_sec, 2),
                               "same_finite": bool(torch.equal(torch.isfinite(F), fin)),
                               "max_rel_diff_vs_squaring": rel}}


def bench_witness(dev, operands, reps=3):
    """The argmin-carrying product on the 8192^3 min-plus fp32 operands (C
    starts at the (+)-identity, K at -1), and the successor matrix of the
    n=16384 graph from its Floyd-Warshall distances (over W's edge lists, and
    as the dense witness product)."""
    import numpy as np
    import torch

    import paper_1701_04733_amd as btas
    from paper_1701_04733_amd import workloads as wl
    A, B, C0 = operands

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = _events()
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts)) / 1e3

    C = torch.empty_like(C0)
    K = torch.empty(C0.shape, dtype=torch.int32, device=dev)

    def witness():
        C.copy_(C0)
        K.fill_(-1)
        btas.tropical_gemm_witness(A, B, C, K)

    ops = 2.0 * N ** 3
    sec = timed(witness)
    out = {"workload": "witness product 8192^3 min-plus fp32 (C, K reset inside the timed region)",
           "ms": round(sec * 1e3, 2), "Gop/s": round(ops / sec / 1e9, 1),
           "frac_valu_peak": round(ops / sec / 1e12 / PEAK_TOPS, 4)}
    del C, K
    n = 16384
    W = torch.from_numpy(wl.apsp_large_f32(n, 16.0, seed=4)).to(dev)
    D, _ = btas.floyd_warshall(W)
    S = torch.empty((n, n), dtype=torch.int32, device=dev)
    sec = timed(lambda: btas.apsp_successors(W, D, out=S))       # over W's edge lists
    os.environ["BTAS_SPARSE_STEPS"] = "0"
    try:
        dsec = timed(lambda: btas.apsp_successors(W, D, out=S))  # the dense witness product
    finally:
        del os.environ["BTAS_SPARSE_STEPS"]
    out["successors_16384"] = {"ms": round(sec * 1e3, 2),
                               "dense_witness_product": {"ms": round(dsec * 1e3, 2),
                                                         "Gop/s": round(2.0 * n ** 3 / dsec / 1e9, 1)}}
    return out


def bench_maxplus(dev, reps=3):
    """Max-plus applications: the maximum cycle mean (Karp: n max-plus gemv
    steps, then the reduction) of a 4096-vertex digraph with int32 weights,
    and the critical paths (max-plus closure with early exit) of a
    4096-task precedence DAG."""
    import numpy as np
    import torch

    import paper_1701_04733_amd as btas
    from paper_1701_04733_amd import workloads as wl
    n = 4096
    A = torch.from_numpy(wl.maxplus_digraph_i32(n, 8.0, -50, 100, seed=21)).to(dev)
    btas.maxplus_cycle_mean(A)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        num, den = btas.maxplus_cycle_mean(A)
        ts.append(time.perf_counter() - t0)
    sec = float(np.median(ts))
    out = {"cycle_mean": {"workload": "max cycle mean, n=4096 digraph, mean out-degree 8, int32 U{-50..100}",
                          "ms": round(sec * 1e3, 2), "lambda": [num, den],
                          "us_per_product": round(sec * 1e6 / n, 2),
                          "path": "one cooperative launch, A held in registers (n <= 4096)"}}
    del A
    W = torch.from_numpy(wl.precedence_dag_f32(n, 8.0, seed=22)).to(dev)
    btas.tropical_closure(W, "max", early_exit=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, steps, _ = btas.tropical_closure(W, "max", early_exit=True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    out["critical_paths"] = {"workload": "max-plus closure, n=4096 precedence DAG, mean out-degree 8, "
                                         "durations U(0,10] fp32, early exit",
                             "ms": round(sec * 1e3, 2), "steps": steps,
                             "Gop/s": round(2.0 * n ** 3 * steps / sec / 1e9, 1)}
    return out


def bench_batched(dev, reps=5):
    """4096 independent graphs, n log-uniform in [16,512], p = 8/n, int32
    weights U{1..1000}: one hipGraph launch (fixed T(n), and with on-device
    early exit), the same graphs by batched blocked Floyd-Warshall, and 4096
    plain solves."""
    import numpy as np
    import torch

    import paper_1701_04733_amd as btas
    from paper_1701_04733_amd import workloads as wl
    Ws = [torch.from_numpy(w).to(dev) for w in wl.batched_graphs_i32(count=4096, seed=5)]
    r = btas.BatchedAPSP(Ws)
    r.run()
    torch.cuda.synchronize()
    info = r.plan_info()
    ms = []
    for _ in range(reps):
        e0, e1 = _events()
        e0.record()
        r.run()
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    bm = float(np.median(ms))
    outs = [torch.empty_like(w) for w in Ws]
    for w, o in zip(Ws[:64], outs):
        btas.apsp(w, out=o, return_steps=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for w, o in zip(Ws, outs):
        btas.apsp(w, out=o, return_steps=False)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    same = all(torch.equal(a, b) for a, b in zip(r.Ds, outs))
    # the same solve with on-device early exit (a graph's squarings stop at
    # its fixpoint; same bits)
    re = btas.BatchedAPSP(Ws, early_exit=True)
    re.run()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = _events()
        e0.record()
        re.run()
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    em = float(np.median(ms))
    same_early = all(torch.equal(a, b) for a, b in zip(re.Ds, outs))
    # the same plan with the graphs of <= 64 vertices solved whole in LDS on
    # their own branch of the captured graph (opt-in) instead of inside the
    # grid-wide squaring launches
    prev = os.environ.get("BTAS_BATCH_LDS")
    os.environ["BTAS_BATCH_LDS"] = "1"
    try:
        h0 = btas.Handle(0)
        h0.bind_stream()
        rg = btas.BatchedAPSP(Ws, handle=h0)
        rg.run()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = _events()
            e0.record()
            rg.run()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        gm = float(np.median(ms))
        same_grid = all(torch.equal(a, b) for a, b in zip(rg.Ds, outs))
        del rg
        h0.close()
    finally:
        if prev is None:
            del os.environ["BTAS_BATCH_LDS"]
        else:
            os.environ["BTAS_BATCH_LDS"] = prev
    # the same graphs by batched blocked Floyd-Warshall (int32: the same bits)
    fw = btas.FloydWarshallBatched(Ws)
    fw.run()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = _events()
        e0.record()
        fw.run()
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    fm = float(np.median(ms))
    same_fw = all(torch.equal(a, b) for a, b in zip(fw.Ds, outs))
    return {"workload": "batched APSP, 4096 graphs, n log-uniform [16,512], p=8/n, int32 U{1..1000}",
            "early_exit": {"batched_ms": round(em, 3), "batched_solves_per_s": round(4096 / (em / 1e3), 1),
                           "bit_identical_to_plain": same_early},
            "small_graphs_whole_in_lds": {"batched_ms": round(gm, 3),
                                          "bit_identical_to_plain": same_grid},
            "floyd_warshall": {"batched_ms": round(fm, 3), "batched_solves_per_s": round(4096 / (fm / 1e3), 1),
                               "bit_identical_to_plain": same_fw},
            "batched_ms": round(bm, 3), "batched_solves_per_s": round(4096 / (bm / 1e3), 1),
            "batched_Gop/s": round(2 * info["terms"] / (bm / 1e3) / 1e9, 1),
            "frac_valu_peak": round(2 * info["terms"] / (bm / 1e3) / 1e12 / PEAK_TOPS, 4),
            "graph_kernel_launches": info["launches"],
            "plain_ms": round(plain * 1e3, 3), "plain_solves_per_s": round(4096 / plain, 1),
            "speedup_vs_plain": round(plain * 1e3 / bm, 2), "bit_identical_to_plain": same}


def bench_int32_wide(dev, reps=5):
    """int32 min-plus products at 8192^3 beyond the binary32-exact range (the
    clamped integer adds): entries uniform in [0, 2^28] and in [0, 2^29 - 1]
    (the whole contract), 10% absent, C = INF."""
    import numpy as np
    import torch

    import paper_1701_04733_amd as btas
    from paper_1701_04733_amd import workloads as wl
    out = {"workload": "int32 min-plus 8192^3 beyond 2^23 (clamped integer adds)"}
    for name, hi in (("values_le_2^28", 1 << 28), ("values_le_2^29-1", (1 << 29) - 1)):
        ops = []
        for seed in (2, 3):
            g = wl.rng(seed)
            X = g.integers(0, hi, size=(N, N), endpoint=True, dtype=np.int32)
            X[g.random((N, N), dtype=np.float32) < 0.1] = wl.I32_INF
            ops.append(torch.from_numpy(X).to(dev))
            del X
        C0 = torch.full((N, N), wl.I32_INF, dtype=torch.int32, device=dev)
        btas.tropical_gemm(ops[0], ops[1], C0.clone())
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            C = C0.clone()
            e0, e1 = _events()
            e0.record()
            btas.tropical_gemm(ops[0], ops[1], C)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        gops = 2.0 * N ** 3 / (ms / 1e3) / 1e9
        out[name] = {"ms": round(ms, 3), "Gop/s": round(gops, 1),
                     "frac_valu_peak": round(gops / 1e3 / PEAK_TOPS, 4)}
        del ops, C0, C
        torch.cuda.empty_cache()
    return out


def bench_batched_squaring(dev, reps=3):
    """The 4096-graph batched squaring alone (fixed T, then early exit), with
    no other solver in the process: the workload for counter collection
    (run it with BTAS_BATCH_GRAPH=0 so that the launches are issued in order
    instead of from a captured graph)."""
    import numpy as np
    import torch

    import paper_1701_04733_amd as btas
    from paper_1701_04733_amd import workloads as wl
    Ws = [torch.from_numpy(w).to(dev) for w in wl.batched_graphs_i32(count=4096, seed=5)]
    out = {"workload": "batched APSP squaring, 4096 graphs, n log-uniform [16,512], p=8/n, int32 U{1..1000}",
           "captured": os.environ.get("BTAS_BATCH_GRAPH", "1") != "0"}
    for name, early in (("fixed_T", False), ("early_exit", True)):
        r = btas.BatchedAPSP(Ws, early_exit=early)
        r.run()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = _events()
            e0.record()
            r.run()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        out[name] = {"batched_ms": round(float(np.median(ms)), 3)}
        del r
    return out


def bench_level12(dev, reps=10):
    """HBM-bound routines: gemv y <- y (+) A (.) x at 8192x8192 and the level-1
    ops on 2^26-element vectors (fp32 min-plus), against 8 TB/s."""
    import numpy as np
    import torch

    import paper_1701_04733_amd as btas
    g = torch.Generator(device=dev).manual_seed(7)
    out = {"workload": "fp32 min-plus: gemv 8192x8192, level 1 on 2^26 elements", "peak_GB/s": 8000.0}

    def timed(fn, nbytes, calls=20):
        # `calls` back-to-back calls between two events, so that the host's
        # per-call work overlaps the previous kernel and the figure is the
        # kernel's own (a single call per event pair also timed the launch)
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = _events()
            e0.record()
            for _ in range(calls):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / calls)
        ms = float(np.median(ts))
        return {"us": round(ms * 1e3, 1), "GB/s": round(nbytes / (ms / 1e3) / 1e9, 1),
                "frac_hbm_peak": round(nbytes / (ms / 1e3) / 8e12, 4)}

    A = torch.rand((8192, 8192), generator=g, device=dev)
    x = torch.rand(8192, generator=g, device=dev)
    y = torch.full((8192,), float("inf"), device=dev)
    out["gemv"] = timed(lambda: btas.tropical_gemv(A, x, y), A.numel() * 4 + 8192 * 12)
    del A
    n = 1 << 26
    u = torch.rand(n, generator=g, device=dev)
    v = torch.rand(n, generator=g, device=dev)
    w = torch.empty_like(u)
    r = torch.empty(1, device=dev)
    out["vadd"] = timed(lambda: btas.vadd(u, v, w), 12 * n)
    out["vmul"] = timed(lambda: btas.vmul(u, v, w), 12 * n)
    out["dot"] = timed(lambda: btas.dot(u, v, out=r), 8 * n)
    out["axpy"] = timed(lambda: btas.axpy(0.5, u, w), 12 * n)
    return out


def _serve_trace(reqs, mode, early_exit=False):
    import threading

    import numpy as np

    import paper_1701_04733_amd as btas
    srv = btas.Server("f32", budget_bytes=64 << 30, mode=mode)
    ids = [None] * len(reqs)
    lat = []
    ready = threading.Event()

    def reaper():
        for i in range(len(reqs)):
            while ids[i] is None:
                time.sleep(0.0002)
            srv.wait(ids[i], -1)
            a, _, d = srv.times(ids[i])
            lat.append((a, d))
            srv.release(ids[i])
        ready.set()

    th = threading.Thread(target=reaper, daemon=True)
    th.start()
    base = srv.now() + 0.05
    for i, r in enumerate(reqs):
        target = base + r.arrival_s
        while True:
            left = target - srv.now()
            if left <= 0:
                break
            time.sleep(left if left > 0.002 else 0)
        ids[i] = srv.submit(r.n, r.rows, r.cols, r.w, early_exit=early_exit, arrival=target)
    th.join()
    st = srv.stats()
    srv.close()
    L = np.array([d - a for a, d in lat]) * 1e3
    span = max(d for _, d in lat) - min(a for a, _ in lat)
    return {"p50_ms": round(float(np.percentile(L, 50)), 2), "p99_ms": round(float(np.percentile(L, 99)), 2),
            "mean_ms": round(float(L.mean()), 2), "solves_per_s": round(len(reqs) / span, 1),
            "launches": st["launches"], "pool_peak_GiB": round(st["pool_peak_bytes"] / 2**30, 2)}


def bench_served(rates, count):
    """Open-loop Poisson trace of fp32 APSP requests (n log-uniform in
    [32,4096], out-degree 12, weights in (0,10], COO in, densified on the
    device, fixed T(n)), served with continuous batching (also with each
    request's early exit: same bits) and with the plain FIFO
    one-solve-per-launch path on the same trace."""
    from paper_1701_04733_amd import workloads as wl
    out = {"workload": f"served APSP fp32, {count} requests per rate, n log-uniform [32,4096], "
                       "out-degree 12, HBM budget 64 GiB"}
    for rate in rates:
        reqs = wl.served_requests(count, float(rate))
        out[f"rate_{rate}"] = {"continuous": _serve_trace(reqs, "continuous"),
                               "continuous_early_exit": _serve_trace(reqs, "continuous", True),
                               "fifo": _serve_trace(reqs, "fifo")}
    # The knee: the highest swept rate that a mode still serves at >= 90% of
    # the arrival rate (above it the queue grows for as long as the trace lasts).
    for mode in ("continuous", "continuous_early_exit", "fifo"):
        keep = [r for r in rates if out[f"rate_{r}"][mode]["solves_per_s"] >= 0.9 * r]
        out[f"knee_req_per_s[{mode}]"] = max(keep) if keep else None
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1701_04733_amd as btas
    from paper_1701_04733_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    host = {}
    tensors = {}
    for sr, dt in VARIANTS:
        A = wl.gemm_operand((N, N), dt, sr, seed=2)
        B = wl.gemm_operand((N, N), dt, sr, seed=3)
        C = wl.semiring_identity_matrix((N, N), dt, sr)
        if (sr, dt) == ("min", "f32"):
            host = {"A": A, "B": B, "C": C}
        tensors[(sr, dt)] = tuple(torch.from_numpy(x).to(dev) for x in (A, B, C))
        del A, B, C
    torch.cuda.synchronize()
    h = btas.default_handle(0)
    if args.calibrate_copy:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)                       # reads and writes 256 MiB
        torch.cuda.synchronize()
        del src, dst

    def run_step(events=None):
        for v in VARIANTS:
            tA, tB, tC = tensors[v]
            if events is not None:
                events[v][0].record()
            btas.tropical_gemm(tA, tB, tC, semiring=v[0], handle=h)
            if events is not None:
                events[v][1].record()

    for _ in range(args.warmup):
        run_step()
    torch.cuda.synchronize()
    per_launch = {v: [] for v in VARIANTS}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev = {v: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for v in VARIANTS}
        run_step(ev)
        torch.cuda.synchronize()
        for v in VARIANTS:
            per_launch[v].append(ev[v][0].elapsed_time(ev[v][1]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    ops_per_launch = 2.0 * N ** 3
    value = ops_per_launch * len(VARIANTS) / (ms_per_step / 1e3) / 1e9
    variants = {}
    for v in VARIANTS:
        ms = float(np.median(per_launch[v]))
        gops = ops_per_launch / (ms / 1e3) / 1e9
        variants[f"{v[0]}-plus/{v[1]}"] = {"ms": round(ms, 3), "Gop/s": round(gops, 1),
                                           "frac_valu_peak": round(gops / 1e3 / PEAK_TOPS, 4)}
    dom = ("min", "f32")
    dom_ms = float(np.mean(per_launch[dom]))
    achieved = ops_per_launch / (dom_ms / 1e3) / 1e12
    out = {
        "metric": "min-plus GEMM Gop/s & %VALU peak @8192^3; batched APSP solves/s, p99 ms",
        "value": round(value, 1),
        "unit": "Gop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+i32",
        "data": "synthetic (seeded numpy PCG64)",
        "config": {"workload": "tropical GEMM m=n=k=8192, {min,max}-plus x {fp32,int32}, "
                               "10% absent entries, C = (+)-identity",
                   "m": N, "n": N, "k": N, "products_per_step": len(VARIANTS)},
        "variants": variants,
        "roofline": {"bound": "alu", "kernel": "tropical_gemm_direct_kernel<256x256x16,8x8> min-plus fp32 (direct global->LDS k-blocks, 1024 threads)",
                     "achieved": round(achieved, 2), "peak": round(PEAK_TOPS, 2), "unit": "Top/s",
                     "frac": round(achieved / PEAK_TOPS, 4), "traffic": measured_traffic(),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes": 4 * N * N * 4},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(host["A"], host["B"], host["C"], args.cpu_rows)
    witness_operands = tensors[("min", "f32")]
    del host, tensors
    torch.cuda.empty_cache()
    if not args.no_extras:
        want = {x for x in args.extras.split(",") if x}
        extras = {}
        if "level12" in want:
            extras["level12"] = bench_level12(dev)
        if "int32_wide" in want:
            extras["int32_wide"] = bench_int32_wide(dev)
        if "apsp_small" in want:
            extras["apsp_small"] = bench_apsp_small(dev)
        if "apsp_large" in want:
            extras["apsp_large"] = bench_apsp_large(dev)
        if "witness" in want:
            extras["witness"] = bench_witness(dev, witness_operands)
        del witness_operands
        if "maxplus" in want:
            extras["maxplus"] = bench_maxplus(dev)
        torch.cuda.empty_cache()
        if "batched" in want:
            extras["batched"] = bench_batched(dev)
        if "batched_squaring" in want:
            extras["batched_squaring"] = bench_batched_squaring(dev)
        torch.cuda.empty_cache()
        if "served" in want:
            rates = [int(x) for x in args.served_rates.split(",") if x]
            extras["served"] = bench_served(rates, args.served_count)
        out["extras"] = extras
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
