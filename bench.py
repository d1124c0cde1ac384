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
    p.add_argument("--cpu-rows", type=int, default=128,
                   help="rows of the 8192^3 min-plus fp32 product timed on the oracle")
    p.add_argument("--extras", action="store_true", help="also time the APSP workloads")
    return p.parse_args()


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
        "roofline": {"bound": "alu", "kernel": "tropical_gemm_kernel<128x128x16,8x8> min-plus fp32",
                     "achieved": round(achieved, 2), "peak": round(PEAK_TOPS, 2), "unit": "Top/s",
                     "frac": round(achieved / PEAK_TOPS, 4), "traffic": None},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(host["A"], host["B"], host["C"], args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
