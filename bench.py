#!/usr/bin/env python3
"""Throughput of the KPM hot path on one MI355X.

One step = one pass of the whole path over one synthetic matrix already
resident in HBM: Lanczos bounds (20 steps, FP64) -> stochastic Chebyshev
moments (probe fill, fused recurrence + dot steps, reductions) -> Jackson
damping -> DOS on 200 points.  Workload (default): 3D Anderson model, 7-point
periodic Laplacian on a 64^3 grid plus uniform[-8, 8] diagonal disorder
(n = 262,144, nnz = 1,835,008), degree M = 256, 64 Rademacher probes, FP32
values and vectors with FP64 dot accumulation.

Metric: nnz * M * nvec / second (Chebyshev degree-moments per second).
The roofline object reports the fused recurrence step kernel: algorithmic
bytes per launch (8 nnz + 4 (n + 1) + 3 * 4 n b for FP32) over its average
device duration, timed with HIP events on the library's stream inside the
timed region.  The CPU baseline is the FP64 oracle (plain C recurrence,
OpenMP over probes) on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per dispatch of the fused step kernel on the default workload,
# from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by
# what the same counters read for a plain copy of known size (2.000 and
# 1.000); see profiles/.  Only valid for the default workload and the
# kernel version it was measured on.
MEASURED_TRAFFIC_BYTES = 271789238


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--M", type=int, default=256)
    ap.add_argument("--nvec", type=int, default=64)
    ap.add_argument("--block", type=int, default=64)
    ap.add_argument("--grid", type=int, default=64, help="side of the periodic cubic grid")
    ap.add_argument("--rows-per-block", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-only", action="store_true",
                    help="only run the streaming-copy bandwidth probe (counter calibration)")
    ap.add_argument("--cpu-sample-vectors", type=int, default=0,
                    help="probes in the oracle sample (0 = all cores' worth)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_1308_5467_amd as kpm
    import synth

    if args.copy_probe_only:
        ctx = kpm.Context(0)
        out = {f"copy_gbs_{sz >> 20}MiB": kpm.kpm_hbm_copy_probe(ctx, sz, 5) for sz in (1 << 30, 1 << 26)}
        print(json.dumps(out))
        return

    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(args.grid), 16.0, 1002)
    vals = A.val.astype(np.float32) if args.precision == "f32" else A.val
    D = kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, vals, args.precision)
    ctx = kpm.Context(0)
    M, nvec, block = args.M, args.nvec, args.block
    x = np.linspace(-10.0, 22.0, 200)
    # validate the matrix once, outside the timed region
    lb, ub = kpm.kpm_bounds(ctx, D, 20, 3002, 0.01)
    kpm.kpm_moments(ctx, D, lb, ub, 2, 1, 2002, precision=args.precision, validate=True)

    def step():
        lb, ub = kpm.kpm_bounds(ctx, D, 20, 3002, 0.01)
        mu = kpm.kpm_moments(ctx, D, lb, ub, M, nvec, 2002, precision=args.precision, block=block,
                             validate=False, rows_per_block=args.rows_per_block)
        g = kpm.kpm_damping_factors(ctx, kpm.KPM_DAMP_JACKSON, M)
        phi = kpm.kpm_dos(ctx, mu, g, lb, ub, x)
        return mu, phi

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kpm.kpm_profile_reset(ctx)
    kpm.kpm_profile_enable(ctx, True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mu, phi = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kpm.kpm_profile_enable(ctx, False)
    copy_gbs = kpm.kpm_hbm_copy_probe(ctx, 1 << 30, 10)
    nl, step_ms_total = kpm.kpm_profile_query(ctx, "cheb_step")
    nf, first_ms_total = kpm.kpm_profile_query(ctx, "cheb_first")
    nlz, lz_ms_total = kpm.kpm_profile_query(ctx, "lanczos")

    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    units = float(A.nnz) * M * nvec
    value = units / (ms_per_step / 1000.0)
    s_v = 4 if args.precision == "f32" else 8
    s_a = s_v
    b = min(block, nvec)
    nblocks_vec = (nvec + b - 1) // b
    bytes_per_launch = (s_a + 4) * A.nnz + 4 * (A.n + 1) + 3 * s_v * A.n * b
    avg_ms = step_ms_total / max(nl, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (MEASURED_TRAFFIC_BYTES if (args.grid, M, nvec, block, args.precision) == (64, 256, 64, 64, "f32")
                        else None),
            "kernel": "cheb_step_kernel", "avg_launch_us": round(avg_ms * 1000, 2),
            "launches": nl, "algorithmic_bytes_per_launch": int(bytes_per_launch),
            "copy_probe_gbs": round(copy_gbs, 1), "frac_of_copy_probe": round(achieved / copy_gbs, 4)}

    out = {
        "metric": "Chebyshev moment nnz*deg*vec/s",
        "value": value,
        "unit": "nnz*deg*vec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"anderson3d_{args.grid}^3_periodic_W16", "n": A.n, "nnz": A.nnz, "M": M,
                   "nvec": nvec, "block": b, "vector_blocks": nblocks_vec, "precision": args.precision,
                   "dot_accumulation": "f64", "lanczos_steps": 20, "dos_points": 200,
                   "parallelism": "single-gpu"},
        "roofline": roof,
        "breakdown_ms_per_step": {"cheb_step_total": step_ms_total / args.steps,
                                  "cheb_first": first_ms_total / args.steps,
                                  "lanczos_enqueue_to_done": lz_ms_total / args.steps},
        "hbm_gbs_whole_step": round(bytes_per_launch * (M + 1) // 2 * nblocks_vec / (ms_per_step * 1e-3) / 1e9, 1),
    }

    if not args.no_cpu_baseline:
        import oracle
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        cores = max(1, min(cores, 16))
        nv = args.cpu_sample_vectors or nvec
        Ao = A.rounded_f32() if args.precision == "f32" else A
        c, d = oracle.rescale(lb, ub)
        ts = time.perf_counter()
        oracle.moments_per_vector(Ao, c, d, M, nv, 2002, nthreads=cores)
        te = time.perf_counter()
        cpu_units = float(A.nnz) * M * nv / (te - ts)
        out["cpu_baseline"] = {"value": cpu_units, "unit": "nnz*deg*vec/s", "cores": cores, "kind": "oracle",
                               "sample": f"{nv} of {nvec} probes, full matrix, full degree M={M}, "
                                         f"FP64 plain recurrence (no doubling); {te - ts:.2f} s"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
