"""Benchmark: local ETKF frames on one MI355X, 84x84-subaperture pupil, m = 64.

One step = one frame of the whole hot path over one slope vector: slope
synthesis (a3), per-domain analysis (a4-a8: gather, C and b, Jacobi
eigensolve, wbar/W/T, update), merge + AR(2) forecast with model noise (a1,
a2, a8) and the prediction mean (a9).  Slopes of every timed frame are
resident in HBM before the timed region starts.

    python bench.py [--steps K] [--warmup W] [--precision fp64|fp32|bf16]

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: this
build runs on one GPU.
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

PEAK_FP64_TFLOPS = 78.6   # MI355X vector FP64 (256 CU x 2.4 GHz x 128 flop/clk)
PEAK_HBM_GBS = 8000.0

METRIC = "frames/s + p50/p99 frame latency (µs), LETKF 84×84 subaps m=64"


def analysis_flops(m: int, dmap, sweeps_total: int, solves: int, frames: int) -> float:
    """Algorithmic FP64 flops of the domain-analysis kernel over `frames`
    launches.  Per domain with p_l slopes and n_l state rows:
      C (symmetric) m(m+1) p_l, r-scaling m p_l, b 2 m p_l,
      Jacobi per sweep: column norms 2m^2 + one dot per pair 2m * m(m-1)/2,
      rotations 6m per pair * m(m-1)/2 in every sweep but the last (check) one,
      lambda/U 3m^2, wbar 4m^2, W 2m^3, update 2 n_l m^2 + 2 n_l m."""
    e = np.diff(dmap.est_ptr).astype(float)
    s = np.diff(dmap.obs_ptr).astype(float)
    p_l, n_l = 2 * s, 2 * e
    L = dmap.n_domains
    fixed = np.sum(m * (m + 1) * p_l + 3 * m * p_l + 2 * n_l * m * m + 2 * n_l * m) + L * (2 * m ** 3 + 7 * m * m)
    dots = 2 * m * m + m * m * (m - 1)
    rots = 3 * m * m * (m - 1)
    return frames * fixed + sweeps_total * dots + (sweeps_total - solves) * rots


def cpu_baseline(case, seconds: float = 15.0):
    """The FP64 oracle on the host, one thread, on the first frames of the
    same workload until `seconds` have passed (at least two frames)."""
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    import oracle
    D = sp.csr_matrix((case.D.val, case.D.col, case.D.rowptr), shape=case.D.shape)
    X = case.X0.copy()
    ys = []
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        k = 0
        while k < 2 or time.perf_counter() - t0 < seconds:
            y = case.slopes(k)
            ts = time.perf_counter()
            Xa = oracle.analysis(X, y, D, case.dmap, case.r_inv, case.inflation)
            X = oracle.forecast(Xa, case.a1, case.a2, case.sigma_v, case.philox_seed, k)
            ys.append(time.perf_counter() - ts)
            k += 1
    fps = len(ys) / float(np.sum(ys))
    return dict(value=round(fps, 3), unit="frames/s", cores=1, kind="oracle",
                sample=f"first {len(ys)} frames of the same 84x84, m=64 workload (NumPy/LAPACK FP64, 1 thread)")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--latency-frames", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps(dict(error="this build runs on one GPU only; --gpus must be 1")))
        return 2

    import torch

    from paper_1310_5954_amd import BF16, FP32, FP64, Filter, Problem
    from workload.configs import build_case

    prec = dict(fp64=FP64, fp32=FP32, bf16=BF16)[args.precision]
    case = build_case(3)
    K, W, NL = args.steps, args.warmup, args.latency_frames
    n_frames = W + K + NL
    print(f"[bench] cfg3 84x84 m=64 domains={case.dmap.n_domains} precision={args.precision} "
          f"frames={n_frames}", file=sys.stderr, flush=True)
    ys_host = np.stack([case.slopes(k) for k in range(n_frames)])
    dev = torch.device("cuda:0")
    ys = torch.tensor(ys_host, dtype=torch.float64, device=dev)
    f = Filter(Problem.from_case(case), case.X0, precision=prec, device=dev)
    for k in range(W):
        f.step(ys[k], pred=False)
    torch.cuda.synchronize()
    sw0, so0 = f.sweep_stats()
    f.kernel_times(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(W, W + K):
        f.step(ys[k], pred=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, calls = f.kernel_times(False)
    sw1, so1 = f.sweep_stats()
    assert calls == K
    fps = K / (t1 - t0)
    print(f"[bench] timed {K} frames: {fps:.1f} frames/s", file=sys.stderr, flush=True)

    # per-frame latency: slopes already resident, prediction mean back on the host
    lat = []
    for k in range(W + K, W + K + NL):
        ts = time.perf_counter()
        f.step(ys[k], pred=True)
        lat.append(time.perf_counter() - ts)
    lat_us = np.array(lat) * 1e6
    assert f.unconverged() == 0

    ana_ms = ms[1] / K
    flops = analysis_flops(case.m, case.dmap, sw1 - sw0, so1 - so0, K) / K
    achieved = flops / (ana_ms * 1e-3) / 1e12
    sweeps_mean = (sw1 - sw0) / max(so1 - so0, 1)
    out = dict(
        metric=METRIC, value=round(fps, 2), unit="frames/s", n_gpus=1, steps=K, warmup=W,
        ms_per_step=round(1e3 / fps, 4), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64" if prec == FP64 else ("f32" if prec == FP32 else "bf16+f64"), data="synthetic",
        config=dict(workload="84x84 circular SH pupil, 5713 actuators (n=11426), 5544 subapertures (p=11088), "
                             f"m=64, {case.dmap.n_domains} overlapping 6x6 domains, halo 2, GC taper; plain "
                             "per-frame path (one instance, analysis + AR(2) forecast per frame)",
                    precision=args.precision, path="plain"),
        p50_us=round(float(np.percentile(lat_us, 50)), 1), p99_us=round(float(np.percentile(lat_us, 99)), 1),
        kernel_ms=dict(slopes=round(ms[0] / K, 4), analysis=round(ana_ms, 4), merge_forecast=round(ms[2] / K, 4)),
        jacobi_sweeps_mean=round(sweeps_mean, 3),
        roofline=dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                      frac=round(achieved / PEAK_FP64_TFLOPS, 4), traffic=None,
                      kernel="k_analysis (FP64 vector ALU: one-sided Jacobi dominates)"),
    )
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
