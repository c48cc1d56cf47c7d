"""Benchmark: local ETKF frames on one MI355X, 84x84-subaperture pupil, m = 64.

A frame is the whole hot path over one slope vector: slope synthesis,
per-domain analysis (gather, C and b, Cholesky + Jacobi eigensolve,
wbar/W/T, update), merge + AR(2) forecast with model noise, and the
prediction mean copied to the host.  Slopes of every timed frame are resident
in HBM before the timed region starts.

Two forms serve the same load, --instances B resident AO instances
(independent ensembles, default 4) in a closed loop: each instance releases
its next frame when its previous one is done.
  serving  the server batches the pending frames of all instances into shared
           launches (by default BF16 contractions and the FP64 eigensolve:
           Cholesky, Jacobi rotations, w-bar, W, T).  This is `value`
           (aggregate frames/s) and p50/p99 (submit -> callback, over at least
           500 frames), with device-resident slopes; the same with host slopes
           and with the opt-in FP32 rotations are reported beside it.
  plain    the plain per-frame FP64 path (letkf_step, one frame per launch
           sequence) serves the same instances one frame at a time; its
           frames/s and p50/p99 are reported beside, together with the
           unloaded single-instance latency and its analysis kernel's
           roofline (plain_fp64.roofline).
The roofline line is the serving path's analysis kernel (BF16 contractions,
FP64 eigensolve), timed with HIP events on one instance per launch.  The CPU
baseline is the FP64 oracle over the host's cores (a process pool over the
domains) and on one core.

    python bench.py [--steps K] [--warmup W] [--instances B] [--precision fp64|fp32|bf16]

Prints one JSON line.  --gpus N > 1 is refused: the library runs on one GPU.
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
FP64_ = 0        # precision code of the FP64 path (the library's LETKF_FP64)

METRIC = "frames/s + p50/p99 frame latency (µs), LETKF 84×84 subaps m=64"
TRAFFIC_FILES = {  # rocprofv3 counter summaries of the analysis kernel, per precision path
    "fp64": os.path.join(ROOT, "profiles", "k_analysis_fp64_84x84_m64_traffic.txt"),
    "bf16": os.path.join(ROOT, "profiles", "k_analysis_bf16_84x84_m64_traffic.txt"),
}


def measured_traffic(path: str, kernels: str, tuning):
    """HBM bytes per k_analysis launch from a committed rocprofv3 counter
    summary (FETCH_SIZE x fetch scale + WRITE_SIZE x write scale) for the
    launch shape (domain order, grid) this run chose, or None when the summary
    was taken on another build of the device code or has no such shape."""
    try:
        kv = dict(line.split(":", 1) for line in open(path) if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    if kv.get("kernels", "").strip() != kernels or not tuning:
        return None
    v = kv.get(f"traffic_bytes_per_launch.{tuning['order']}.{tuning['grid']}")
    return float(v) if v is not None else None


def unique_bytes(case, esize: int) -> int:
    """Bytes the analysis kernel must move at least per launch: every slope row
    of Y' and every state row of X read once (esize bytes per value), d and
    r (8 bytes each per slope), and the per-domain analysis rows Z written
    once.  The ratio of the measured HBM traffic to this is the re-read and
    scratch overhead."""
    m, p, n = case.m, 2 * case.n_sub, 2 * case.n_act
    zrows = 2 * int(case.dmap.est_ptr[-1])
    return int(p * m * esize + n * m * esize + 16 * p + zrows * m * esize)


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


def run_phases(case, W, ys, prec=None):
    """Per-phase cycles of every domain's analysis workgroup (shader-clock
    stamps of a debug instance, FP64 unless `prec` (the plain path in that
    precision), one frame after W warm-up frames and
    six frames whose per-domain sweep counts are kept), where each domain ran
    (CU, sharing it with other domains or not), and
    the bytes each phase moves, for the bandwidth view of the analysis
    kernel: gather + C/b reads the domain's slope rows of Y' (8m bytes each)
    plus d and r (16 bytes per observation); the update reads the domain's
    state rows of X' and writes as many rows of Z (8m bytes each).  The
    clock is calibrated from the kernel's HIP-event time (the slowest
    domain's cycles over the launch's duration)."""
    import torch

    from paper_1310_5954_amd import FP64, Filter, Problem
    f = Filter(Problem.from_case(case), case.X0, precision=FP64 if prec is None else prec, device="cuda:0", debug=True)
    for k in range(W):
        f.step(ys[k], pred=False)
    m, dm = case.m, case.dmap
    # sweeps of every domain over the frames before the measured one (how well a
    # frame's sweep counts predict the next frame's)
    F = min(6, len(ys) - W - 1)
    sweep_frames = []
    for k in range(F):
        f.step(ys[W + k], pred=False)
        sweep_frames.append([f.debug_domain(l)["sweeps"] for l in range(dm.n_domains)])
    f.kernel_times(True)
    f.step(ys[W + F], pred=False)
    torch.cuda.synchronize()
    ms, _ = f.kernel_times(False)
    names = ("gather_C", "cholesky", "jacobi", "transform", "update")
    dbg = [f.debug_domain(l) for l in range(dm.n_domains)]
    cyc = np.array([[d["cycles"][n] for n in names] for d in dbg])
    sweeps = np.array([d["sweeps"] for d in dbg])
    place = [f.debug_placement(l) for l in range(dm.n_domains)]
    sub = np.array([list(f.debug_substeps(l).values()) for l in range(dm.n_domains)])
    f.close()
    total = cyc.sum(axis=1)
    clock_hz = total.max() / (ms[1] * 1e-3)
    s_obs = 2 * np.diff(dm.obs_ptr).astype(float)
    n_rows = 2 * np.diff(dm.est_ptr).astype(float)
    bytes_gather = s_obs * (8 * m + 16)
    bytes_update = n_rows * 8 * m * 2
    out = dict(domains=int(dm.n_domains), analysis_ms=round(ms[1], 4), clock_ghz=round(clock_hz / 1e9, 3),
               cycles_mean={n: round(float(cyc[:, i].mean())) for i, n in enumerate(names)},
               share={n: round(float(cyc[:, i].sum() / cyc.sum()), 4) for i, n in enumerate(names)},
               transform_substeps_mean={n: round(float(sub[:, i].mean()))
                                        for i, n in enumerate(("U", "wbar", "refine", "T"))})
    # placement: the CU each domain ran on and how many other domains shared it while it ran
    cu_key = [(p["xcd"], p["se"], p["sh"], p["cu"]) for p in place]
    t0 = np.array([p["start_clock"] for p in place])
    t1 = t0 + total
    shared = np.array([sum(1 for k in range(len(place)) if k != l and cu_key[k] == cu_key[l]
                           and t0[k] < t1[l] and t0[l] < t1[k]) for l in range(len(place))])
    per_cu = {}
    for k in cu_key:
        per_cu[k] = per_cu.get(k, 0) + 1
    hist = {}
    for v in per_cu.values():
        hist[v] = hist.get(v, 0) + 1
    slow = int(np.argmax(total))
    out["placement"] = dict(
        cus_used=len(per_cu), domains_per_cu={str(k): v for k, v in sorted(hist.items())},
        cycles_by_sharing={str(k): dict(domains=int((shared == k).sum()),
                                        cycles_mean=round(float(total[shared == k].mean())),
                                        sweeps_mean=round(float(sweeps[shared == k].mean()), 2))
                           for k in sorted(set(shared.tolist()))},
        cycles_per_sweep_jacobi=round(float((cyc[:, 2] / np.maximum(sweeps, 1)).mean())),
        sweeps_hist={str(k): int((sweeps == k).sum()) for k in sorted(set(sweeps.tolist()))},
        slowest=dict(domain=slow, cycles=round(float(total[slow])), sweeps=int(sweeps[slow]),
                     sharing=int(shared[slow])),
        # which workgroup indices ran alone on their CU (one item each at this grid)
        alone_workgroups=_ranges(sorted(p["workgroup"] for p, sh in zip(place, shared) if sh == 0)))
    sf = np.array(sweep_frames + [sweeps.tolist()], dtype=float)
    same = float(np.mean(sf[1:] == sf[:-1]))
    top = []
    for k in range(len(sf) - 1):
        a, b = np.argsort(-sf[k], kind="stable")[:16], set(np.argsort(-sf[k + 1], kind="stable")[:48].tolist())
        top.append(np.mean([x in b for x in a]))
    out["sweep_stability"] = dict(
        frames=len(sf), same_as_previous_frame=round(same, 3),
        corr_with_previous=round(float(np.mean([np.corrcoef(sf[k], sf[k + 1])[0, 1] for k in range(len(sf) - 1)])), 3),
        top16_in_next_top48=round(float(np.mean(top)), 3),
        mean_over_frames_vs_last=round(float(np.corrcoef(sf[:-1].mean(axis=0), sf[-1])[0, 1]), 3))
    for name, i, b in (("gather_C", 0, bytes_gather), ("update", 4, bytes_update)):
        t = cyc[:, i] / clock_hz
        # every domain's gather starts with the launch, so the gathers overlap: aggregate = bytes / longest gather
        out[name] = dict(bytes_total=int(b.sum()), per_domain_gbs_mean=round(float(np.mean(b / t) / 1e9), 2),
                         aggregate_gbs=round(float(b.sum() / t.max() / 1e9), 1) if i == 0 else None,
                         aggregate_frac_of_hbm=round(float(b.sum() / t.max() / 1e9 / PEAK_HBM_GBS), 4)
                         if i == 0 else None)
    return out


def _ranges(xs):
    """[a, b] runs of consecutive integers in a sorted list."""
    out = []
    for x in xs:
        if out and x == out[-1][1] + 1:
            out[-1][1] = x
        else:
            out.append([x, x])
    return out


def big_analysis_flops(m: int, p_obs: int, n_rows: int, sweeps: float) -> float:
    """Algorithmic FP64 flops of one global-domain analysis with m members,
    p_obs observations and n_rows state rows: C (symmetric) m(m+1) p, b 2mp,
    Cholesky m^3/3, per Jacobi sweep 2m^2 + m^2(m-1) for the dots and 3m^2(m-1)
    for the rotations (all sweeps but the last), wbar 8m^2, T 2m^3, update
    2 n m^2 + 2 n m."""
    fixed = m * (m + 1) * p_obs + 2 * m * p_obs + m ** 3 / 3 + 8 * m * m + 2 * m ** 3 + 2 * n_rows * m * m + 2 * n_rows * m
    return fixed + sweeps * (2 * m * m + m * m * (m - 1)) + (sweeps - 1) * 3 * m * m * (m - 1)


def run_global(K, W, NL, with_cpu: bool):
    """The global ETKF of Sec. 3.1 at its m = 197: one domain over a 32x32
    circular pupil (877 actuators, 812 subapertures), plain FP64 path (the
    m > 128 launch sequence)."""
    import torch

    from paper_1310_5954_amd import build_id
    from workload.configs import build_case
    cfg = dict(build_case(2).cfg)
    cfg.update(lenslets=32, frames=W + K + NL)
    case = build_case(cfg, m=197, global_map=True)
    ys = torch.tensor(np.stack([case.slopes(k) for k in range(W + K + NL)]), dtype=torch.float64, device="cuda:0")
    plain = run_plain(case, FP64_, K, W, NL, ys, tune=False)
    p_obs = 2 * case.n_sub
    sweeps = plain["sweeps"] / max(plain["solves"], 1)
    flops = big_analysis_flops(case.m, p_obs, 2 * case.n_act, sweeps)
    ana_ms = plain["kernel_ms"][1]
    achieved = flops / (ana_ms * 1e-3) / 1e12
    out = dict(metric="frames/s + p50/p99 frame latency (µs), global ETKF 32×32 subaps m=197",
               value=round(plain["fps"], 2), unit="frames/s", n_gpus=1, steps=K, warmup=W,
               ms_per_step=round(1e3 / plain["fps"], 4), higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64", data="synthetic",
               config=dict(workload=f"32x32 circular SH pupil, {case.n_act} actuators, {case.n_sub} subapertures, "
                                    f"m=197, one global domain; one frame = analysis + AR(2) forecast",
                           path="plain FP64, m > 128 launch sequence"),
               p50_us=round(plain["p50_us"], 1), p99_us=round(plain["p99_us"], 1),
               kernel_ms=dict(slopes=round(plain["kernel_ms"][0], 4), analysis=round(ana_ms, 4),
                              merge_forecast=round(plain["kernel_ms"][2], 4)),
               jacobi_sweeps_mean=round(sweeps, 3),
               roofline=dict(bound="alu", achieved=round(achieved, 4), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                             frac=round(achieved / PEAK_FP64_TFLOPS, 5), traffic=None,
                             kernel="the m > 128 analysis launch sequence (one domain: at most 7 workgroups per Jacobi round)"),
               library=build_id())
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline(case)
    return out


K_BAND = (0.5 / 2.2) ** 2   # phase variance at 2.2 um from the 500 nm of r0 (phase scales as 1 / wavelength)


def run_closed_loop(ms, frames: int, burn_in: int) -> dict:
    """The closed loop of Sec. 3 (workload.closed_loop) on a 32x32 pupil
    (877 actuators) with 5x5-actuator domains (stride 3, halo 2, taper),
    the plain FP64 filter for each ensemble size in `ms`; coherent energy
    against m, with the open loop and the truth-fed controller's floor."""
    from paper_1310_5954_amd import FP64, Filter, Problem, build_id
    from workload.closed_loop import ClosedLoop
    from workload.configs import build_case
    rows = []
    floor = None
    for m in ms:
        cfg = dict(build_case(2).cfg)
        cfg.update(lenslets=32, frames=frames + 2)
        case = build_case(cfg, m=m)
        cl = ClosedLoop(case)
        if floor is None:
            floor = cl.run(cl.perfect_step(), frames, burn_in)
        f = Filter(Problem.from_case(case), case.X0, precision=FP64, device="cuda:0")

        def step(y):
            f.step(y, pred=False)
            return f.last_means()
        t0 = time.perf_counter()
        r = cl.run(step, frames, burn_in)
        dt = time.perf_counter() - t0
        f.close()
        rows.append(dict(m=m, coherent_energy=r["coherent_energy"], residual_var_rad2=round(r["residual_var"], 4),
                         coherent_energy_2200nm=round(float(np.exp(-r["residual_var"] * K_BAND)), 5),
                         loop_frames_per_s=round(frames / dt, 1)))
        print(f"[bench] closed loop m={m}: residual {r['residual_var']:.3f} rad^2, E {r['coherent_energy']:.3e}",
              file=sys.stderr, flush=True)
    return dict(closed_loop=dict(workload=f"32x32 circular SH pupil, {case.n_act} actuators, {case.dmap.n_domains} "
                                          "5x5-actuator domains, FP64 plain path, 2-frame delay, DM coupling 0.3",
                                 frames=frames, burn_in=burn_in,
                                 open_loop_var_rad2=round(r["open_loop_var"], 3),
                                 truth_fed_floor_var_rad2=round(floor["residual_var"], 4),
                                 truth_fed_floor_coherent_energy=floor["coherent_energy"],
                                 truth_fed_floor_coherent_energy_2200nm=round(float(np.exp(-floor["residual_var"] * K_BAND)), 5),
                                 note="phases are at the 500 nm of r0; *_2200nm scales the variance by (0.5/2.2)^2",
                                 by_m=rows), library=build_id())


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), as lscpu reports it."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores(cap: int = 16) -> int:
    """Cores this process may run on, at most `cap` (a GPU machine's CPU share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


_CPU = {}   # per worker process of the CPU baseline: shared arrays and the domain map


def _cpu_init(shm_names, shapes, dmap, n_act, n_sub, r_inv, rho):
    from multiprocessing import shared_memory

    from threadpoolctl import threadpool_limits
    _CPU["limit"] = threadpool_limits(limits=1)          # BLAS at one thread per worker
    _CPU["shm"] = [shared_memory.SharedMemory(name=n) for n in shm_names]
    _CPU["arr"] = [np.ndarray(sh, dtype=np.float64, buffer=m.buf) for m, sh in zip(_CPU["shm"], shapes)]
    _CPU.update(dmap=dmap, n_act=n_act, n_sub=n_sub, r_inv=r_inv, rho=rho)


def _cpu_domains(ls):
    """The oracle's per-domain analysis of domains `ls`; Z rows into the shared output."""
    import oracle
    from oracle.letkf import domain_rows
    Xp, xbar, Yp, d, Z = _CPU["arr"]
    dm = _CPU["dmap"]
    for l in ls:
        E, O, srows, orows = domain_rows(dm, l, _CPU["n_act"], _CPU["n_sub"])
        taper = np.asarray(dm.taper(l), dtype=float)
        r_O = np.concatenate([taper, taper]) * _CPU["r_inv"][orows]
        res = oracle.domain_analysis(Xp[srows], xbar[srows], Yp[orows], d[orows], r_O, _CPU["rho"])
        z0 = 2 * int(dm.est_ptr[l])
        Z[z0:z0 + len(srows)] = res["Z"]
    return len(ls)


def cpu_baseline_pool(case, seconds: float, cores: int):
    """The FP64 oracle on `cores` host cores: per frame the parent forms the
    ensemble mean, perturbations and slopes (oracle.letkf), a pool of worker
    processes (one per core, BLAS at one thread each, started before the GPU
    is touched) runs the oracle's domain analysis on interleaved shares of the
    domains through shared memory, and the parent merges and forecasts.
    Frames of the same workload until `seconds` have passed (at least two)."""
    import multiprocessing as mp
    from multiprocessing import shared_memory

    import scipy.sparse as sp

    import oracle
    from oracle.letkf import domain_rows
    D = sp.csr_matrix((case.D.val, case.D.col, case.D.rowptr), shape=case.D.shape)
    dm, m, n_act, n_sub = case.dmap, case.m, case.n_act, case.n_sub
    zrows = 2 * int(dm.est_ptr[-1])
    shapes = [(2 * n_act, m), (2 * n_act,), (2 * n_sub, m), (2 * n_sub,), (zrows, m)]
    shms = [shared_memory.SharedMemory(create=True, size=int(np.prod(sh)) * 8) for sh in shapes]
    try:
        Xp_s, xbar_s, Yp_s, d_s, Z_s = (np.ndarray(sh, dtype=np.float64, buffer=mm.buf) for mm, sh in zip(shms, shapes))
        shares = [list(range(k, dm.n_domains, cores)) for k in range(cores)]
        ctx = mp.get_context("fork")
        with ctx.Pool(cores, initializer=_cpu_init,
                      initargs=([mm.name for mm in shms], shapes, dm, n_act, n_sub, case.r_inv, case.inflation)) as pool:
            X = case.X0.copy()
            times = []
            t0 = time.perf_counter()
            k = 0
            while k < 2 or time.perf_counter() - t0 < seconds:
                y = case.slopes(k)
                ts = time.perf_counter()
                xbar, Xp = oracle.ensemble_mean_perturbations(X)
                ybar, Yp = oracle.slope_synthesis(D, X, n_act)
                Xp_s[:], xbar_s[:], Yp_s[:], d_s[:] = Xp, xbar, Yp, y - ybar
                pool.map(_cpu_domains, shares)
                Xa = np.zeros_like(X)
                for l in range(dm.n_domains):       # the oracle's merge
                    E, O, srows, orows = domain_rows(dm, l, n_act, n_sub)
                    w = np.asarray(dm.weights(l), dtype=float)
                    z0 = 2 * int(dm.est_ptr[l])
                    Xa[srows] += np.concatenate([w, w])[:, None] * Z_s[z0:z0 + len(srows)]
                X = oracle.forecast(Xa, case.a1, case.a2, case.sigma_v, case.philox_seed, k)
                times.append(time.perf_counter() - ts)
                k += 1
    finally:
        for mm in shms:
            mm.close()
            mm.unlink()
    return len(times) / float(np.sum(times)), len(times)


def cpu_baseline(case, seconds: float = 12.0, single_seconds: float = 6.0):
    """The FP64 oracle timed on the host: over the host's cores (a process pool,
    the plan of the baseline) and on one core, each on the first frames of the
    same workload for about `seconds` / `single_seconds`."""
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    import oracle
    cores = host_cores()
    fps, n_pool = cpu_baseline_pool(case, seconds, cores)
    D = sp.csr_matrix((case.D.val, case.D.col, case.D.rowptr), shape=case.D.shape)
    X = case.X0.copy()
    ys = []
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        k = 0
        while k < 2 or time.perf_counter() - t0 < single_seconds:
            y = case.slopes(k)
            ts = time.perf_counter()
            Xa = oracle.analysis(X, y, D, case.dmap, case.r_inv, case.inflation)
            X = oracle.forecast(Xa, case.a1, case.a2, case.sigma_v, case.philox_seed, k)
            ys.append(time.perf_counter() - ts)
            k += 1
    fps1 = len(ys) / float(np.sum(ys))
    L_ = case.cfg["lenslets"]
    return dict(value=round(fps, 3), unit="frames/s", cores=cores, kind="oracle",
                cpu=cpu_model(),
                sample=f"first {n_pool} frames of the same {L_}x{L_}, m={case.m} workload: NumPy/LAPACK FP64 oracle, "
                       f"domains over a pool of {cores} worker processes (BLAS at 1 thread each)",
                single_core=dict(value=round(fps1, 3), unit="frames/s", cores=1,
                                 sample=f"first {len(ys)} frames, oracle.analysis + forecast on one thread"))


PISTONS = False  # set from --pistons
TUNE = True      # autotune the analysis launch of every filter / server class first (--no-tune: defaults)
GRAPHS = False   # server batches replayed from captured graphs (--server-graphs 1); measured slower here
MAX_BATCH = 0    # frames per server batch (--max-batch; 0: half the instances, so that two batches
                 # alternate and each one's host turnaround overlaps the other's kernels)


def run_plain(case, prec, K, W, NL, ys, tune=True):
    """Plain per-frame path on one instance: throughput, latency, kernel times."""
    import torch

    from paper_1310_5954_amd import Filter, Problem
    f = Filter(Problem.from_case(case), case.X0, precision=prec, device="cuda:0", pistons=PISTONS)
    for k in range(W):
        f.step(ys[k], pred=False)
    # tuned on the live ensemble after the warm-up frames (the balanced order
    # places the domains by their sweeps so far); state and counters unchanged
    tuning = f.autotune() if (TUNE and tune) else None
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
    lat = []
    for k in range(W + K, W + K + NL):
        ts = time.perf_counter()
        f.step(ys[k], pred=True)
        lat.append(time.perf_counter() - ts)
    assert f.unconverged() == 0
    f.close()
    lat_us = np.array(lat) * 1e6
    return dict(fps=K / (t1 - t0), p50_us=float(np.percentile(lat_us, 50)), p99_us=float(np.percentile(lat_us, 99)),
                kernel_ms=[v / K for v in ms], sweeps=sw1 - sw0, solves=so1 - so0, tuning=tuning)


def run_plain_graph(case, K, W, NL, ys):
    """The plain FP64 path with the frame's launch sequence replayed from a
    captured hipGraph (LETKF_FLAG_GRAPH): throughput and latency only (kernel
    timing would switch the replay off)."""
    import torch

    from paper_1310_5954_amd import FP64, Filter, Problem
    f = Filter(Problem.from_case(case), case.X0, precision=FP64, device="cuda:0", pistons=PISTONS, graph=True)
    for k in range(W // 2):
        f.step(ys[k], pred=False)
    if TUNE:
        f.autotune()
    for k in range(W // 2, W):  # the frame graph is captured again after tuning
        f.step(ys[k], pred=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(W, W + K):
        f.step(ys[k], pred=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat = []
    for k in range(W + K, W + K + NL):
        ts = time.perf_counter()
        f.step(ys[k], pred=True)
        lat.append(time.perf_counter() - ts)
    assert f.unconverged() == 0
    f.close()
    lat_us = np.array(lat) * 1e6
    return dict(fps=K / (t1 - t0), p50_us=float(np.percentile(lat_us, 50)), p99_us=float(np.percentile(lat_us, 99)))


def run_plain_loaded(case, B, K, W, ys):
    """The plain per-frame FP64 path under the serving load: B resident
    instances in a closed loop (an instance releases its next frame when the
    previous one is done), served one frame at a time in release order through
    letkf_step.  Latency = release to prediction on the host."""
    import collections

    from paper_1310_5954_amd import FP64, Filter, Problem
    pr = Problem.from_case(case)
    fs = [Filter(pr, np.roll(case.X0, i, axis=1), precision=FP64, device="cuda:0", pistons=PISTONS)
          for i in range(B)]
    if TUNE:
        for f in fs:
            f.autotune()
    t_start = time.perf_counter()
    queue = collections.deque((i, 0, t_start) for i in range(B))
    lat, t0, timed = [], None, 0
    while queue:
        i, k, rel = queue.popleft()
        if k == W and t0 is None and all(kk >= W for _, kk, _ in queue):
            t0 = time.perf_counter()
        fs[i].step(ys[(k + 7 * i) % len(ys)], pred=True)
        done = time.perf_counter()
        if k >= W:
            lat.append(done - rel)
            timed += 1
        if k + 1 < W + K:
            queue.append((i, k + 1, done))
    t1 = time.perf_counter()
    for f in fs:
        assert f.unconverged() == 0
        f.close()
    lat_us = np.array(lat) * 1e6
    return dict(fps=B * K / (t1 - t0), p50_us=float(np.percentile(lat_us, 50)),
                p99_us=float(np.percentile(lat_us, 99)))


def run_serving(case, prec, B, K, W, ys, depth=1, NL=0, fp32_rotations=False):
    """B resident instances in a closed loop through the batching server, each
    keeping `depth` frames submitted (depth 1: a frame is submitted when the
    previous one of that instance is done).  Frames W .. W+K-1 of every
    instance are timed (throughput: their count over the span from the first
    one's submission to the last one's completion); latency = submit to
    callback over frames W .. W+K+NL-1, so the loop continues for NL frames
    per instance past the timed ones.  ys: device slopes (a CUDA tensor, read
    in place) or host slopes (a numpy array, copied at submission)."""
    import threading

    import torch

    from paper_1310_5954_amd import Problem, Server
    from paper_1310_5954_amd import _lib as L
    pr = Problem.from_case(case)
    flags = (L.FLAG_PISTONS if PISTONS else 0) | (L.FLAG_FP32_ROTATIONS if fp32_rotations else 0)
    budget = B * pr.workspace_size(prec, flags) + L.lib().letkf_server_reserved_bytes() + (16 << 20)
    # instance i starts from the ensemble shifted by i columns and reads frame k + 7 i of the slope stream
    total = W + K + NL
    state = dict(t_sub={}, t_done={}, done=0)
    cv = threading.Condition()
    preds = [np.empty(case.n_act) for _ in range(B)]

    def submit(i, k):
        fid = i * 1_000_000 + k
        state["t_sub"][fid] = time.perf_counter()
        rc = srv.submit(insts[i], ys[(k + 7 * i) % len(ys)], fid, preds[i])
        assert rc == 0, rc

    def on_done(fid, status, t):
        assert status == 0, status
        i, k = divmod(fid, 1_000_000)
        state["t_done"][fid] = t
        if k + depth < total:
            submit(i, k + depth)
        with cv:
            state["done"] += 1
            cv.notify_all()

    srv = Server(budget, on_done=on_done, graphs=GRAPHS, max_batch=MAX_BATCH or max(1, (B + 1) // 2))
    insts = [srv.add(pr, np.roll(case.X0, i, axis=1), prec, pistons=PISTONS, fp32_rotations=fp32_rotations)
             for i in range(B)]
    tuning = list(srv.autotune().values())[0] if TUNE else None
    torch.cuda.synchronize()
    # warm-up frames 0..W-1 run in the same closed loop; the clock starts when every instance has finished them
    with cv:
        for k in range(min(depth, total)):
            for i in range(B):
                submit(i, k)
    with cv:
        cv.wait_for(lambda: state["done"] >= B * total, timeout=600)
    srv.drain()
    st = srv.stats()
    srv.close()
    # timed frames: W <= k < W + K of every instance, on the completion thread's
    # clock, so the main thread's wake-ups do not enter it
    timed = [i * 1_000_000 + k for i in range(B) for k in range(W, W + K)]
    sampled = [i * 1_000_000 + k for i in range(B) for k in range(W, total)]
    lat_us = np.array([state["t_done"][f] - state["t_sub"][f] for f in sampled]) * 1e6
    span = max(state["t_done"][f] for f in timed) - min(state["t_sub"][f] for f in timed)
    return dict(fps=len(timed) / span, p50_us=float(np.percentile(lat_us, 50)),
                p99_us=float(np.percentile(lat_us, 99)), latency_frames=len(sampled), batches=st["batches"],
                mean_batch=st["batched_frames"] / max(st["batches"], 1), tuning=tuning)


def run_mix(seconds: float, rate_scale: float, window_us: int):
    """Six resident instances of different pupils, ensemble sizes and paths
    (FP32 / BF16 contractions) admitted into one server by HBM budget; each
    receives frames as an independent Poisson stream.  Smaller instances get
    the higher rates (2000 Hz ... 500 Hz, times rate_scale).  Latency = the
    frame's scheduled arrival time -> completion callback, so pacing jitter of
    the submitting thread counts against the server."""
    import threading

    import torch

    from paper_1310_5954_amd import BF16, FP32, Problem, Server, build_id
    from workload.configs import (PREC_BF16, SERVING_INSTANCES, SERVING_RATES_HZ, build_case,
                                  serving_config)
    cases = [build_case(serving_config(i)) for i in range(len(SERVING_INSTANCES))]
    precs = [BF16 if SERVING_INSTANCES[i][2] == PREC_BF16 else FP32 for i in range(len(cases))]
    rates = [rate_scale * r for r in sorted(SERVING_RATES_HZ, reverse=True)]
    probs = [Problem.from_case(c) for c in cases]
    need = sum(pr.workspace_size(pc) for pr, pc in zip(probs, precs))
    budget = need + (64 << 20)
    NF = 64
    ys = [torch.tensor(np.stack([c.slopes(k) for k in range(NF)]), dtype=torch.float64, device="cuda:0")
          for c in cases]
    rng = np.random.default_rng(4)
    arrivals = []
    for i, r in enumerate(rates):
        t = 0.0
        while True:
            t += rng.exponential(1.0 / r)
            if t >= seconds:
                break
            arrivals.append((t, i))
    arrivals.sort()
    B = len(cases)
    sched, lat, done_t = {}, [[] for _ in range(B)], []
    lock = threading.Lock()
    preds = [np.empty(c.n_act) for c in cases]

    def on_done(fid, status, t):
        assert status == 0, status
        i = fid >> 32
        with lock:
            lat[i].append(t - sched.pop(fid))
            done_t.append(t)

    srv = Server(budget, on_done=on_done, graphs=GRAPHS)
    srv.set_window(window_us)
    insts = [srv.add(pr, c.X0, pc) for pr, c, pc in zip(probs, cases, precs)]
    if TUNE:
        srv.autotune()
    torch.cuda.synchronize()
    # one untimed frame per instance so every kernel variant is loaded
    for i in range(B):
        sched[(i << 32) | 0xFFFFFFFF] = time.perf_counter()
        assert srv.submit(insts[i], ys[i][0], (i << 32) | 0xFFFFFFFF, preds[i]) == 0
    srv.drain()
    for L in lat:
        L.clear()
    done_t.clear()
    counts, drops = [0] * B, [0] * B
    # completion callbacks run Python code (they need the GIL): hand the GIL
    # over often and sleep through long gaps so that they are not held back
    # by the submitting loop
    switch = sys.getswitchinterval()
    sys.setswitchinterval(2e-5)
    t0 = time.perf_counter()
    for ta, i in arrivals:
        gap = ta - (time.perf_counter() - t0)
        if gap > 3e-4:
            time.sleep(gap - 2e-4)
        while time.perf_counter() - t0 < ta:
            pass
        k = counts[i]
        fid = (i << 32) | k
        with lock:
            sched[fid] = t0 + ta
        if srv.submit(insts[i], ys[i][k % NF], fid, preds[i]) != 0:
            drops[i] += 1
            with lock:
                sched.pop(fid)
        counts[i] += 1
    srv.drain()
    sys.setswitchinterval(switch)
    st = srv.stats()
    srv.close()
    per = []
    for i, c in enumerate(cases):
        L = np.array(lat[i]) * 1e6
        per.append(dict(lenslets=c.cfg["lenslets"], n_act=c.n_act, m=c.m, domains=c.dmap.n_domains,
                        path="bf16" if precs[i] == BF16 else "fp32", rate_hz=round(rates[i], 1),
                        frames=int(len(L)), dropped=drops[i],
                        p50_us=round(float(np.percentile(L, 50)), 1) if len(L) else None,
                        p99_us=round(float(np.percentile(L, 99)), 1) if len(L) else None))
    all_lat = np.concatenate([np.array(L) for L in lat]) * 1e6
    span = max(done_t) - t0
    return dict(metric="serving mix: frames/s + p50/p99 frame latency (us), 6 AO instances, Poisson arrivals",
                value=round(len(all_lat) / span, 1), unit="frames/s", n_gpus=1, seconds=seconds,
                rate_scale=rate_scale, offered_fps=round(sum(rates), 1), p50_us=round(float(np.percentile(all_lat, 50)), 1),
                p99_us=round(float(np.percentile(all_lat, 99)), 1), mean_batch=round(st["batched_frames"] / max(st["batches"], 1), 3),
                hbm_budget_bytes=int(budget), instances=per, data="synthetic", library=build_id())


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--instances", type=int, default=4)
    ap.add_argument("--precision", default="bf16", choices=["fp64", "fp32", "bf16"],
                    help="precision path of the serving form (the plain form is always FP64)")
    ap.add_argument("--phases-precision", default="fp64", choices=["fp64", "fp32", "bf16"],
                    help="--phases: precision path of the debug instance")
    ap.add_argument("--latency-frames", type=int, default=500,
                    help="plain path: frames timed one by one for the latency percentiles")
    ap.add_argument("--serving-latency-frames", type=int, default=500,
                    help="serving: at least this many frames in the latency percentiles (the closed loop "
                         "continues past the timed frames)")
    ap.add_argument("--fp32-rotations", action="store_true",
                    help="--serving-only: the opt-in FP32 Jacobi rotations (BF16 path)")
    ap.add_argument("--plain-only", action="store_true",
                    help="only the plain per-frame path (precision --plain-precision)")
    ap.add_argument("--plain-precision", default="fp64", choices=["fp64", "fp32", "bf16"],
                    help="--plain-only: precision path of the plain instance")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mix", type=float, default=0.0, metavar="SECONDS",
                    help="instead of the headline run: six mixed instances with Poisson arrivals for SECONDS")
    ap.add_argument("--rate-scale", type=float, default=1.0, help="--mix: multiplies every arrival rate")
    ap.add_argument("--window-us", type=int, default=100, help="server batching window (microseconds)")
    ap.add_argument("--workload", type=int, default=84, choices=[84, 128, 32],
                    help="84: 84x84 subapertures, m = 64 (headline); 128: 128x128, m = 128; "
                         "32: global ETKF, 32x32 subapertures, m = 197 (plain FP64 only)")
    ap.add_argument("--partitions", type=int, default=1, choices=[1, 2],
                    help="2: the window partition plus one staggered by half a stride, averaged (Sec. 5)")
    ap.add_argument("--pistons", action="store_true",
                    help="remove the differential pistons between domains before the merge (Sec. 3.2)")
    ap.add_argument("--serving-only", action="store_true",
                    help="skip the plain-path runs (for profiling the serving kernels); no roofline line")
    ap.add_argument("--max-batch", type=int, default=0,
                    help="server: most frames in one batch (0: half the instances, two batches alternate)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip autotuning the analysis launch shapes (default grid and order)")
    ap.add_argument("--server-graphs", type=int, default=0, choices=[0, 1],
                    help="1: server batches replayed from captured hipGraphs; 0: launched one by one")
    ap.add_argument("--closed-loop", action="store_true",
                    help="only the closed-loop coherent energy against m (32x32 pupil, FP64), 300 frames each")
    ap.add_argument("--phases", action="store_true",
                    help="only report per-phase cycles and bytes of the FP64 analysis (debug stamps), one frame")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps(dict(error="the library runs on one GPU only; --gpus must be 1")))
        return 2

    import torch

    if args.copy_ref:
        nbytes = 512 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_ref_bytes_read=nbytes, copy_ref_bytes_written=nbytes, dispatches=5)))
        return 0

    global PISTONS, TUNE, GRAPHS, MAX_BATCH
    PISTONS = args.pistons
    TUNE = not args.no_tune
    GRAPHS = bool(args.server_graphs)
    MAX_BATCH = args.max_batch
    if args.closed_loop:
        print(json.dumps(run_closed_loop((8, 16, 32, 64, 128), 300, 100)), flush=True)
        return 0
    if args.workload == 32:
        print(json.dumps(run_global(args.steps, args.warmup, args.latency_frames, not args.no_cpu_baseline)),
              flush=True)
        return 0
    if args.mix > 0:
        print(json.dumps(run_mix(args.mix, args.rate_scale, args.window_us)), flush=True)
        return 0

    from paper_1310_5954_amd import BF16, FP32, FP64, build_id
    from paper_1310_5954_amd.build import kernel_hash
    from workload.configs import build_case

    prec = dict(fp64=FP64, fp32=FP32, bf16=BF16)[args.precision]
    case = build_case(3 if args.workload == 84 else 5, partitions=args.partitions)
    K, W, NL, B = args.steps, args.warmup, args.latency_frames, args.instances
    NLS = -(-max(0, args.serving_latency_frames - B * K) // B)  # serving frames per instance past the timed ones
    n_frames = W + K + NL
    L_ = case.cfg["lenslets"]
    print(f"[bench] {L_}x{L_} m={case.m} domains={case.dmap.n_domains} library={build_id()} frames={n_frames}",
          file=sys.stderr, flush=True)
    # the CPU baseline's worker processes are forked before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline and not (args.phases or args.serving_only):
        cpu = cpu_baseline(case)
        print(f"[bench] cpu baseline (oracle): {cpu['value']:.2f} frames/s on {cpu['cores']} cores "
              f"({cpu['cpu']}), {cpu['single_core']['value']:.2f} frames/s on one", file=sys.stderr, flush=True)
    ys_host = np.stack([case.slopes(k) for k in range(max(n_frames, W + K + NLS))])
    ys = torch.tensor(ys_host, dtype=torch.float64, device="cuda:0")

    if args.phases:
        prec = None if args.phases_precision == "fp64" else dict(fp32=FP32, bf16=BF16)[args.phases_precision]
        print(json.dumps(dict(phases=run_phases(case, W, ys, prec), precision=args.phases_precision,
                              library=build_id())), flush=True)
        return 0
    if args.serving_only:
        lat = run_serving(case, prec, B, K, W, ys, depth=1, NL=NLS, fp32_rotations=args.fp32_rotations)
        print(json.dumps(dict(metric=METRIC, value=round(lat["fps"], 2), unit="frames/s", n_gpus=1, steps=K,
                              warmup=W, p50_us=round(lat["p50_us"], 1), p99_us=round(lat["p99_us"], 1),
                              latency_frames=lat["latency_frames"], mean_batch=round(lat["mean_batch"], 3),
                              precision=args.precision, fp32_rotations=args.fp32_rotations,
                              graphs=GRAPHS, tuning=lat["tuning"], library=build_id())), flush=True)
        return 0

    def roofline_of(run, path_name):
        """Algorithmic FP64-dominated work of one analysis launch over its
        HIP-event duration; HBM traffic from the committed counter summary."""
        ana_ms = run["kernel_ms"][1]
        flops = analysis_flops(case.m, case.dmap, run["sweeps"], run["solves"], K) / K
        achieved = flops / (ana_ms * 1e-3) / 1e12
        es = 8 if path_name == "fp64" else 4
        traffic = measured_traffic(TRAFFIC_FILES[path_name], kernel_hash(), run["tuning"]) if args.workload == 84 else None
        uniq = unique_bytes(case, es)
        return dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP64_TFLOPS, 4), traffic=traffic,
                    unique_bytes=uniq, traffic_over_unique=round(traffic / uniq, 3) if traffic else None,
                    kernel_us=round(ana_ms * 1e3, 2), flops_per_launch=round(flops),
                    jacobi_sweeps_mean=round(run["sweeps"] / max(run["solves"], 1), 3))

    if args.plain_only and args.plain_precision != "fp64":
        pp = dict(fp32=FP32, bf16=BF16)[args.plain_precision]
        run = run_plain(case, pp, K, W, NL, ys)
        rl = roofline_of(run, args.plain_precision)
        rl["kernel"] = f"k_analysis<{args.plain_precision.upper()}, m={case.m}>, one instance per launch"
        out = dict(metric=METRIC, value=round(run["fps"], 2), unit="frames/s", n_gpus=1, steps=K, warmup=W,
                   ms_per_step=round(1e3 / run["fps"], 4), higher_is_better=True, scaling="weak", vs_baseline=None,
                   dtype={"fp32": "f32+f64", "bf16": "bf16+f64"}[args.plain_precision], data="synthetic",
                   config=dict(workload=f"{L_}x{L_} circular SH pupil, m={case.m}, {case.dmap.n_domains} domains",
                               path="plain", precision=args.plain_precision),
                   p50_us=round(run["p50_us"], 1), p99_us=round(run["p99_us"], 1), roofline=rl,
                   tuning=run["tuning"], library=build_id())
        print(json.dumps(out), flush=True)
        return 0
    plain = run_plain(case, FP64, K, W, NL, ys)
    print(f"[bench] plain fp64: {plain['fps']:.1f} frames/s p50 {plain['p50_us']:.0f} us "
          f"p99 {plain['p99_us']:.0f} us", file=sys.stderr, flush=True)
    graph = run_plain_graph(case, K, W, NL, ys)
    print(f"[bench] plain fp64, graph replay: {graph['fps']:.1f} frames/s p50 {graph['p50_us']:.0f} us "
          f"p99 {graph['p99_us']:.0f} us", file=sys.stderr, flush=True)
    rf64 = roofline_of(plain, "fp64")
    rf64["kernel"] = f"k_analysis<FP64, m={case.m}> (vector FP64: Cholesky + one-sided Jacobi dominate)"
    plain_out = dict(frames_per_s=round(plain["fps"], 2), p50_us=round(plain["p50_us"], 1),
                     p99_us=round(plain["p99_us"], 1), latency_frames=NL,
                     kernel_ms=dict(slopes=round(plain["kernel_ms"][0], 4), analysis=round(plain["kernel_ms"][1], 4),
                                    merge_forecast=round(plain["kernel_ms"][2], 4)),
                     jacobi_sweeps_mean=round(plain["sweeps"] / max(plain["solves"], 1), 3),
                     graph_replay=dict(frames_per_s=round(graph["fps"], 2), p50_us=round(graph["p50_us"], 1),
                                       p99_us=round(graph["p99_us"], 1)),
                     tuning=plain["tuning"], roofline=rf64)
    if args.plain_only:
        out = dict(metric=METRIC if args.workload == 84 else METRIC.replace("84×84", "128×128").replace("m=64", "m=128"),
                   value=round(plain["fps"], 2), unit="frames/s", n_gpus=1, steps=K, warmup=W,
                   ms_per_step=round(1e3 / plain["fps"], 4), higher_is_better=True, scaling="weak", vs_baseline=None,
                   dtype="f64", data="synthetic",
                   config=dict(workload=f"{L_}x{L_} circular SH pupil, m={case.m}, {case.dmap.n_domains} domains",
                               path="plain", precision="fp64"),
                   p50_us=round(plain["p50_us"], 1), p99_us=round(plain["p99_us"], 1), roofline=rf64,
                   plain_fp64=plain_out, library=build_id())
        if cpu:
            out["cpu_baseline"] = cpu
        print(json.dumps(out), flush=True)
        return 0
    # the serving path's analysis kernel, one instance per launch (HIP events on its stream)
    plain_s = run_plain(case, prec, K, W, min(NL, 50), ys)
    print(f"[bench] plain {args.precision}: analysis {plain_s['kernel_ms'][1] * 1e3:.1f} us per launch",
          file=sys.stderr, flush=True)
    roofline = roofline_of(plain_s, "bf16" if prec == BF16 else ("fp64" if prec == FP64 else "fp32"))
    roofline["kernel"] = (f"k_analysis<{args.precision.upper()}, m={case.m}>, the serving path's analysis kernel, "
                          f"one instance ({case.dmap.n_domains} domains) per launch (vector FP64: Cholesky + one-sided "
                          f"Jacobi dominate; C and X'T on {args.precision.upper()} MFMA)")
    loaded = run_plain_loaded(case, B, K, W, ys)
    print(f"[bench] plain fp64 x{B} closed loop: {loaded['fps']:.1f} frames/s p50 {loaded['p50_us']:.0f} us "
          f"p99 {loaded['p99_us']:.0f} us", file=sys.stderr, flush=True)
    lat = run_serving(case, prec, B, K, W, ys, depth=1, NL=NLS)
    print(f"[bench] serving {args.precision} x{B} closed loop: {lat['fps']:.1f} frames/s p50 {lat['p50_us']:.0f} us "
          f"p99 {lat['p99_us']:.0f} us ({lat['latency_frames']} latency frames), mean batch {lat['mean_batch']:.2f}",
          file=sys.stderr, flush=True)
    host = run_serving(case, prec, B, K, W, ys_host, depth=1, NL=NLS)
    print(f"[bench] serving {args.precision}, host slopes: {host['fps']:.1f} frames/s p50 {host['p50_us']:.0f} us "
          f"p99 {host['p99_us']:.0f} us", file=sys.stderr, flush=True)
    rot32 = None
    if prec == BF16:
        rot32 = run_serving(case, prec, B, K, W, ys, depth=1, NL=NLS, fp32_rotations=True)
        print(f"[bench] serving bf16 with FP32 rotations: {rot32['fps']:.1f} frames/s p50 {rot32['p50_us']:.0f} us "
              f"p99 {rot32['p99_us']:.0f} us", file=sys.stderr, flush=True)
    # whole-job rate of the serving form: the analysis kernel's algorithmic work per frame at `value` frames/s
    flops_frame = roofline["flops_per_launch"]
    roofline["serving_wall"] = dict(achieved=round(flops_frame * lat["fps"] / 1e12, 3),
                                    frac=round(flops_frame * lat["fps"] / 1e12 / PEAK_FP64_TFLOPS, 4),
                                    note="analysis work per frame x serving frames/s (wall clock, batches overlap)")
    mb = MAX_BATCH or max(1, (B + 1) // 2)
    path = (f"serving: {B} resident instances in a closed loop (each submits its next frame when the previous one "
            f"is done), continuous batching through the server in batches of at most {mb} frames, device-resident "
            f"slopes; latency = submit to completion callback")
    dname = {FP64: "f64", FP32: "f32+f64", BF16: "bf16+f64"}
    pname = {FP64: "fp64", FP32: "fp32 contractions (FP32 MFMA), FP64 eigensolve, wbar and W",
             BF16: "bf16 contractions (BF16 MFMA, FP32 accumulation), FP64 eigensolve (Cholesky, Jacobi rotations), "
                   "FP64 wbar and W"}
    out = dict(
        metric=METRIC if args.workload == 84 else METRIC.replace("84×84", "128×128").replace("m=64", "m=128"),
        value=round(lat["fps"], 2), unit="frames/s", n_gpus=1, steps=K, warmup=W,
        ms_per_step=round(1e3 * B / lat["fps"], 4), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype=dname[prec], data="synthetic",
        config=dict(workload=f"{L_}x{L_} circular SH pupil, {case.n_act} actuators (n={2 * case.n_act}), "
                             f"{case.n_sub} subapertures (p={2 * case.n_sub}), "
                             f"m={case.m}, {case.dmap.n_domains} overlapping 6x6-actuator domains"
                             + (" (two staggered partitions, averaged)" if args.partitions == 2 else "")
                             + (", differential pistons removed before the merge" if args.pistons else "")
                             + ", halo 2, Gaspari-Cohn taper; one frame = analysis + AR(2) forecast",
                    path=path, precision=pname[prec]),
        p50_us=round(lat["p50_us"], 1), p99_us=round(lat["p99_us"], 1), latency_frames=lat["latency_frames"],
        roofline=roofline,
        serving=dict(instances=B, max_batch=mb, mean_batch=round(lat["mean_batch"], 3), graphs=GRAPHS,
                     tuning=lat["tuning"],
                     beats_plain_fp64=bool(lat["fps"] > loaded["fps"] and lat["p99_us"] < loaded["p99_us"]),
                     host_slopes=dict(frames_per_s=round(host["fps"], 2), p50_us=round(host["p50_us"], 1),
                                      p99_us=round(host["p99_us"], 1), latency_frames=host["latency_frames"],
                                      note="slopes submitted from host memory (letkf_submit_frame): 88 KB H2D "
                                           "per frame inside the latency")),
        plain_fp64=dict(plain_out, closed_loop=dict(instances=B, frames_per_s=round(loaded["fps"], 2),
                                                    p50_us=round(loaded["p50_us"], 1), p99_us=round(loaded["p99_us"], 1))),
        library=build_id(),
    )
    if rot32:
        out["serving_fp32_rotations"] = dict(frames_per_s=round(rot32["fps"], 2), p50_us=round(rot32["p50_us"], 1),
                                             p99_us=round(rot32["p99_us"], 1), latency_frames=rot32["latency_frames"],
                                             note="opt-in LETKF_FLAG_FP32_ROTATIONS: the Jacobi rotations in FP32, a "
                                                  "departure from the FP64 eigensolve")
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
