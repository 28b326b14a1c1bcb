"""Benchmark: spin-flip attempts/ns of the non-equilibrium Renyi-entropy
estimator on one MI355X.

Workload (one step): the 2D 64x64 job set -- 64 jobs l = 0..63 (S_2 for
l = 1..64), n = 2, beta_c, N = 1000 protocol sweeps after 100 thermalisation
sweeps, 1024 trajectories per job, int8 spins -- run through the persistent
batched path (one fused sweep+work launch over all 65536 trajectories, then
the estimator launch), followed by the host assembly of S_2(l) and C_2(x).
Inputs are synthetic (the job descriptions); every spin and uniform is drawn
on the device.

Prints one JSON line.  --gpus N > 1 is not supported (one-GPU build).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E
# Algorithmic HBM bytes of one Metropolis attempt: an int8 spin read and
# written once per sweep.  The persistent kernel keeps every lattice in LDS
# and moves far less (the measured traffic is reported beside it); the
# figure is the per-attempt traffic of the method streamed at one byte per
# spin, the basis on which the HBM roofline of the path is stated.
BYTES_PER_ATTEMPT = 2.0
# The HBM-streaming path as built: one launch per colour, each reading the
# opposite plane and reading and writing its own plane, i.e. 3 bytes per
# site per sweep.
STREAM_BYTES_PER_ATTEMPT = 3.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_kernel_2d64_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2304_03311_amd", "csrc", f)
                  for f in ("ee_kernels.hip", "ee_internal.hpp", "ee_dd.hpp", "ee_lanes.hpp")]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def hbm_frac(attempts: float, seconds: float, bytes_per_attempt: float = BYTES_PER_ATTEMPT) -> float:
    return bytes_per_attempt * attempts / seconds / 1e9 / PEAK_HBM_GBPS


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_range(args):
    """One worker of the parallel CPU leg: trajectories [j0, j1) of a job."""
    from oracle import oracle as eo
    spec, n_therm, j0, j1 = args
    job = eo.Job(*spec)
    t0 = time.perf_counter()
    eo.run(job, n_therm, j0, j1)
    return time.perf_counter() - t0


def cpu_baseline(n_traj_sample: int, procs: int | None = None) -> dict:
    """The CPU oracle on the host: one process on trajectories 0..n-1 of the
    l = 32 job of the 2D 64x64 set, then P processes (the host's usable
    cores, at most 16) on n trajectories each, disjoint.  Runs before the GPU
    is touched (the workers are forked)."""
    import multiprocessing as mp
    from oracle import oracle as eo
    from paper_2304_03311_amd import workloads
    s = workloads.config2_jobs()[32]
    spec = (s.dim, s.lt, s.lx, s.ly, s.n, s.beta, s.l, s.n_step, s.n_traj, s.seed)
    per_traj = s.sites * (workloads.N_THERM + s.n_step)
    t0 = time.perf_counter()
    eo.run(eo.Job(*spec), workloads.N_THERM, 0, n_traj_sample)
    dt1 = time.perf_counter() - t0
    if procs is None:
        procs = min(16, len(os.sched_getaffinity(0)))
    ranges = [(spec, workloads.N_THERM, p * n_traj_sample, (p + 1) * n_traj_sample) for p in range(procs)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        pool.map(_oracle_range, ranges)
    dtp = time.perf_counter() - t0
    att1 = n_traj_sample * per_traj
    attp = procs * n_traj_sample * per_traj
    return {"value": attp / (dtp * 1e9), "unit": "attempts/ns", "cores": procs, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": f"job l=32 of the 2D 64x64 set: {procs} processes of the single-threaded C oracle, "
                      f"{n_traj_sample} disjoint trajectories each ({attp:.3g} attempts, {dtp:.1f} s wall)",
            "single_core": {"value": att1 / (dt1 * 1e9), "cores": 1,
                            "sample": f"trajectories 0..{n_traj_sample - 1} ({att1:.3g} attempts, {dt1:.1f} s)"}}


def serving_run(n_jobs: int, rate: float = 200.0) -> dict:
    """The serving loop on a Poisson stream of n_jobs requests at `rate`
    jobs/s (about 70% of capacity), then the same requests all at once
    (saturation).  Delivered attempts/ns, its HBM-roofline fraction on the
    2 bytes per attempt, and p50/p99 arrival-to-result latency."""
    from paper_2304_03311_amd import serve, workloads
    stream = workloads.serving_stream(n_jobs, rate, seed=1, **workloads.SERVE_MIX)
    offered = sum(s.n_traj * s.sites * (workloads.N_THERM + s.n_step) for _, s in stream) / stream[-1][0]
    out = {"rate_jobs_per_s": rate, "offered_attempts_per_ns": offered / 1e9, "mix": workloads.SERVE_MIX,
           "launch": {(f"{k[0]}d_L{k[1]}" if isinstance(k, tuple) else f"{k}d"): v
                      for k, v in workloads.SERVE_LAUNCH.items()},
           "hbm_budget_bytes": workloads.SERVE_HBM_BUDGET,
           "jobs_streamed_from_hbm": sum(1 for _, s in stream if s.dim == 3 and s.lx >= 48)}
    for name, realtime in (("poisson", True), ("saturation", False)):
        srv = serve.Server(hbm_budget_bytes=workloads.SERVE_HBM_BUDGET, n_therm=workloads.N_THERM,
                           launch=workloads.SERVE_LAUNCH)
        srv.run(serve.requests_from_stream(stream), realtime=realtime)
        srv.close()
        r = srv.stats.summary()
        r["hbm_frac"] = hbm_frac(r["attempts_per_ns"] * 1e9, 1.0)
        out[name] = r
    return out


def _time_batch(jobs, n_therm, launch, reps=2):
    import torch
    from paper_2304_03311_amd import ee
    best = None
    for _ in range(reps):
        for j in jobs:
            j.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ee.batch_run(jobs, n_therm, cfg=launch)
        res = [j.estimate() for j in jobs]
        dt = time.perf_counter() - t0
        kms = ee.ee_batch_kernel_ms()
        if best is None or dt < best[0]:
            best = (dt, kms, res)
    return best


def _time_per_job(jobs, n_therm):
    import torch
    for j in jobs:
        j.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in jobs:
        j.thermalize(n_therm)
        j.run_protocol()
    res = [j.estimate() for j in jobs]
    return time.perf_counter() - t0, res


def configs_run() -> dict:
    """The other job sets, each through the persistent batched path (the
    tuner's launch shape) and through the per-job launch path."""
    from paper_2304_03311_amd import autotune, ee, workloads
    n_therm = workloads.N_THERM
    sets = {"c1_2d_16x16": [workloads.config1_job()],
            "c3_3d_32cube_bitpacked": [workloads.config3_job()],
            "c4_24_uneven_jobs": workloads.config4_jobs()}
    out = {}
    for name, specs in sets.items():
        launch = autotune.cached(specs, n_therm) or autotune.tune(specs, n_therm)
        jobs = [ee.Job(s) for s in specs]
        att = sum(s.n_traj * s.sites * (n_therm + s.n_step) for s in specs)
        # the best of several runs; ten for the sub-millisecond set, whose
        # wall time varies by tens of microseconds from run to run
        reps = 10 if att < 10 ** 9 else 2
        dt, kms, res = _time_batch(jobs, n_therm, launch, reps=reps)
        dtp, _ = _time_per_job(jobs, n_therm)
        out[name] = {"jobs": len(specs), "attempts": att, "batched_ms": dt * 1e3,
                     "batched_attempts_per_ns": att / (dt * 1e9), "kernel_ms": kms,
                     "hbm_frac": hbm_frac(att, kms * 1e-3),
                     "jobs_per_s": len(specs) / dt, "per_job_path_ms": dtp * 1e3,
                     "per_job_path_attempts_per_ns": att / (dtp * 1e9),
                     "dS_first": res[0].dS, "dS_err_first": res[0].dF_err, "launch": launch}
        for j in jobs:
            j.close()
    return out


def streaming_run(n_traj: int = 32, march: bool = False) -> dict:
    """Throughput of the HBM-streaming path on the largest serving shape
    (3D 96^3, n = 2, N = 100 after 10 thermalisation sweeps): 32
    trajectories on the two-pass kernel (3 B per attempt), or 256 on the
    plane-marching kernel (each plane read and written once per sweep,
    2 B per attempt)."""
    import torch
    from paper_2304_03311_amd import ee, workloads
    spec = ee.JobSpec(dim=3, lt=96, lx=96, ly=96, n=2, beta=workloads.BETA_3D, l=40, n_step=100, n_traj=n_traj,
                      seed=5)
    flags = ee.EE_LAUNCH_MARCH if march else ee.EE_LAUNCH_TWO_PASS
    job = ee.Job(spec)
    job.set_launch({"flags": flags})
    job.thermalize(2)  # warm-up launches
    torch.cuda.synchronize()
    job.reset()
    t0 = time.perf_counter()
    job.thermalize(10)
    job.run_protocol()
    r = job.estimate()
    dt = time.perf_counter() - t0
    job.close()
    bpa = BYTES_PER_ATTEMPT if march else STREAM_BYTES_PER_ATTEMPT
    kernel = "march_kernel + march_fixup_kernel" if march else "stream_sweep_kernel (one launch per colour)"
    return {"workload": f"3D 96^3, n=2, n_t={n_traj}, N=100, N_therm=10, int8 in HBM", "kernel": kernel,
            "attempts_per_ns": r.attempts / (dt * 1e9), "ms": dt * 1e3, "launches": 2 * 110 + 3,
            "algorithmic_bytes_per_attempt": bpa, "hbm_GBps_algorithmic": bpa * r.attempts / dt / 1e9,
            "hbm_frac": hbm_frac(r.attempts, dt, bpa)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=32, help="oracle trajectories timed for cpu_baseline")
    ap.add_argument("--per-job", action="store_true", help="also time the per-job launch path")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving (latency) measurement")
    ap.add_argument("--serve-jobs", type=int, default=2000)
    ap.add_argument("--tune", action="store_true",
                    help="re-tune the headline set's launch shape instead of taking the shipped tuned one")
    ap.add_argument("--no-configs", action="store_true", help="skip the c1/c3/c4 job sets")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving measurement and print its JSON")
    ap.add_argument("--stream-only", action="store_true",
                    help="run only the HBM-streaming measurement (3D 96^3) and print its JSON (profiled runs)")
    ap.add_argument("--launch", default=None,
                    help='launch shape as JSON (ee_launch_cfg fields), e.g. \'{"block_threads": 256, '
                         '"lds_bytes": 54272}\'; replaces the tuned shape')
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the run, copy 256 MiB device-to-device once (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: this build runs on one GPU "
              f"(trajectories shard across GPUs by index; no multi-GPU path is built)", file=sys.stderr)
        return 2

    # the CPU leg first: its worker processes are forked before the GPU is touched
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_sample)

    import numpy as np
    import torch

    from paper_2304_03311_amd import analysis, autotune, ee, serve, workloads

    torch.cuda.set_device(0)
    if args.stream_only:
        print(json.dumps({"streaming_path": streaming_run(),
                          "streaming_march": streaming_run(256, march=True)}), flush=True)
        return 0
    if args.serve_only:
        print(json.dumps({"serving": serving_run(args.serve_jobs)}), flush=True)
        return 0
    specs = workloads.config2_jobs()
    stream = torch.cuda.current_stream()
    n_therm = workloads.N_THERM
    if args.launch is not None:
        launch = json.loads(args.launch)
    else:
        launch = (None if args.tune else autotune.cached(specs, n_therm)) or autotune.tune(specs, n_therm,
                                                                                            stream=stream)
    jobs = [ee.Job(s, stream=stream) for s in specs]
    attempts_per_step = sum(s.n_traj * s.sites * (n_therm + s.n_step) for s in specs)

    def step():
        for j in jobs:
            j.reset()
        ee.batch_run(jobs, n_therm, stream=stream, cfg=launch)
        res = [j.estimate() for j in jobs]
        return res, ee.ee_batch_kernel_ms()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, kms = step()
        kernel_ms.append(kms)
        curve = analysis.assemble([r.dS for r in res], [r.dF_err for r in res], L=64, dim=2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    ms_per_step = dt * 1e3 / args.steps
    value = attempts_per_step * args.steps / (dt * 1e9)
    k_avg_s = float(np.mean(kernel_ms)) * 1e-3
    achieved = BYTES_PER_ATTEMPT * attempts_per_step / k_avg_s / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash():
            traffic = tr.get("bytes_per_launch")
    out = {
        "metric": "spin-flip attempts/ns",
        "value": value,
        "unit": "attempts/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "dtype_note": "int8 spins, uint32 uniforms and thresholds (integer compare), int32 work, fp64 estimator",
        "data": "synthetic (seeded job descriptions; spins and uniforms drawn on device)",
        "config": {"workload": "2D Ising 64x64, n=2, beta_c, l=0..63 (64 jobs), N=1000, "
                               "N_therm=100, n_t=1024, int8, persistent batched path",
                   "jobs": len(specs), "trajectories": sum(s.n_traj for s in specs),
                   "attempts_per_step": attempts_per_step, "parallelism": "1 GPU"},
        "jobs_per_s": len(specs) * args.steps / dt,
        "dS2_err_median": float(np.median([r.dF_err for r in res])),
        # HBM roofline of the dominant kernel on the algorithmic bytes (2 per
        # attempt) of one launch; traffic = the bytes rocprofv3 counted per
        # launch (FETCH_SIZE + WRITE_SIZE, calibrated), null when the kernel
        # changed since they were taken.
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBPS, "traffic": traffic,
                     "kernel": "sweep_kernel (persistent)", "kernel_ms": k_avg_s * 1e3,
                     "bytes_per_attempt": BYTES_PER_ATTEMPT, "attempts_per_launch": attempts_per_step,
                     "attempts_per_ns_in_kernel": attempts_per_step / (k_avg_s * 1e9)},
        "c2_fit_k": curve.get("fit_k"),
        "launch": launch,
    }
    if args.per_job:
        t0 = time.perf_counter()
        for j in jobs:
            j.reset()
            j.thermalize(n_therm)
            j.run_protocol()
        for j in jobs:
            j.estimate()
        torch.cuda.synchronize()
        out["per_job_path_attempts_per_ns"] = attempts_per_step / ((time.perf_counter() - t0) * 1e9)
    if not args.no_configs:
        out["configs"] = configs_run()
    if not args.no_serve:
        out["serving"] = serving_run(args.serve_jobs)
        out["streaming_path"] = streaming_run()
        out["streaming_march"] = streaming_run(256, march=True)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    for j in jobs:
        j.close()
    if args.calib_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = src.numel() * 4
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
