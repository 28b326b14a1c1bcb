"""Autotuner of the persistent sweep kernel's launch shape.

The shape is the workgroup size (64..1024 threads) and the LDS budget per
workgroup.  Together they fix how many trajectories share a workgroup (LDS
slots), how many rows each lane walks between barriers, and how many
workgroups stay resident per CU.  Every shape gives bit-identical results,
because the random numbers are indexed by site, sweep and trajectory and
never by thread.  So the tuner only measures time.

Trials run the same job shapes with a shortened protocol.  The kernel time
is measured with HIP events (ee_batch_kernel_ms).  The best shape is cached
in a JSON file keyed by a signature of the job shapes.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import os

from . import ee

# The shipped cache holds the shapes tuned on an MI355X for the benchmark
# job sets; EE_TUNE_CACHE points the tuner at another file.
CACHE = os.environ.get("EE_TUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_launch.json"))
MAX_LDS = 160 * 1024 - 256


def _cfg(block: int, lds: int) -> dict:
    return {"block_threads": block, "lds_bytes": lds, "grid_blocks": 0, "use_graph": 1, "flags": 0}


# block size x LDS budget per workgroup.  The small shapes (a wave or two,
# an LDS budget of a few trajectories) spread latency-bound sets of small
# lattices over more CUs.
CANDIDATES = [
    _cfg(b, lds)
    for blocks, ldss in (((256, 512, 1024), (40 * 1024, 53 * 1024, 80 * 1024, MAX_LDS)),
                         ((64, 128), (1024, 2048, 4096)))
    for b in blocks
    for lds in ldss
]


def traj_bytes(s: ee.JobSpec) -> int:
    """LDS bytes of one trajectory (int8 colour planes, whole 32-bit words per row)."""
    return 2 * s.n * s.lt * s.ly * ((s.lx // 2 + 3) // 4) * 4


def candidates_for(specs: list[ee.JobSpec]) -> list[dict]:
    """The static shapes plus one to four trajectories of the set's largest
    lattice per workgroup of one or two waves (each wave then owns whole
    trajectories, so its barriers wait for no other wave)."""
    tb = max(traj_bytes(s) for s in specs)
    extra = [_cfg(b, k * tb) for b in (64, 128) for k in (1, 2, 3, 4) if k * tb <= MAX_LDS]
    out = []
    for c in CANDIDATES + extra:
        if c not in out:
            out.append(c)
    return out


def signature(specs: list[ee.JobSpec], n_therm: int) -> str:
    key = json.dumps([[s.dim, s.lt, s.lx, s.ly, s.n, s.n_step, s.n_traj, s.spin_format] for s in specs]
                     + [n_therm])
    return hashlib.sha256(key.encode()).hexdigest()[:16]


def _load() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def cached(specs, n_therm):
    return _load().get(signature(specs, n_therm))


def _wall_ms(jobs, n_therm: int, cfg: dict, repeats: int, stream=None) -> float:
    """Shortest wall time of the whole batch (launch, sweeps, estimates read
    back) over `repeats` runs, in ms."""
    import time

    import torch
    best = float("inf")
    for _ in range(repeats):
        for j in jobs:
            j.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ee.batch_run(jobs, n_therm, stream=stream, cfg=cfg)
        for j in jobs:
            j.estimate()
        best = min(best, (time.perf_counter() - t0) * 1e3)
    return best


def tune(specs: list[ee.JobSpec], n_therm: int, trial_steps: int = 200, trial_therm: int = 20,
         candidates=None, repeats: int = 3, stream=None, save: bool = True, verbose: bool = False) -> dict:
    """Pick the fastest launch shape for this job set; returns the ee_launch_cfg dict.

    The shape is chosen on the sweep kernel's time (HIP events).  Then,
    for that shape, whether the batch replays as a HIP graph is chosen on
    the wall time of the whole batch: a graph replay costs the host a few
    tens of microseconds more than direct launches, which shows on small,
    latency-bound sets, so the graph is dropped only where doing so is more
    than 2% faster."""
    import torch
    candidates = candidates_for(specs) if candidates is None else candidates
    # same lattice shapes and trajectory counts, shorter protocol
    trial_specs = [dataclasses.replace(s, n_step=min(s.n_step, trial_steps)) for s in specs]
    jobs = [ee.Job(s, stream=stream) for s in trial_specs]
    results = []
    try:
        for cfg in candidates:
            times = []
            for _ in range(repeats):
                for j in jobs:
                    j.reset()
                ee.batch_run(jobs, trial_therm, stream=stream, cfg=cfg)
                times.append(ee.ee_batch_kernel_ms())
            t = min(times)
            results.append((t, cfg))
            if verbose:
                print(f"autotune {cfg} -> {t:.3f} ms", flush=True)
        results.sort(key=lambda x: x[0])
        best = dict(results[0][1])
        best["trial_ms"] = results[0][0]
        walls = {g: _wall_ms(jobs, trial_therm, dict(best, use_graph=g), 4 * repeats, stream) for g in (1, 0)}
        best["use_graph"] = 0 if walls[0] < 0.98 * walls[1] else 1
        best["trial_wall_ms"] = walls[best["use_graph"]]
        if verbose:
            print(f"autotune wall time with / without a graph: {walls[1]:.3f} / {walls[0]:.3f} ms", flush=True)
        torch.cuda.synchronize()
    finally:
        for j in jobs:
            j.close()
    if save:
        db = _load()
        db[signature(specs, n_therm)] = best
        with open(CACHE, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
    return best
