"""Seeded synthetic job sets of the benchmark configurations.

This module holds only problem statements (lattice shapes, couplings,
protocol lengths, seeds, arrival times); none of the estimator's
arithmetic.  The GPU path and the CPU oracle receive the same job lists.

Configurations (the paper's own runs use L_tau = 8L in 2D and 4L in 3D,
Sec. 4 and Sec. 5; the benchmark shapes below read L_tau = L literally):
  1. 2D 16x16, n = 2, beta_c, l = 4 -> 5, N = 256, 100 thermalisation
     sweeps, 64 trajectories, int8, seed 1.
  2. 2D 64x64, n = 2, beta_c, l = 0..63 (64 jobs, S_2(1..64)), N = 1000,
     1024 trajectories per job, int8, seeds 1 + l.
  3. 3D 32^3, n = 2, beta = 0.2216546, l = 8, N = 2000, 512 trajectories,
     bit-packed, seed 1.
  4. 24 uneven jobs: 2D L in {24,32,48,64,96} and 3D L in {16,24,32}, each
     with N in {500,1000,2000}; L_tau = L, beta = beta_c of the dimension,
     l uniform in [0, L) from a PCG64 stream (seed 1), 256 trajectories,
     2D int8 and 3D bit-packed, seeds 1 + index.
  5. serving stream: see ``serving_stream``.
"""
from __future__ import annotations

import math

import numpy as np

from .ee import EE_SPINS_BITPACKED, EE_SPINS_INT8, JobSpec

BETA_C_2D = 0.5 * math.log(1.0 + math.sqrt(2.0))  # Sec. 4
BETA_3D = 0.2216546                                 # Sec. 5 (beta_c = 0.221654626(5))
N_THERM = 100

# launch shape of the headline set (2D 64x64, 64 jobs x 1024 trajectories)
# when no tuned shape is at hand: one 64-thread workgroup (one wave) per
# trajectory, the tuner's choice on an MI355X (each wave owns a whole
# trajectory, so its barriers wait for no other wave)
BENCH_LAUNCH = {"block_threads": 64, "lds_bytes": 8192, "grid_blocks": 0, "use_graph": 1, "flags": 0}

# serving benchmark: size mix of the Poisson stream at 200 jobs/s (n_t up to
# 4096; the mix sets the offered load, about 70% of the served path's
# measured capacity), the HBM admission budget (288 GB of HBM3E minus a
# reserve for the rest of the process) and the launch shapes of the server's
# chunk launches, by dimension and, for two 3D sizes, by lattice extent:
# 2D lattices in one-wave workgroups of up to 4 KiB (the tuner's shapes for
# the 2D sets), 3D in 512-thread workgroups (the tuner's shape for the
# 3D-heavy 24-job set; one 32^3 trajectory each), except 24^3, one
# trajectory per three-wave workgroup (96 row slots per replica, a multiple
# of L_y: the parity-major row order, three steps per half-sweep, where 256
# or 512 lanes take the lane-map order with a partly idle last pass), and
# 16^3, one trajectory per one-wave workgroup (measured on an MI355X over
# 8 jobs x 512 trajectories: 24^3 2353 against 2243 attempts/ns at 256
# threads, 16^3 2579 against 2393 at 512 threads)
SERVE_MIX = {"max_l3": 96, "n_traj_choices": (64, 256, 1024, 4096), "n_traj_weights": (0.48, 0.32, 0.155, 0.045),
             "n_step_choices": (500, 1000), "large_n_traj": (8, 16)}
SERVE_HBM_BUDGET = 256 * 1024 ** 3
SERVE_LAUNCH = {2: {"block_threads": 64, "lds_bytes": 4096, "grid_blocks": 0, "use_graph": 1, "flags": 0},
                3: {"block_threads": 512, "lds_bytes": 54272, "grid_blocks": 0, "use_graph": 1, "flags": 0},
                (3, 24): {"block_threads": 192, "lds_bytes": 28672, "grid_blocks": 0, "use_graph": 1, "flags": 0},
                (3, 16): {"block_threads": 64, "lds_bytes": 8192, "grid_blocks": 0, "use_graph": 1, "flags": 0}}


def config1_job() -> JobSpec:
    return JobSpec(dim=2, lt=16, lx=16, ly=1, n=2, beta=BETA_C_2D, l=4, n_step=256, n_traj=64, seed=1)


def config2_jobs(L: int = 64, n_step: int = 1000, n_traj: int = 1024, lt: int | None = None) -> list[JobSpec]:
    lt = L if lt is None else lt
    return [JobSpec(dim=2, lt=lt, lx=L, ly=1, n=2, beta=BETA_C_2D, l=l, n_step=n_step, n_traj=n_traj,
                    seed=1 + l) for l in range(L)]


def config3_job(spin_format: int = EE_SPINS_BITPACKED) -> JobSpec:
    return JobSpec(dim=3, lt=32, lx=32, ly=32, n=2, beta=BETA_3D, l=8, n_step=2000, n_traj=512, seed=1,
                   spin_format=spin_format)


def config4_jobs(n_traj: int = 256) -> list[JobSpec]:
    rng = np.random.Generator(np.random.PCG64(1))
    shapes = [(2, L) for L in (24, 32, 48, 64, 96)] + [(3, L) for L in (16, 24, 32)]
    out = []
    idx = 0
    for dim, L in shapes:
        for n_step in (500, 1000, 2000):
            l = int(rng.integers(0, L))
            out.append(JobSpec(dim=dim, lt=L, lx=L, ly=L if dim == 3 else 1, n=2,
                               beta=BETA_C_2D if dim == 2 else BETA_3D, l=l, n_step=n_step, n_traj=n_traj,
                               seed=1 + idx, spin_format=EE_SPINS_INT8 if dim == 2 else EE_SPINS_BITPACKED))
            idx += 1
    return out


def serving_stream(n_jobs: int, rate_per_s: float, seed: int = 1, max_l3: int = 96,
                   n_traj_choices=(64, 128, 256), n_step_choices=(500, 1000),
                   l2_choices=(24, 32, 48, 64, 96), l3_weights=None, large_n_traj=(16, 32),
                   n_traj_weights=None):
    """Poisson arrivals (mean rate_per_s) of jobs of random dimension, size,
    beta, l, N and n_t.  Returns [(arrival_time_s, JobSpec)].

    2D: L uniform in l2_choices.  3D: L drawn with l3_weights (default: 16,
    24, 32 at 30 % each and 48, 64, 96 at 5, 3 and 2 %), restricted to
    L <= max_l3.  beta uniform in {0.21, 0.2216546, 0.23}.  n_t from
    n_traj_choices, except 3D lattices of L >= 48 (streamed from HBM), which
    take n_t from large_n_traj.  n_t is uniform over n_traj_choices, or drawn
    with n_traj_weights.  2D and on-chip 3D jobs store bit-packed 3D / int8
    2D spins; streamed jobs int8."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if l3_weights is None:
        l3_weights = {16: 0.30, 24: 0.30, 32: 0.30, 48: 0.05, 64: 0.03, 96: 0.02}
    l3 = [L for L in l3_weights if L <= max_l3]
    w3 = np.array([l3_weights[L] for L in l3], dtype=float)
    w3 /= w3.sum()
    t = 0.0
    out = []
    for i in range(n_jobs):
        t += float(rng.exponential(1.0 / rate_per_s))
        dim = int(rng.integers(2, 4))
        if dim == 2:
            L = int(rng.choice(l2_choices))
        else:
            L = int(rng.choice(l3, p=w3))
        beta = float(rng.choice([0.21, BETA_3D, 0.23]))
        l = int(rng.integers(0, L))
        n_step = int(rng.choice(n_step_choices))
        streamed = dim == 3 and L >= 48
        if streamed:
            n_traj = int(rng.choice(large_n_traj))
        elif n_traj_weights is not None:
            n_traj = int(rng.choice(n_traj_choices, p=np.asarray(n_traj_weights, dtype=float)))
        else:
            n_traj = int(rng.choice(n_traj_choices))
        fmt = EE_SPINS_INT8 if (dim == 2 or streamed) else EE_SPINS_BITPACKED
        out.append((t, JobSpec(dim=dim, lt=L, lx=L, ly=L if dim == 3 else 1, n=2, beta=beta, l=l,
                               n_step=n_step, n_traj=n_traj, seed=1000 + i, spin_format=fmt)))
    return out
