"""Seeded random small jobs against the oracle, bit for bit.

Forty job descriptions drawn from a fixed seed cover the kernels' code
paths together: 2D and 3D, two or three replicas, row half-lengths of
1..24 sites (one to four words per lane, partial words), every protocol
(forward, reverse, the row-subset protocol of App. B in 3D, the
whole-region protocol of Sec. 3), both spin storage formats, zero and
finite beta, and launch shapes on both sides of the parity-major /
lane-map choice.  Each job runs through the persistent batched path
(ten jobs per batch, one launch shape per batch) and through the per-job
path, and its works and final spins must equal the oracle's.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as eo
from paper_2304_03311_amd import ee

pytestmark = pytest.mark.gpu

CFGS = [None,
        dict(block_threads=64, lds_bytes=1024),
        dict(block_threads=64, lds_bytes=4096),
        dict(block_threads=128),
        dict(block_threads=256, lds_bytes=16384),
        dict(block_threads=512),
        dict(block_threads=1024, use_graph=0)]


def _specs(count=40, seed=20240):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        dim = int(rng.choice([2, 3]))
        n = int(rng.choice([2, 3]))
        lt = 2 * int(rng.integers(1, 6))
        lx = 2 * int(rng.integers(1, 25))
        ly = 1 if dim == 2 else 2 * int(rng.integers(1, 4))
        proto = str(rng.choice(["forward", "reverse", "whole", "subsets" if dim == 3 else "forward"]))
        l = int(rng.integers(1, lx + 1)) if proto == "whole" else int(rng.integers(0, lx))  # noqa: E741
        n_step = ly * int(rng.integers(1, 4)) if proto == "subsets" else int(rng.integers(1, 9))
        beta = 0.0 if rng.random() < 0.15 else float(rng.uniform(0.05, 0.6))
        kw = dict(dim=dim, lt=lt, lx=lx, ly=ly, n=n, beta=beta, l=l, n_step=n_step,
                  n_traj=int(rng.integers(1, 6)), seed=int(rng.integers(1, 1 << 30)),
                  reverse=proto == "reverse", subsets=proto == "subsets", whole=proto == "whole",
                  spin_format=int(rng.integers(0, 2)))
        out.append((ee.JobSpec(**kw), int(rng.integers(0, 4))))
    return out


SPECS = _specs()


def _oracle(s: ee.JobSpec, n_therm: int):
    job = eo.Job(s.dim, s.lt, s.lx, s.ly, s.n, s.beta, s.l, s.n_step, s.n_traj, s.seed, s.reverse, s.subsets,
                 s.whole)
    return eo.run(job, n_therm, want_spins=True)


@pytest.mark.parametrize("b", range(4))
def test_random_jobs_batched(b):
    group = SPECS[10 * b:10 * (b + 1)]
    cfg = CFGS[(3 * b + 1) % len(CFGS)]
    print(f"[gpu] random batch {b}: launch {cfg}", flush=True)
    for n_therm in sorted({t for _, t in group}):
        specs = [s for s, t in group if t == n_therm]
        jobs = [ee.Job(s) for s in specs]
        ee.batch_run(jobs, n_therm, cfg=cfg)
        for s, j in zip(specs, jobs):
            I_or, sp_or = _oracle(s, n_therm)
            assert np.array_equal(j.work(), I_or), s
            assert np.array_equal(j.spins(), sp_or), s
            j.close()


@pytest.mark.parametrize("i", range(len(SPECS)))
def test_random_jobs_per_job(i):
    s, n_therm = SPECS[i]
    cfg = CFGS[i % len(CFGS)]
    print(f"[gpu] random job {i}: {s} n_therm={n_therm} launch {cfg}", flush=True)
    j = ee.Job(s)
    if cfg is not None:
        j.set_launch(cfg)
    j.thermalize(n_therm)
    j.run_protocol()
    I_or, sp_or = _oracle(s, n_therm)
    assert np.array_equal(j.work(), I_or), s
    assert np.array_equal(j.spins(), sp_or), s
    j.close()
