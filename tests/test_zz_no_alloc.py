"""The allocation-free batch entry point (ee_batch_run_noalloc) against
ee_batch_run_cfg, through the C ABI: two calls in a row, the second with a
smaller batch, each bit-identical to the allocating path (works, spins and
every field of the estimate); and the size limit of its fixed scratch."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2304_03311_amd import ee

pytestmark = pytest.mark.gpu

BC2 = 0.44068679350977147
BC3 = 0.2216546

FIRST = [
    ee.JobSpec(dim=2, lt=16, lx=64, ly=1, n=2, beta=BC2, l=21, n_step=12, n_traj=40, seed=81),
    ee.JobSpec(dim=2, lt=8, lx=24, ly=1, n=3, beta=0.5, l=7, n_step=9, n_traj=33, seed=82, reverse=True),
    ee.JobSpec(dim=3, lt=8, lx=8, ly=8, n=2, beta=BC3, l=3, n_step=10, n_traj=17, seed=83, spin_format=1),
    ee.JobSpec(dim=3, lt=4, lx=16, ly=4, n=2, beta=BC3, l=5, n_step=8, n_traj=9, seed=84, subsets=True),
    ee.JobSpec(dim=2, lt=8, lx=12, ly=1, n=2, beta=BC2, l=3, n_step=10, n_traj=21, seed=85, whole=True),
]
SECOND = [
    ee.JobSpec(dim=2, lt=8, lx=16, ly=1, n=2, beta=BC2, l=4, n_step=7, n_traj=5, seed=86),
    ee.JobSpec(dim=3, lt=4, lx=6, ly=2, n=2, beta=0.3, l=5, n_step=5, n_traj=3, seed=87),
]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    ee.lib()


def _same(a: ee.Job, b: ee.Job):
    assert np.array_equal(a.work(), b.work())
    assert np.array_equal(a.spins(), b.spins())
    ra, rb = a.estimate(), b.estimate()
    for k in ("dF", "dS", "w_mean", "w_var", "ess", "i_min", "i_max", "attempts", "n_traj"):
        assert getattr(ra, k) == getattr(rb, k), k
    assert ra.dF_err == rb.dF_err or (np.isnan(ra.dF_err) and np.isnan(rb.dF_err))


@pytest.mark.parametrize("cfg", [None, dict(block_threads=64, lds_bytes=4096), dict(block_threads=256)])
def test_noalloc_batch_equals_batch_run_twice(cfg):
    for label, specs in (("first", FIRST), ("second, smaller", SECOND)):
        say(f"[gpu] no-alloc batch, {label}: {len(specs)} jobs, cfg {cfg}")
        ref = [ee.Job(s) for s in specs]
        ee.batch_run(ref, 4, cfg=cfg)
        na = [ee.Job(s) for s in specs]
        ee.batch_run_noalloc(na, 4, cfg=cfg)
        for a, b in zip(ref, na):
            _same(a, b)
        for j in ref + na:
            j.close()


def test_noalloc_rejects_tables_beyond_its_scratch():
    # one trajectory per work unit (LDS budget = one trajectory): three jobs
    # of 65535 trajectories need 3 x 65535 x 16 bytes of unit table > 2 MiB
    s = ee.JobSpec(dim=2, lt=2, lx=2, ly=1, n=2, beta=0.3, l=0, n_step=1, n_traj=65535, seed=1)
    jobs = [ee.Job(s) for _ in range(3)]
    with pytest.raises(ee.EEError) as e:
        ee.batch_run_noalloc(jobs, 0, cfg=dict(block_threads=64, lds_bytes=16))
    assert e.value.status == ee.EE_EINVAL
    assert "scratch" in str(e.value)
    # the jobs were not touched: the allocating path still runs them
    ee.batch_run(jobs[:1], 0, cfg=dict(block_threads=64, lds_bytes=16))
    assert jobs[0].work().shape == (65535,)
    for j in jobs:
        j.close()
