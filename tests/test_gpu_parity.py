"""GPU parity of the HIP path with the CPU oracle, through the C ABI.

Bar: spins and integer works bit-exact; Delta F within
1e-12 max(|Delta F|, 1e-3), the mean and variance of W equal, the jackknife
error and the ESS within 1e-12 relative (see check_estimate).
"""
from __future__ import annotations

import dataclasses
import math
import sys

import numpy as np
import pytest

from oracle import oracle as eo
from paper_2304_03311_amd import ee, workloads

BC2 = 0.5 * math.log(1.0 + math.sqrt(2.0))
BC3 = 0.2216546

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    ee.lib()


def say(*a):
    print(*a, file=sys.stderr, flush=True)


# Largest |dF_gpu - dF_oracle| / max(|dF_oracle|, 1e-3) seen in this session,
# printed by the last test of the module.
_DF_WORST = [0.0, ""]


def oracle_job(s: ee.JobSpec) -> eo.Job:
    return eo.Job(s.dim, s.lt, s.lx, s.ly, s.n, s.beta, s.l, s.n_step, s.n_traj, s.seed, s.reverse, s.subsets,
                  s.whole)


def check_estimate(res: ee.ee_result, I: np.ndarray, s: ee.JobSpec, label: str = ""):
    """The GPU estimate against the oracle's on the same integer works.

    The kernel forms every FP64 output by the oracle's operations in the
    oracle's order, with correctly rounded exp and log, so the two differ
    only where the host's libm rounds exp or log the other way (about one
    evaluation in a thousand, each by one ulp).  Delta F: within
    1e-12 max(|Delta F|, 1e-3) (1e-12 relative; the floor keeps the bound
    meaningful where Delta F crosses zero).  The mean and variance of W are
    sums of correctly rounded products in the same order: equal.  The
    jackknife error and the ESS: 1e-12 relative."""
    est = eo.estimate(I, s.beta, s.S, s.n)
    floor = max(abs(est.dF), 1e-3)
    rel = abs(res.dF - est.dF) / floor
    say(f"[gpu]   {label} dF gpu {res.dF!r} oracle {est.dF!r} |diff|/max(|dF|,1e-3) = {rel:.3g}")
    if rel > _DF_WORST[0]:
        _DF_WORST[:] = [rel, label]
    assert abs(res.dF - est.dF) <= 1e-12 * floor, (res.dF, est.dF)
    assert abs(res.dS - est.dS) <= 1e-12 * max(abs(est.dS), 1e-3)
    assert res.i_min == est.i_min and res.i_max == est.i_max
    if s.n_traj >= 2:
        assert res.dF_err == pytest.approx(est.dF_err, rel=1e-12, abs=1e-300)
    else:
        assert math.isnan(res.dF_err) and math.isnan(est.dF_err)
    assert res.w_mean == est.w_mean
    assert res.w_var == est.w_var
    assert res.ess == pytest.approx(est.ess, rel=1e-12)


CASES = [
    # name, spec, n_therm
    ("c1_16x16_l4", dict(dim=2, lt=16, lx=16, ly=1, n=2, beta=BC2, l=4, n_step=256, n_traj=64, seed=1), 100),
    ("2d_ragged_lx6", dict(dim=2, lt=8, lx=6, ly=1, n=2, beta=0.5, l=2, n_step=20, n_traj=6, seed=3), 10),
    ("2d_lx10_l9_last_column", dict(dim=2, lt=6, lx=10, ly=1, n=2, beta=0.4, l=9, n_step=15, n_traj=5, seed=5), 7),
    ("2d_lx2_lt2_minimal", dict(dim=2, lt=2, lx=2, ly=1, n=2, beta=0.7, l=1, n_step=9, n_traj=7, seed=9), 5),
    ("2d_n3_l0", dict(dim=2, lt=8, lx=12, ly=1, n=3, beta=0.45, l=0, n_step=12, n_traj=5, seed=11), 6),
    ("2d_n4_l7", dict(dim=2, lt=4, lx=14, ly=1, n=4, beta=0.6, l=7, n_step=10, n_traj=3, seed=12), 4),
    ("2d_reverse", dict(dim=2, lt=12, lx=16, ly=1, n=2, beta=BC2, l=5, n_step=30, n_traj=9, seed=4, reverse=True), 12),
    ("2d_bitpacked_lx70", dict(dim=2, lt=10, lx=70, ly=1, n=2, beta=0.42, l=33, n_step=11, n_traj=4, seed=6,
                               spin_format=1), 5),
    ("2d_beta0", dict(dim=2, lt=8, lx=8, ly=1, n=2, beta=0.0, l=3, n_step=5, n_traj=4, seed=8), 3),
    ("2d_one_traj", dict(dim=2, lt=8, lx=8, ly=1, n=2, beta=BC2, l=3, n_step=7, n_traj=1, seed=8), 3),
    ("2d_seed_hi_bits", dict(dim=2, lt=8, lx=16, ly=1, n=2, beta=BC2, l=8, n_step=7, n_traj=3,
                             seed=(0xDEADBEEF << 32) | 0x12345678), 3),
    ("3d_8cube", dict(dim=3, lt=8, lx=8, ly=8, n=2, beta=BC3, l=3, n_step=20, n_traj=6, seed=2), 8),
    ("3d_ragged_lx6_ly2", dict(dim=3, lt=4, lx=6, ly=2, n=2, beta=0.3, l=5, n_step=9, n_traj=5, seed=13), 4),
    ("3d_bitpacked_reverse", dict(dim=3, lt=6, lx=10, ly=4, n=2, beta=0.25, l=4, n_step=8, n_traj=4, seed=14,
                                  spin_format=1, reverse=True), 5),
    ("3d_n3", dict(dim=3, lt=4, lx=8, ly=4, n=3, beta=BC3, l=0, n_step=6, n_traj=3, seed=15), 3),
    ("3d_protocol2", dict(dim=3, lt=6, lx=8, ly=4, n=2, beta=BC3, l=3, n_step=12, n_traj=5, seed=16, subsets=True), 4),
    ("3d_protocol2_reverse", dict(dim=3, lt=4, lx=16, ly=6, n=2, beta=0.23, l=9, n_step=18, n_traj=4, seed=17,
                                  subsets=True, reverse=True), 3),
    ("3d_protocol2_bitpacked", dict(dim=3, lt=4, lx=6, ly=2, n=3, beta=0.3, l=5, n_step=4, n_traj=3, seed=18,
                                    subsets=True, spin_format=1), 3),
    ("2d_protocol2_is_protocol1", dict(dim=2, lt=8, lx=16, ly=1, n=2, beta=BC2, l=4, n_step=9, n_traj=4, seed=19,
                                       subsets=True), 3),
    # whole-region protocol (Sec. 3): every cut link of x < l ramped at once
    ("2d_whole_l3", dict(dim=2, lt=8, lx=12, ly=1, n=2, beta=BC2, l=3, n_step=10, n_traj=5, seed=51, whole=True), 4),
    ("2d_whole_every_column_n3_reverse", dict(dim=2, lt=6, lx=8, ly=1, n=3, beta=0.5, l=8, n_step=6, n_traj=4,
                                              seed=52, whole=True, reverse=True), 3),
    ("2d_whole_ragged_lx70", dict(dim=2, lt=4, lx=70, ly=1, n=2, beta=0.42, l=41, n_step=4, n_traj=3, seed=54,
                                  whole=True), 3),
    ("3d_whole_bitpacked", dict(dim=3, lt=4, lx=10, ly=4, n=2, beta=BC3, l=7, n_step=5, n_traj=3, seed=53,
                                whole=True, spin_format=1), 3),
]


@pytest.mark.parametrize("name,kw,n_therm", CASES, ids=[c[0] for c in CASES])
def test_per_job_path_matches_oracle(name, kw, n_therm):
    s = ee.JobSpec(**kw)
    say(f"[gpu] per-job {name}: {kw} n_therm={n_therm}")
    job = ee.Job(s)
    # thermalisation split over two calls must equal one call
    job.thermalize(n_therm // 2)
    job.thermalize(n_therm - n_therm // 2)
    job.run_protocol()
    res = job.estimate()
    I_gpu = job.work()
    sp_gpu = job.spins()
    I_or, sp_or = eo.run(oracle_job(s), n_therm, want_spins=True)
    assert np.array_equal(I_gpu, I_or)
    assert np.array_equal(sp_gpu, sp_or)
    check_estimate(res, I_or, s, name)
    assert res.attempts == s.n_traj * s.sites * (n_therm + s.n_step)
    job.close()


@pytest.mark.parametrize("name,kw,n_therm", CASES[:4] + CASES[11:13], ids=[c[0] for c in CASES[:4] + CASES[11:13]])
def test_initial_and_thermalised_spins_match_oracle(name, kw, n_therm):
    s = ee.JobSpec(**kw)
    say(f"[gpu] init/therm spins {name}")
    job = ee.Job(s)
    job.thermalize(0)
    _, sp0 = eo.run(oracle_job(s), 0, n_step_run=0, want_spins=True)
    assert np.array_equal(job.spins(), sp0)
    job.thermalize(3)
    _, sp3 = eo.run(oracle_job(s), 3, n_step_run=0, want_spins=True)
    assert np.array_equal(job.spins(), sp3)
    job.close()


def test_batch_path_matches_per_job_and_oracle():
    specs = [ee.JobSpec(**kw) for _, kw, _ in CASES if kw["dim"] == 2][:8]
    specs += [ee.JobSpec(**kw) for name, kw, _ in CASES if name.startswith("3d_protocol2")]
    n_therm = 6
    say(f"[gpu] batch of {len(specs)} uneven 2D jobs")
    jobs = [ee.Job(s) for s in specs]
    ee.batch_run(jobs, n_therm)
    for s, job in zip(specs, jobs):
        I_or, sp_or = eo.run(oracle_job(s), n_therm, want_spins=True)
        assert np.array_equal(job.work(), I_or), s
        assert np.array_equal(job.spins(), sp_or), s
        check_estimate(job.estimate(), I_or, s, f"batch l={s.l}")
    # replay of the recorded graph: identical results
    first = [j.work() for j in jobs]
    for j in jobs:
        j.reset()
    ee.batch_run(jobs, n_therm)
    for a, j in zip(first, jobs):
        assert np.array_equal(a, j.work())
    assert ee.ee_batch_kernel_ms() > 0.0
    for j in jobs:
        j.close()


@pytest.mark.parametrize("cfg", [dict(block_threads=64), dict(block_threads=256, lds_bytes=32768),
                                 dict(block_threads=512, grid_blocks=3), dict(block_threads=1024, use_graph=0)])
def test_launch_shapes_give_identical_bits(cfg):
    specs = [ee.JobSpec(dim=3, lt=8, lx=8, ly=8, n=2, beta=BC3, l=2, n_step=10, n_traj=7, seed=21),
             ee.JobSpec(dim=3, lt=4, lx=12, ly=6, n=2, beta=0.23, l=11, n_step=4, n_traj=5, seed=22,
                        spin_format=1)]
    say(f"[gpu] launch shape {cfg}")
    jobs = [ee.Job(s) for s in specs]
    ee.batch_run(jobs, 5, cfg=cfg)
    for s, j in zip(specs, jobs):
        I_or, sp_or = eo.run(oracle_job(s), 5, want_spins=True)
        assert np.array_equal(j.work(), I_or)
        assert np.array_equal(j.spins(), sp_or)
    # per-job path with the same shape
    for s in specs:
        j = ee.Job(s)
        j.set_launch(cfg)
        j.thermalize(5)
        j.run_protocol()
        I_or, _ = eo.run(oracle_job(s), 5)
        assert np.array_equal(j.work(), I_or)
        j.close()


WIDE_SPECS = [
    # lx/2 a multiple of 16: a lane takes four words (16 sites) of a row
    dict(dim=2, lt=16, lx=32, ly=1, n=2, beta=BC2, l=13, n_step=8, n_traj=6, seed=31),
    dict(dim=2, lt=8, lx=64, ly=1, n=3, beta=BC2, l=37, n_step=6, n_traj=5, seed=32, reverse=True),
    dict(dim=2, lt=4, lx=96, ly=1, n=2, beta=0.3, l=70, n_step=5, n_traj=3, seed=33, spin_format=1),
    dict(dim=3, lt=8, lx=32, ly=4, n=2, beta=BC3, l=22, n_step=8, n_traj=4, seed=34, subsets=True),
    dict(dim=2, lt=6, lx=32, ly=1, n=2, beta=BC2, l=31, n_step=4, n_traj=3, seed=35),
    # rows of three words: one lane takes a whole row (12 sites)
    dict(dim=2, lt=8, lx=24, ly=1, n=2, beta=BC2, l=17, n_step=6, n_traj=5, seed=36),
    dict(dim=3, lt=4, lx=24, ly=4, n=3, beta=BC3, l=10, n_step=8, n_traj=3, seed=37, subsets=True),
    dict(dim=3, lt=6, lx=24, ly=2, n=2, beta=0.25, l=23, n_step=4, n_traj=4, seed=38, spin_format=1, reverse=True),
    dict(dim=2, lt=8, lx=64, ly=1, n=2, beta=BC2, l=45, n_step=5, n_traj=3, seed=39, whole=True),
    # 3D with ly = 6: the row slots of a replica are not a multiple of ly, so
    # the rows go in the order of the lane map instead of parity-major
    dict(dim=3, lt=4, lx=16, ly=6, n=2, beta=BC3, l=5, n_step=6, n_traj=4, seed=40),
    dict(dim=3, lt=4, lx=16, ly=6, n=3, beta=0.0, l=9, n_step=4, n_traj=3, seed=44, whole=True),
]


@pytest.mark.parametrize("cfg", [dict(block_threads=256),
                                 dict(block_threads=128, lds_bytes=32768),
                                 dict(block_threads=1024, use_graph=0),
                                 dict(block_threads=512),
                                 dict(block_threads=64, lds_bytes=1024),
                                 dict()])
def test_multiword_lanes_give_identical_bits(cfg):
    specs = [ee.JobSpec(**kw) for kw in WIDE_SPECS]
    say(f"[gpu] multi-word lanes, launch shape {cfg}")
    jobs = [ee.Job(s) for s in specs]
    ee.batch_run(jobs, 4, cfg=cfg)
    for s, j in zip(specs, jobs):
        I_or, sp_or = eo.run(oracle_job(s), 4, want_spins=True)
        assert np.array_equal(j.work(), I_or), s
        assert np.array_equal(j.spins(), sp_or), s
        j.close()
    for s in specs:
        j = ee.Job(s)
        j.set_launch(cfg)
        j.thermalize(4)
        j.run_protocol()
        I_or, sp_or = eo.run(oracle_job(s), 4, want_spins=True)
        assert np.array_equal(j.work(), I_or), s
        assert np.array_equal(j.spins(), sp_or), s
        j.close()


# The same jobs under launch shapes that take either row order of the
# on-chip kernel: with T lanes per trajectory, S = T / (G / W) row slots and
# B = S / n per replica, the parity-major order runs when B < R (and, in 3D,
# ly divides B), the lane-map order otherwise.  The batch path packs as many
# trajectories per workgroup as the LDS budget allows (ties to the larger
# count); the per-job path keeps one per workgroup for jobs this small.
ROW_ORDER_CASES = [
    # 2D 16x64 (2 KiB per trajectory): G = 8, W = 4, R = 16.  One trajectory
    # per 64 lanes: B = 16 = R (lane map); two: B = 8 (parity-major).
    ("2d_lanemap", dict(dim=2, lt=16, lx=64, ly=1, n=2, beta=BC2, l=21, n_step=6, n_traj=4, seed=71),
     dict(block_threads=64, lds_bytes=2048)),
    ("2d_paritymajor", dict(dim=2, lt=16, lx=64, ly=1, n=2, beta=BC2, l=21, n_step=6, n_traj=4, seed=71),
     dict(block_threads=64, lds_bytes=4096)),
    # 3D 4x32x4 (1 KiB per trajectory): G = 4, W = 4, R = 16.  T = 64: B = 32
    # (lane map); four trajectories per 64 lanes: B = 8, a multiple of ly
    # (parity-major).
    ("3d_lanemap", dict(dim=3, lt=4, lx=32, ly=4, n=2, beta=BC3, l=9, n_step=6, n_traj=4, seed=72),
     dict(block_threads=64, lds_bytes=1024)),
    ("3d_paritymajor", dict(dim=3, lt=4, lx=32, ly=4, n=2, beta=BC3, l=9, n_step=6, n_traj=4, seed=72),
     dict(block_threads=64, lds_bytes=4096)),
    # the serving shapes of the 3D lattices.  24^3 (27 KiB, G = W = 3,
    # R = 576) in three-wave workgroups: B = 96, a multiple of ly = 24
    # (parity-major, three steps of both classes per half-sweep).
    ("3d_24cube_192", dict(dim=3, lt=24, lx=24, ly=24, n=2, beta=BC3, l=11, n_step=4, n_traj=3, seed=73,
                           spin_format=1), dict(block_threads=192, lds_bytes=28672)),
    # 16^3 (8 KiB, G = W = 2, R = 256) in one-wave workgroups: B = 32
    # (parity-major, eight steps).
    ("3d_16cube_64", dict(dim=3, lt=16, lx=16, ly=16, n=2, beta=BC3, l=5, n_step=5, n_traj=3, seed=74,
                          spin_format=1, reverse=True), dict(block_threads=64, lds_bytes=8192)),
]


@pytest.mark.parametrize("name,kw,cfg", ROW_ORDER_CASES, ids=[c[0] for c in ROW_ORDER_CASES])
def test_both_row_orders_match_oracle(name, kw, cfg):
    s = ee.JobSpec(**kw)
    say(f"[gpu] row order {name}: {cfg}")
    I_or, sp_or = eo.run(oracle_job(s), 3, want_spins=True)
    j = ee.Job(s)
    j.set_launch(cfg)
    j.thermalize(3)
    j.run_protocol()
    assert np.array_equal(j.work(), I_or)
    assert np.array_equal(j.spins(), sp_or)
    j.close()
    jobs = [ee.Job(s)]
    ee.batch_run(jobs, 3, cfg=cfg)
    assert np.array_equal(jobs[0].work(), I_or)
    assert np.array_equal(jobs[0].spins(), sp_or)
    jobs[0].close()


# The lattice, order and beta at which a since-removed 64-VGPR build of the
# sweep kernel gave wrong protocol results: 8x8, n = 2, one word per row
# (lane-map order), beta = 0 (every attempt flips, so a skipped or repeated
# site shows in the spins and the work).  The shipped kernel at every block
# size and several trajectory counts per workgroup, on both paths.
BETA0_CFGS = [dict(block_threads=b, lds_bytes=l) for b in (64, 128, 256, 512, 1024) for l in (256, 1024, 4096)]


@pytest.mark.parametrize("cfg", BETA0_CFGS, ids=[f"b{c['block_threads']}_lds{c['lds_bytes']}" for c in BETA0_CFGS])
def test_beta0_lanemap_every_block_size(cfg):
    s = ee.JobSpec(dim=2, lt=8, lx=8, ly=1, n=2, beta=0.0, l=3, n_step=40, n_traj=9, seed=8)
    say(f"[gpu] beta = 0 lane map, launch {cfg}")
    I_or, sp_or = eo.run(oracle_job(s), 3, want_spins=True)
    j = ee.Job(s)
    j.set_launch(cfg)
    j.thermalize(3)
    j.run_protocol()
    assert np.array_equal(j.work(), I_or)
    assert np.array_equal(j.spins(), sp_or)
    j.close()
    jobs = [ee.Job(s)]
    ee.batch_run(jobs, 3, cfg=cfg)
    assert np.array_equal(jobs[0].work(), I_or)
    assert np.array_equal(jobs[0].spins(), sp_or)
    jobs[0].close()


@pytest.mark.parametrize("cfg", [dict(block_threads=64), dict(block_threads=128), dict()])
def test_rows_wider_than_the_requested_block(cfg):
    # lx = 2048: 256 words per row; a 64-thread block is raised to 256 so
    # that every word of a row has a lane
    s = ee.JobSpec(dim=2, lt=4, lx=2048, ly=1, n=2, beta=BC2, l=1001, n_step=3, n_traj=3, seed=41)
    say(f"[gpu] wide rows {cfg}")
    I_or, sp_or = eo.run(oracle_job(s), 2, want_spins=True)
    j = ee.Job(s)
    j.set_launch(cfg)
    j.thermalize(2)
    j.run_protocol()
    assert np.array_equal(j.work(), I_or)
    assert np.array_equal(j.spins(), sp_or)
    j.close()
    jobs = [ee.Job(s), ee.Job(dataclasses.replace(s, lx=64, l=5, seed=42))]
    ee.batch_run(jobs, 2, cfg=cfg)
    assert np.array_equal(jobs[0].work(), I_or)
    assert np.array_equal(jobs[0].spins(), sp_or)
    I2, sp2 = eo.run(oracle_job(jobs[1].spec), 2, want_spins=True)
    assert np.array_equal(jobs[1].work(), I2)
    assert np.array_equal(jobs[1].spins(), sp2)
    for j in jobs:
        j.close()


def test_rows_wider_than_a_workgroup_stream():
    # 1025 words per row: streamed from HBM although the trajectory is small
    s = ee.JobSpec(dim=2, lt=2, lx=8200, ly=1, n=2, beta=BC2, l=4099, n_step=3, n_traj=2, seed=43)
    say("[gpu] rows of 1025 words")
    j = ee.Job(s)
    j.thermalize(2)
    j.run_protocol()
    I_or, sp_or = eo.run(oracle_job(s), 2, want_spins=True)
    assert np.array_equal(j.work(), I_or)
    assert np.array_equal(j.spins(), sp_or)
    j.close()


def test_whole_region_of_one_column_is_the_increment_from_no_cut():
    """A(0) -> A(1): the whole-region protocol with l = 1 and the c-function
    protocol with l = 0 are the same geometry, so the GPU gives the same bits."""
    kw = dict(dim=2, lt=8, lx=16, ly=1, n=2, beta=BC2, n_step=12, n_traj=6, seed=61)
    a, b = ee.Job(ee.JobSpec(l=1, whole=True, **kw)), ee.Job(ee.JobSpec(l=0, **kw))
    for j in (a, b):
        j.thermalize(4)
        j.run_protocol()
    assert np.array_equal(a.work(), b.work()) and np.array_equal(a.spins(), b.spins())
    a.close()
    b.close()


def test_whole_region_descriptions_are_checked():
    base = dict(dim=2, lt=8, lx=8, ly=1, n=2, beta=0.4, n_step=4, n_traj=2, seed=1, whole=True)
    for l in (0, 9):
        with pytest.raises(ee.EEError) as e:
            ee.ee_job_footprint(ee.JobSpec(l=l, **base).desc())
        assert e.value.status == ee.EE_EINVAL
    with pytest.raises(ee.EEError):
        ee.ee_job_footprint(ee.JobSpec(**dict(base, dim=3, ly=2, l=3, subsets=True)).desc())
    assert ee.ee_job_footprint(ee.JobSpec(l=8, **base).desc()) > 0


ONE_ROW_SPECS = [
    dict(dim=2, lt=8, lx=6, ly=1, n=2, beta=0.5, l=2, n_step=20, n_traj=6, seed=3),
    dict(dim=2, lt=2, lx=2, ly=1, n=2, beta=0.7, l=1, n_step=9, n_traj=7, seed=9),
    dict(dim=2, lt=12, lx=16, ly=1, n=2, beta=BC2, l=5, n_step=30, n_traj=9, seed=4, reverse=True),
    dict(dim=2, lt=16, lx=16, ly=1, n=2, beta=BC2, l=4, n_step=40, n_traj=8, seed=1),
    dict(dim=3, lt=4, lx=6, ly=2, n=2, beta=0.3, l=5, n_step=9, n_traj=5, seed=13),
    dict(dim=3, lt=4, lx=8, ly=4, n=3, beta=BC3, l=0, n_step=6, n_traj=3, seed=15),
    dict(dim=2, lt=6, lx=8, ly=1, n=3, beta=0.5, l=8, n_step=6, n_traj=4, seed=52, whole=True, reverse=True),
    dict(dim=3, lt=4, lx=16, ly=6, n=2, beta=0.23, l=9, n_step=18, n_traj=4, seed=17, subsets=True, reverse=True),
]


@pytest.mark.parametrize("kw", ONE_ROW_SPECS, ids=[f"D{k['dim']}_{k['lt']}x{k['lx']}x{k['ly']}_n{k['n']}"
                                                    for k in ONE_ROW_SPECS])
def test_one_row_per_lane_lookahead_matches_oracle(kw):
    """Launch shapes in which every lane owns at most one row (the lane-map
    order with the Philox outputs computed a half-sweep ahead), from one to
    sixteen waves per workgroup: bit-identical to the oracle."""
    s = ee.JobSpec(**kw)
    I_or, sp_or = eo.run(oracle_job(s), 5, want_spins=True)
    for block in (64, 256, 1024):
        say(f"[gpu] one row per lane {kw} block={block}")
        job = ee.Job(s)
        ee.batch_run([job], 5, cfg=dict(block_threads=block))
        assert np.array_equal(job.work(), I_or), block
        assert np.array_equal(job.spins(), sp_or), block
        job.close()


def test_launch_flags_are_checked():
    s = ee.JobSpec(dim=2, lt=8, lx=32, ly=1, n=2, beta=0.4, l=2, n_step=4, n_traj=2, seed=1)
    job = ee.Job(s)
    for flags in (6, 8, 16):
        with pytest.raises(ee.EEError) as e:
            job.set_launch(dict(flags=flags))
        assert e.value.status == ee.EE_EINVAL
    job.close()


def test_state_machine_errors():
    s = ee.JobSpec(dim=2, lt=8, lx=8, ly=1, n=2, beta=0.4, l=2, n_step=4, n_traj=2, seed=1)
    job = ee.Job(s)
    with pytest.raises(ee.EEError) as e:
        job.run_protocol()  # no spins yet
    assert e.value.status == ee.EE_ESTATE
    with pytest.raises(ee.EEError) as e:
        job.estimate()
    assert e.value.status == ee.EE_ESTATE
    with pytest.raises(ee.EEError):
        job.spins()
    job.thermalize(1)
    job.run_protocol()
    with pytest.raises(ee.EEError) as e:
        job.run_protocol()
    assert e.value.status == ee.EE_ESTATE
    with pytest.raises(ee.EEError) as e:
        job.thermalize(1)
    assert e.value.status == ee.EE_ESTATE
    with pytest.raises(ee.EEError) as e:
        ee.batch_run([job], 1)  # not fresh
    assert e.value.status == ee.EE_ESTATE
    with pytest.raises(ee.EEError):
        ee.ee_job_read_work(job.handle, 3)
    r1 = job.estimate()
    r2 = job.estimate()
    assert r1.dF == r2.dF
    job.reset()
    job.thermalize(1)
    job.run_protocol()
    assert job.estimate().dF == r1.dF
    job.close()


def _bench_launch(specs):
    """The launch shape bench.py times for a job set: the tuner's cached
    choice, else a fresh tuning."""
    from paper_2304_03311_amd import autotune
    return autotune.cached(specs, workloads.N_THERM) or autotune.tune(specs, workloads.N_THERM)


def test_full_size_2d_64x64_batch_sampled():
    """The 2D 64x64 workload (64 jobs, l = 0..63, N = 1000, n_t = 1024) in the
    benchmark's launch configuration; sampled trajectories vs the oracle and
    whole-batch invariants."""
    specs = workloads.config2_jobs()
    n_therm = workloads.N_THERM
    launch = _bench_launch(specs)
    say(f"[gpu] full 64x64 batch: {len(specs)} jobs x {specs[0].n_traj} trajectories, launch {launch}")
    jobs = [ee.Job(s) for s in specs]
    ee.batch_run(jobs, n_therm, cfg=launch)
    rng = np.random.default_rng(7)
    for ji, j in [(0, 0), (17, 1023), (40, int(rng.integers(0, 1024))), (63, 511), (31, 300), (32, 777)]:
        s = specs[ji]
        I_or, sp_or = eo.run(oracle_job(s), n_therm, j, j + 1, want_spins=True)
        say(f"[gpu]   sample job l={s.l} j={j}")
        assert jobs[ji].work()[j] == I_or[0]
        assert np.array_equal(jobs[ji].spins(j + 1)[j], sp_or[0])
    for s, job in zip(specs, jobs):
        I = job.work()
        assert np.all(np.abs(I) <= 2 * s.n * s.ly * s.n_step)
        assert np.all(I % 2 == 0)
        check_estimate(job.estimate(), I, s, f"64x64 l={s.l}")  # the estimator at n_t = 1024
    for j in jobs:
        j.close()


def test_full_size_2d_16x16_bench_launch():
    """The 16x16 job (64 trajectories, N = 256 after 100 thermalisation
    sweeps) in the launch the benchmark times (the tuner's choice: one-wave
    workgroups, no graph): every trajectory's work and final spins against
    the oracle, then a second run on the same arena gives the same bits."""
    s = workloads.config1_job()
    launch = _bench_launch([s])
    say(f"[gpu] 16x16 job, launch {launch}")
    I_or, sp_or = eo.run(oracle_job(s), workloads.N_THERM, want_spins=True)
    job = ee.Job(s)
    for rep in range(2):
        job.reset()
        ee.batch_run([job], workloads.N_THERM, cfg=launch)
        assert np.array_equal(job.work(), I_or)
        assert np.array_equal(job.spins(), sp_or)
    check_estimate(job.estimate(), I_or, s, "16x16")
    job.close()


def test_full_size_3d_32cube_sampled():
    """The 3D 32^3 bit-packed job through the per-job path and through the
    batched launch shape the benchmark times."""
    s = workloads.config3_job()
    say(f"[gpu] full 32^3 job: {s}")
    job = ee.Job(s)
    job.thermalize(workloads.N_THERM)
    job.run_protocol()
    launch = _bench_launch([s])
    say(f"[gpu]   batched with launch {launch}")
    bjob = ee.Job(s)
    ee.batch_run([bjob], workloads.N_THERM, cfg=launch)
    for j in (257, 3, 511):
        I_or, sp_or = eo.run(oracle_job(s), workloads.N_THERM, j, j + 1, want_spins=True)
        say(f"[gpu]   sample j={j}")
        for jb in (job, bjob):
            assert jb.work()[j] == I_or[0]
            assert np.array_equal(jb.spins(j + 1)[j], sp_or[0])
    I = job.work()
    assert np.array_equal(I, bjob.work())
    assert np.all(np.abs(I) <= 2 * s.n * s.ly * s.n_step)
    check_estimate(job.estimate(), I, s, "32^3")
    check_estimate(bjob.estimate(), I, s, "32^3 batched")
    job.close()
    bjob.close()


def test_full_size_streaming_96cube_sampled():
    """The two streaming workloads the benchmark times, in its launch
    configurations: 3D 96^3 (n = 2, N = 100 after 10 thermalisation sweeps)
    with 32 trajectories on the two-pass kernel and with 256 on the
    plane-marching kernel (the runtime's segment count).  The random numbers
    of trajectory j depend on (seed, site, sweep, j) only, so trajectories
    0..31 of both runs are bit-identical; sampled trajectories of each run
    are checked against the oracle."""
    base = dict(dim=3, lt=96, lx=96, ly=96, n=2, beta=workloads.BETA_3D, l=40, n_step=100, seed=5)
    runs = []
    for n_traj, flags in ((32, ee.EE_LAUNCH_TWO_PASS), (256, ee.EE_LAUNCH_MARCH)):
        s = ee.JobSpec(n_traj=n_traj, **base)
        say(f"[gpu] full 96^3 streaming: {n_traj} trajectories, flags {flags}")
        job = ee.Job(s)
        job.set_launch({"flags": flags})
        job.thermalize(10)
        job.run_protocol()
        runs.append((s, job))
    (s2, two), (sm, mar) = runs
    assert np.array_equal(two.work(), mar.work()[:32])
    assert np.array_equal(two.spins(), mar.spins(32))
    for s, job, j in ((s2, two, 29), (sm, mar, 200)):
        say(f"[gpu]   sample n_t={s.n_traj} j={j}")
        I_or, sp_or = eo.run(oracle_job(s), 10, j, j + 1, want_spins=True)
        assert job.work()[j] == I_or[0]
        assert np.array_equal(job.spins(j + 1)[j], sp_or[0])
    for s, job in runs:
        check_estimate(job.estimate(), job.work(), s, f"96^3 n_t={s.n_traj}")
        job.close()


def test_full_size_serving_shapes_3d_sampled():
    """The serving benchmark's own 3D shapes at full size: 24^3 in three-wave
    workgroups (parity-major rows) and 16^3 in one-wave workgroups, each
    with N = 1000 after the benchmark's thermalisation, 256 trajectories in
    one persistent launch of its shape; the first and the last trajectory
    against the oracle, and the estimate."""
    for L in (24, 16):
        s = ee.JobSpec(dim=3, lt=L, lx=L, ly=L, n=2, beta=workloads.BETA_3D, l=L // 3, n_step=1000, n_traj=256,
                       seed=600 + L, spin_format=ee.EE_SPINS_BITPACKED)
        launch = workloads.SERVE_LAUNCH[(3, L)]
        say(f"[gpu] full {L}^3 in the serving shape {launch}")
        job = ee.Job(s)
        ee.batch_run([job], workloads.N_THERM, cfg=launch)
        for j in (0, s.n_traj - 1):
            say(f"[gpu]   sample j={j}")
            I_or, sp_or = eo.run(oracle_job(s), workloads.N_THERM, j, j + 1, want_spins=True)
            assert job.work()[j] == I_or[0]
            assert np.array_equal(job.spins(j + 1)[j], sp_or[0])
        check_estimate(job.estimate(), job.work(), s, f"{L}^3 serving shape")
        job.close()


def test_full_size_24_uneven_jobs_sampled():
    """The 24 uneven jobs (2D L = 24..96, 3D L = 16..32, N = 500..2000) in one
    persistent launch of the benchmark's shape: one sampled trajectory of
    every job against the oracle, and every estimate."""
    specs = workloads.config4_jobs()
    launch = _bench_launch(specs)
    say(f"[gpu] 24 uneven jobs, launch {launch}")
    jobs = [ee.Job(s) for s in specs]
    ee.batch_run(jobs, workloads.N_THERM, cfg=launch)
    rng = np.random.default_rng(24)
    for s, job in zip(specs, jobs):
        j = int(rng.integers(0, s.n_traj))
        say(f"[gpu]   sample D={s.dim} L={s.lx} N={s.n_step} l={s.l} j={j}")
        I_or, sp_or = eo.run(oracle_job(s), workloads.N_THERM, j, j + 1, want_spins=True)
        assert job.work()[j] == I_or[0]
        assert np.array_equal(job.spins(j + 1)[j], sp_or[0])
        check_estimate(job.estimate(), job.work(), s, f"c4 D={s.dim} L={s.lx} N={s.n_step}")
    for j in jobs:
        j.close()


STREAM_CASES = [c for c in CASES if c[1].get("spin_format", 0) == 0 and c[1]["n_traj"] <= 16]


@pytest.mark.parametrize("name,kw,n_therm", STREAM_CASES, ids=[c[0] for c in STREAM_CASES])
def test_streaming_path_matches_oracle(name, kw, n_therm):
    """The HBM-streaming path (one launch per half-sweep), forced on lattices
    that would fit on chip, is bit-identical to the oracle."""
    s = ee.JobSpec(**kw)
    say(f"[gpu] streaming {name}")
    job = ee.Job(s)
    job.set_launch({"flags": ee.EE_LAUNCH_STREAMING})
    job.thermalize(n_therm // 2)
    job.thermalize(n_therm - n_therm // 2)
    job.run_protocol()
    I_or, sp_or = eo.run(oracle_job(s), n_therm, want_spins=True)
    assert np.array_equal(job.work(), I_or)
    assert np.array_equal(job.spins(), sp_or)
    check_estimate(job.estimate(), I_or, s, f"streaming {name}")
    job.close()


WIDE_STREAM = [kw for kw in WIDE_SPECS if kw.get("spin_format", 0) == 0]


@pytest.mark.parametrize("kw", WIDE_STREAM, ids=[f"lx{kw['lx']}_d{kw['dim']}" for kw in WIDE_STREAM])
def test_streaming_with_wide_rows_matches_oracle(kw):
    """Rows of a multiple of 16 sites per colour stream through the 4-wave
    kernel with four words per lane (rows of three words take W = 3)."""
    s = ee.JobSpec(**kw)
    say(f"[gpu] streaming wide rows {kw}")
    job = ee.Job(s)
    job.set_launch({"flags": ee.EE_LAUNCH_STREAMING})
    job.thermalize(3)
    job.run_protocol()
    I_or, sp_or = eo.run(oracle_job(s), 3, want_spins=True)
    assert np.array_equal(job.work(), I_or)
    assert np.array_equal(job.spins(), sp_or)
    job.close()


def _march_segments(lt):
    return sorted({min(k, max(1, lt // 2)) for k in (1, 2, 3, lt // 2)})


@pytest.mark.parametrize("name,kw,n_therm", STREAM_CASES, ids=[c[0] for c in STREAM_CASES])
def test_marching_path_matches_oracle(name, kw, n_therm):
    """The plane-marching streaming kernel, forced with 1, 2, 3 and lt/2
    segments per trajectory (every segment boundary takes the fix-up pass),
    is bit-identical to the oracle."""
    s = ee.JobSpec(**kw)
    I_or, sp_or = eo.run(oracle_job(s), n_therm, want_spins=True)
    for nseg in _march_segments(s.lt):
        say(f"[gpu] marching {name} segments={nseg}")
        job = ee.Job(s)
        job.set_launch({"flags": ee.EE_LAUNCH_MARCH, "grid_blocks": nseg})
        job.thermalize(n_therm // 2)
        job.thermalize(n_therm - n_therm // 2)
        job.run_protocol()
        assert np.array_equal(job.work(), I_or), nseg
        assert np.array_equal(job.spins(), sp_or), nseg
        check_estimate(job.estimate(), I_or, s, f"marching {name}")
        job.close()


@pytest.mark.parametrize("kw", WIDE_STREAM, ids=[f"lx{kw['lx']}_d{kw['dim']}" for kw in WIDE_STREAM])
def test_marching_with_wide_rows_matches_oracle(kw):
    s = ee.JobSpec(**kw)
    I_or, sp_or = eo.run(oracle_job(s), 3, want_spins=True)
    for nseg in _march_segments(s.lt):
        say(f"[gpu] marching wide rows {kw} segments={nseg}")
        job = ee.Job(s)
        job.set_launch({"flags": ee.EE_LAUNCH_MARCH, "grid_blocks": nseg})
        job.thermalize(3)
        job.run_protocol()
        assert np.array_equal(job.work(), I_or), nseg
        assert np.array_equal(job.spins(), sp_or), nseg
        job.close()


def test_streaming_kernel_choice_and_errors():
    """The marching kernel with the runtime's segment count gives the
    two-pass kernel's bits on a many-trajectory job; forcing the march where
    its plane ring exceeds LDS is refused."""
    s = ee.JobSpec(dim=3, lt=12, lx=32, ly=24, n=2, beta=BC3, l=9, n_step=6, n_traj=64, seed=61)
    out = []
    for flags in (ee.EE_LAUNCH_MARCH, ee.EE_LAUNCH_TWO_PASS):
        say(f"[gpu] kernel choice flags={flags}")
        job = ee.Job(s)
        job.set_launch({"flags": flags})
        job.thermalize(2)
        job.run_protocol()
        out.append((job.work(), job.spins()))
        job.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    I_or, sp_or = eo.run(oracle_job(s), 2, 37, 38, want_spins=True)
    assert out[0][0][37] == I_or[0] and np.array_equal(out[0][1][37], sp_or[0])
    # a plane (one replica) of 2 * 128 * 64 words: its five-slot ring is 320 KiB
    big = ee.JobSpec(dim=3, lt=4, lx=512, ly=128, n=2, beta=BC3, l=3, n_step=2, n_traj=1, seed=62)
    job = ee.Job(big)
    with pytest.raises(ee.EEError) as e:
        job.set_launch({"flags": ee.EE_LAUNCH_MARCH})
    assert e.value.status == ee.EE_EUNSUPPORTED
    job.close()


@pytest.mark.parametrize("kw", [
    dict(dim=3, lt=48, lx=48, ly=48, n=2, beta=BC3, l=20, n_step=10, n_traj=4, seed=31),
    dict(dim=2, lt=1024, lx=128, ly=1, n=2, beta=BC2, l=64, n_step=6, n_traj=2, seed=32, reverse=True),
], ids=["3d_48cube", "2d_1024x128"])
def test_lattices_beyond_lds_stream_from_hbm(kw):
    s = ee.JobSpec(**kw)
    say(f"[gpu] large lattice {kw}")
    job = ee.Job(s)
    job.thermalize(4)
    job.run_protocol()
    I_or, sp_or = eo.run(oracle_job(s), 4, want_spins=True)
    assert np.array_equal(job.work(), I_or)
    assert np.array_equal(job.spins(), sp_or)
    check_estimate(job.estimate(), I_or, s, "large lattice")
    with pytest.raises(ee.EEError) as e:
        j2 = ee.Job(s)
        ee.batch_run([j2], 1)
    assert e.value.status == ee.EE_EUNSUPPORTED
    job.close()


def test_zz_estimator_worst_case_report():
    """Prints the largest Delta F deviation of the module's parity checks."""
    say(f"[gpu] largest |dF_gpu - dF_oracle| / max(|dF_oracle|, 1e-3) = {_DF_WORST[0]:.3g} ({_DF_WORST[1]})")
    assert _DF_WORST[0] <= 1e-12
