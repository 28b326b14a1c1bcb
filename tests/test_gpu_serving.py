"""Serving: continuous batching through the persistent kernel, with HBM
admission.  Each result must be the same alone and in the mix (bit-identical
works, spins and estimates), and every served job is checked against the
oracle on a sampled trajectory."""
from __future__ import annotations

import math
import sys
import time

import numpy as np
import pytest

from oracle import oracle as eo
from paper_2304_03311_amd import ee, serve, workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def small_mix(n=14, seed=3):
    stream = workloads.serving_stream(n, rate_per_s=1000.0, seed=seed, max_l3=48,
                                      n_traj_choices=(16, 32, 64), n_step_choices=(20, 40, 80),
                                      l3_weights={16: 0.6, 48: 0.4}, large_n_traj=(2,))
    return serve.requests_from_stream(stream)


def oracle_job(s: ee.JobSpec) -> eo.Job:
    return eo.Job(s.dim, s.lt, s.lx, s.ly, s.n, s.beta, s.l, s.n_step, s.n_traj, s.seed, s.reverse, s.subsets,
                  s.whole)


def alone(spec, n_therm):
    job = ee.Job(spec)
    job.thermalize(n_therm)
    job.run_protocol()
    r = job.estimate()
    w = job.work()
    job.close()
    return r, w


def test_results_identical_alone_and_in_the_mix():
    reqs = small_mix()
    srv = serve.Server(hbm_budget_bytes=1 << 34, n_therm=20, keep_work=True, keep_spins=True,
                       launch=dict(block_threads=256), chunk_units=8)
    say(f"[gpu] serving {len(reqs)} requests")
    done = srv.run(reqs, realtime=False)
    srv.close()
    assert len(done) == len(reqs)
    assert srv.stats.max_resident > 1
    for req in done:
        s = req.spec
        r, w = alone(s, 20)
        assert np.array_equal(req.work, w), s
        assert req.result.dF == r.dF and (req.result.dF_err == r.dF_err or (
            math.isnan(r.dF_err) and math.isnan(req.result.dF_err)))
        # every served job against the oracle on its first trajectory
        say(f"[gpu]   oracle check D={s.dim} L={s.lx} n_t={s.n_traj} N={s.n_step} streamed={req.streamed}")
        I_or, sp_or = eo.run(oracle_job(s), 20, 0, 1, want_spins=True)
        assert req.work[0] == I_or[0]
        assert np.array_equal(req.spins, sp_or[0])
    assert any(r.streamed for r in done)  # a job on the HBM-streaming path took part
    assert any(not r.streamed for r in done)


def test_shipped_serving_shapes_match_alone_and_oracle():
    """The serving benchmark's launch shapes (by dimension, and by extent for
    16^3 and 24^3, each size in chunks of its own shape): every job is
    bit-identical to its run alone and to the oracle on its first
    trajectory."""
    specs = [ee.JobSpec(dim=3, lt=24, lx=24, ly=24, n=2, beta=0.23, l=7, n_step=6, n_traj=5, seed=501,
                        spin_format=ee.EE_SPINS_BITPACKED),
             ee.JobSpec(dim=3, lt=16, lx=16, ly=16, n=2, beta=workloads.BETA_3D, l=3, n_step=8, n_traj=9,
                        seed=502, spin_format=ee.EE_SPINS_BITPACKED, reverse=True),
             ee.JobSpec(dim=3, lt=32, lx=32, ly=32, n=2, beta=0.21, l=20, n_step=4, n_traj=3, seed=503,
                        spin_format=ee.EE_SPINS_BITPACKED),
             ee.JobSpec(dim=2, lt=64, lx=64, ly=1, n=2, beta=workloads.BETA_C_2D, l=30, n_step=10, n_traj=17,
                        seed=504),
             ee.JobSpec(dim=3, lt=24, lx=24, ly=24, n=2, beta=workloads.BETA_3D, l=0, n_step=3, n_traj=2,
                        seed=505, spin_format=ee.EE_SPINS_BITPACKED)]
    reqs = serve.requests_from_stream([(0.0, s) for s in specs])
    srv = serve.Server(hbm_budget_bytes=1 << 34, n_therm=6, keep_work=True, keep_spins=True,
                       launch=workloads.SERVE_LAUNCH)
    say(f"[gpu] serving {len(reqs)} requests in the benchmark's shapes")
    done = srv.run(reqs, realtime=False)
    srv.close()
    assert len(done) == len(reqs) and not any(r.streamed for r in done)
    for req in done:
        s = req.spec
        say(f"[gpu]   check D={s.dim} L={s.lx} n_t={s.n_traj} N={s.n_step}")
        r, w = alone(s, 6)
        assert np.array_equal(req.work, w), s
        assert req.result.dF == r.dF
        I_or, sp_or = eo.run(oracle_job(s), 6, 0, 1, want_spins=True)
        assert req.work[0] == I_or[0]
        assert np.array_equal(req.spins, sp_or[0])


def test_server_matches_batch_path_across_chunks():
    """Jobs whose units span several chunks (chunk_units = 3) give the batch
    path's bits."""
    specs = [ee.JobSpec(dim=2, lt=16, lx=32, ly=1, n=2, beta=workloads.BETA_C_2D, l=7, n_step=30, n_traj=13,
                        seed=91),
             ee.JobSpec(dim=3, lt=8, lx=8, ly=8, n=2, beta=workloads.BETA_3D, l=2, n_step=25, n_traj=9, seed=92,
                        spin_format=ee.EE_SPINS_BITPACKED),
             ee.JobSpec(dim=2, lt=8, lx=24, ly=1, n=3, beta=0.5, l=11, n_step=12, n_traj=7, seed=93, reverse=True)]
    cfg = dict(block_threads=64, lds_bytes=4096)
    ref = [ee.Job(s) for s in specs]
    ee.batch_run(ref, 10, cfg=cfg)
    srv = ee.ee_server_create(cfg, 10, 2, 3)
    jobs = [ee.Job(s) for s in specs]
    for j in jobs:
        ee.ee_server_submit(srv, j.handle)
    got = []
    t0 = time.perf_counter()
    while len(got) < len(jobs) and time.perf_counter() - t0 < 60:
        got += ee.ee_server_poll(srv)
        time.sleep(1e-3)
    assert sorted(got) == sorted(j.handle for j in jobs)
    assert ee.ee_server_open_jobs(srv) == 0
    for a, b in zip(ref, jobs):
        assert np.array_equal(a.work(), b.work())
        assert np.array_equal(a.spins(), b.spins())
        assert a.estimate().dF == b.estimate().dF
    ee.ee_server_destroy(srv)
    for j in ref + jobs:
        j.close()


def test_server_runs_a_later_short_job_beside_a_long_one():
    """Work of jobs submitted at different times overlaps on the device: a
    short job submitted after a long one (whose units leave most CUs idle)
    finishes first."""
    long = ee.JobSpec(dim=3, lt=16, lx=16, ly=16, n=2, beta=workloads.BETA_3D, l=5, n_step=3000, n_traj=8, seed=94)
    short = ee.JobSpec(dim=2, lt=16, lx=16, ly=1, n=2, beta=workloads.BETA_C_2D, l=4, n_step=20, n_traj=8, seed=95)
    srv = ee.ee_server_create(dict(block_threads=256), 20, 2, 0)
    a, b = ee.Job(long), ee.Job(short)
    ee.ee_server_submit(srv, a.handle)
    # the job under way is SERVED: other calls on it are refused
    for call in (lambda: a.thermalize(1), a.spins, a.reset, a.close):
        with pytest.raises(ee.EEError) as e:
            call()
        assert e.value.status == ee.EE_ESTATE
    ee.ee_server_submit(srv, b.handle)
    order = []
    t0 = time.perf_counter()
    while len(order) < 2 and time.perf_counter() - t0 < 60:
        order += ee.ee_server_poll(srv)
        time.sleep(1e-4)
    assert order == [b.handle, a.handle]
    ee.ee_server_destroy(srv)
    # reported jobs are read on their own streams after the server is gone
    I_or, _ = eo.run(oracle_job(short), 20)
    assert np.array_equal(b.work(), I_or)
    assert a.estimate().n_traj == long.n_traj
    a.close()
    b.close()


def test_server_rejects_streamed_jobs_and_bad_arguments():
    srv = ee.ee_server_create(None, 5, 1, 0)
    big = ee.JobSpec(dim=3, lt=48, lx=48, ly=48, n=2, beta=workloads.BETA_3D, l=3, n_step=2, n_traj=1, seed=1)
    assert not ee.ee_job_on_chip(big.desc())
    j = ee.Job(big)
    with pytest.raises(ee.EEError) as e:
        ee.ee_server_submit(srv, j.handle)
    assert e.value.status == ee.EE_EUNSUPPORTED
    j.close()
    ee.ee_server_destroy(srv)
    for bad in ((None, -1, 1, 0), (None, 5, 0, 0), (None, 5, 9, 0), (None, 5, 1, -1)):
        with pytest.raises(ee.EEError) as e:
            ee.ee_server_create(*bad)
        assert e.value.status == ee.EE_EINVAL


def test_admission_respects_the_hbm_budget():
    reqs = small_mix(10, seed=5)
    fps = [ee.ee_job_footprint(r.spec.desc()) for r in reqs]
    budget = 2 * max(fps)
    srv = serve.Server(hbm_budget_bytes=budget, n_therm=10)
    done = srv.run(reqs, realtime=False)
    srv.close()
    assert len(done) == len(reqs)
    assert srv.stats.max_resident_bytes <= budget
    assert srv.used == 0 and srv.resident == 0


def test_realtime_poisson_stream_reports_latency():
    stream = workloads.serving_stream(60, rate_per_s=200.0, seed=9, max_l3=16, n_traj_choices=(32, 64),
                                      n_step_choices=(50, 100))
    srv = serve.Server(hbm_budget_bytes=1 << 34, n_therm=20)
    done = srv.run(serve.requests_from_stream(stream), realtime=True)
    srv.close()
    s = srv.stats.summary()
    assert s["completed"] == 60 and s["p99_ms"] >= s["p50_ms"] > 0
    assert all(r.done >= r.admitted >= r.arrival for r in done)
