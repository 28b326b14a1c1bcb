"""Serving: continuous batching with HBM admission.  Each result must be the
same alone and in the mix (bit-identical works and estimates)."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

from oracle import oracle as eo
from paper_2304_03311_amd import ee, serve, workloads

pytestmark = pytest.mark.gpu


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
    srv = serve.Server(hbm_budget_bytes=1 << 34, slots=4, n_therm=20, keep_work=True)
    print(f"[gpu] serving {len(reqs)} requests", file=sys.stderr, flush=True)
    done = srv.run(reqs, realtime=False)
    assert len(done) == len(reqs)
    assert srv.stats.max_resident > 1  # requests overlapped on the device
    for req in done:
        r, w = alone(req.spec, 20)
        assert np.array_equal(req.work, w), req.spec
        assert req.result.dF == r.dF and req.result.dF_err == r.dF_err or (
            math.isnan(r.dF_err) and math.isnan(req.result.dF_err))
    assert any(r.spec.dim == 3 and r.spec.lx == 48 for r in done)  # a streamed job took part
    # and the oracle agrees with a served job
    req = min(done, key=lambda r: r.spec.n_traj * r.spec.sites)
    s = req.spec
    I, _ = eo.run(eo.Job(s.dim, s.lt, s.lx, s.ly, s.n, s.beta, s.l, s.n_step, s.n_traj, s.seed, s.reverse), 20)
    assert np.array_equal(I, req.work)


def test_admission_respects_the_hbm_budget():
    reqs = small_mix(10, seed=5)
    fps = [ee.ee_job_footprint(r.spec.desc()) for r in reqs]
    budget = 2 * max(fps)
    srv = serve.Server(hbm_budget_bytes=budget, slots=8, n_therm=10)
    done = srv.run(reqs, realtime=False)
    assert len(done) == len(reqs)
    assert srv.stats.max_resident_bytes <= budget
    assert srv.used == 0 and not srv.resident


def test_realtime_poisson_stream_reports_latency():
    stream = workloads.serving_stream(60, rate_per_s=200.0, seed=9, max_l3=16, n_traj_choices=(32, 64),
                                      n_step_choices=(50, 100))
    srv = serve.Server(hbm_budget_bytes=1 << 34, slots=8, n_therm=20)
    done = srv.run(serve.requests_from_stream(stream), realtime=True)
    s = srv.stats.summary()
    assert s["completed"] == 60 and s["p99_ms"] >= s["p50_ms"] > 0
    assert all(r.done >= r.admitted >= r.arrival for r in done)
