"""Continuous-batching request loop for entropy-increment jobs.

Requests (job descriptions) arrive over time.  A request is admitted first
come, first served, as soon as its arena (ee_job_footprint bytes) fits the
HBM budget minus what the resident jobs hold; a request that does not fit
blocks the queue until memory frees, so large jobs cannot starve.

An admitted job's lattices stay in its arena from admission to completion.
Jobs whose trajectories fit one workgroup's LDS go to the native server
(ee_server_*): their work units join the server's queue and run in the
persistent sweep kernel's chunked launches, on the device together with the
units of every other admitted job, and the server launches a job's
estimator when its last unit has run.  Jobs too large for LDS run the
HBM-streaming per-job path on one of a few side streams; a worker thread
enqueues each such job's launches (a few thousand), so the serving loop
keeps feeding the server meanwhile.  When a job is done its result is read
(an 80-byte copy), its arena is released and the waiting requests are
admitted.

A job's result does not depend on which other jobs share the device: its
random numbers are indexed by (seed, site, sweep, trajectory) only, so a
result is bit-identical alone and in any mix (tests/test_gpu_serving.py).
"""
from __future__ import annotations

import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import ee


@dataclass
class Request:
    rid: int
    spec: ee.JobSpec
    arrival: float  # seconds, relative to the start of the run
    admitted: float = float("nan")
    done: float = float("nan")
    result: ee.ee_result | None = None
    work: np.ndarray | None = None
    spins: np.ndarray | None = None
    streamed: bool = False

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServeStats:
    completed: int = 0
    attempts: int = 0
    wall_s: float = 0.0
    max_resident: int = 0
    max_resident_bytes: int = 0
    latencies: list = field(default_factory=list)
    streamed_attempts: int = 0
    last_on_chip_s: float = 0.0
    last_streamed_s: float = 0.0
    host_s: dict = field(default_factory=lambda: {"create": 0.0, "submit": 0.0, "reap": 0.0, "finish": 0.0})

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.array([float("nan")])
        return {"completed": self.completed, "wall_s": self.wall_s,
                "jobs_per_s": self.completed / self.wall_s if self.wall_s > 0 else 0.0,
                "attempts_per_ns": self.attempts / (self.wall_s * 1e9) if self.wall_s > 0 else 0.0,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "max_resident_jobs": self.max_resident, "max_resident_bytes": self.max_resident_bytes,
                "streamed_attempts": self.streamed_attempts, "last_on_chip_done_s": self.last_on_chip_s,
                "last_streamed_done_s": self.last_streamed_s, "host_s": self.host_s}


def is_shape_map(launch) -> bool:
    """Whether `launch` maps dimensions (2, 3) or (dimension, L) pairs to
    launch shapes, rather than being one shape."""
    return isinstance(launch, dict) and bool(launch) and all(
        k in (2, 3) or (isinstance(k, tuple) and len(k) == 2 and k[0] in (2, 3)) for k in launch)


def launch_shape(shape_map: dict, spec: ee.JobSpec):
    """The launch shape of a job under a shape map: its (dimension, L)
    entry, else its dimension's, else None (the server's own shape)."""
    return shape_map.get((spec.dim, spec.lx), shape_map.get(spec.dim))


class Server:
    """hbm_budget_bytes: device memory the resident arenas may hold.
    launch: ee_launch_cfg of the chunk launches (dict or None), or a dict
    {dimension: cfg}: each job then takes the shape of its dimension (the
    server runs each shape's units in chunks of their own); keys
    (dimension, L) give the shape of the lattices of extent L in x and take
    precedence over the dimension's.
    max_inflight, chunk_units: the native server's launch slots and units per
    chunk.  stream_slots: side streams (and worker threads) for jobs on the
    HBM-streaming path.
    keep_work / keep_spins: copy each job's works / the spins of its first
    trajectory to the request (for checks)."""

    def __init__(self, hbm_budget_bytes: int, n_therm: int = 100, launch=None, max_inflight: int = 2,
                 chunk_units: int = 0, stream_slots: int = 3, keep_work: bool = False, keep_spins: bool = False):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget_bytes)
        self.n_therm = n_therm
        self.keep_work = keep_work
        self.keep_spins = keep_spins
        by_dim = is_shape_map(launch)
        self.launch_by_dim = launch if by_dim else {}
        self.native = ee.ee_server_create(None if by_dim else launch, n_therm, max_inflight, chunk_units)
        # Streams, all of default priority: the server's chunk slots and its
        # service stream (estimators, and the table uploads of the jobs made
        # for it), plus the side streams of streamed jobs.  The device has
        # four hardware queues; streams beyond that share in-order queues and
        # wait on each other's kernels.  Three side streams still pay: the
        # streamed jobs, whose kernels get CUs only as chunk workgroups
        # retire, then end well before the on-chip work instead of trailing
        # it (2000-job saturation run: about 2150-2200 attempts/ns against
        # about 2000 with one side stream).
        self.upload = ee.ee_server_stream(self.native)
        self.side = [torch.cuda.Stream() for _ in range(stream_slots)]
        self.free_side = list(range(stream_slots))
        self.pool = ThreadPoolExecutor(max_workers=stream_slots)
        self.waiting: deque[Request] = deque()
        self.streamed_queue: deque[Request] = deque()  # admitted streamed jobs without a side stream yet
        self.on_server: dict[int, tuple] = {}  # job handle -> (request, job)
        self.on_side: dict[int, tuple] = {}  # side slot -> (request, future of (job, event))
        self.used = 0
        self.stats = ServeStats()
        self._t0 = None

    @property
    def resident(self) -> int:
        return len(self.on_server) + len(self.on_side) + len(self.streamed_queue)

    def now(self) -> float:
        return time.perf_counter() - self._t0

    def submit(self, req: Request) -> None:
        fp = ee.ee_job_footprint(req.spec.desc())
        if fp > self.budget:
            raise ValueError(f"request {req.rid} needs {fp} bytes, more than the whole budget")
        self.waiting.append(req)

    def _admit(self, max_jobs: int = 16) -> None:
        """Admit up to max_jobs waiting requests (first come, first served)."""
        while self.waiting and max_jobs > 0:
            max_jobs -= 1
            req = self.waiting[0]
            desc = req.spec.desc()
            fp = ee.ee_job_footprint(desc)
            if self.used + fp > self.budget:
                return  # first come, first served: wait for memory
            self.waiting.popleft()
            req.admitted = self.now()
            self.used += fp
            if ee.ee_job_on_chip(desc):
                t0 = time.perf_counter()
                job = ee.Job(req.spec, stream=self.upload)
                shape = launch_shape(self.launch_by_dim, req.spec)
                if shape is not None:
                    job.set_launch(shape)
                t1 = time.perf_counter()
                ee.ee_server_submit(self.native, job.handle)
                t2 = time.perf_counter()
                self.stats.host_s["create"] += t1 - t0
                self.stats.host_s["submit"] += t2 - t1
                self.on_server[job.handle] = (req, job)
            else:
                req.streamed = True
                self.streamed_queue.append(req)
            self.stats.max_resident = max(self.stats.max_resident, self.resident)
            self.stats.max_resident_bytes = max(self.stats.max_resident_bytes, self.used)

    def _run_streamed(self, spec: ee.JobSpec, stream):
        job = ee.Job(spec, stream=stream)
        job.thermalize(self.n_therm)
        job.run_protocol()
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return job, ev

    def _start_streamed(self) -> None:
        """Jobs on the HBM-streaming path: the per-job path on a side stream,
        enqueued by a worker thread (their arenas are counted from admission)."""
        while self.streamed_queue and self.free_side:
            req = self.streamed_queue.popleft()
            slot = self.free_side.pop()
            self.on_side[slot] = (req, self.pool.submit(self._run_streamed, req.spec, self.side[slot]))

    def _finish(self, req: Request, job: ee.Job) -> None:
        req.result = job.estimate()
        if self.keep_work:
            req.work = job.work()
        if self.keep_spins:
            req.spins = job.spins(1)[0]
        req.done = self.now()
        self.used -= job.bytes
        job.close()
        self.stats.completed += 1
        self.stats.attempts += req.result.attempts
        self.stats.latencies.append(req.latency)
        if req.streamed:
            self.stats.streamed_attempts += req.result.attempts
            self.stats.last_streamed_s = req.done
        else:
            self.stats.last_on_chip_s = req.done

    def _reap(self) -> list[Request]:
        out = []
        t0 = time.perf_counter()
        handles = ee.ee_server_poll(self.native)
        t1 = time.perf_counter()
        for h in handles:
            req, job = self.on_server.pop(h)
            self._finish(req, job)
            out.append(req)
        self.stats.host_s["reap"] += t1 - t0
        self.stats.host_s["finish"] += time.perf_counter() - t1
        for slot in list(self.on_side):
            req, fut = self.on_side[slot]
            if not fut.done():
                continue
            job, ev = fut.result()
            if not ev.query():
                continue
            del self.on_side[slot]
            self.free_side.append(slot)
            self._finish(req, job)
            out.append(req)
        return out

    def run(self, requests: list[Request], realtime: bool = True, idle_sleep: float = 2e-4) -> list[Request]:
        """Serve the requests (sorted by arrival).  realtime=False submits every
        request at once (a saturation run)."""
        self._t0 = time.perf_counter()
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        finished: list[Request] = []
        while pending or self.waiting or self.resident:
            t = self.now()
            while pending and (not realtime or pending[0].arrival <= t):
                req = pending.popleft()
                if not realtime:
                    req.arrival = t
                self.submit(req)
            n_wait = len(self.waiting)
            self._admit()
            self._start_streamed()
            done = self._reap()
            finished.extend(done)
            if done or len(self.waiting) < n_wait:
                continue
            if realtime and pending and not self.waiting and not self.resident:
                time.sleep(max(0.0, min(pending[0].arrival - self.now(), 10 * idle_sleep)))
            else:
                time.sleep(idle_sleep)
        self.torch.cuda.synchronize()
        self.stats.wall_s = self.now()
        return finished

    def close(self) -> None:
        if self.native:
            self.pool.shutdown(wait=True)
            ee.ee_server_destroy(self.native)
            self.native = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def requests_from_stream(stream) -> list[Request]:
    return [Request(i, spec, t) for i, (t, spec) in enumerate(stream)]
