"""Continuous-batching request loop for entropy-increment jobs.

Requests (job descriptions) arrive over time.  A request is admitted as soon
as two resources are free:

* a device slot: one of ``slots`` HIP streams, each holding one resident job;
* HBM: the job's arena (ee_job_footprint bytes) must fit the budget minus
  what the resident jobs hold.

Admission is first-come first-served.  A request that does not fit blocks
the queue until memory frees, so large jobs cannot starve.  An admitted job
gets its arena, and its launches (initial spins + thermalisation, protocol,
estimator) are enqueued on its slot's stream.  Those launches overlap on the
device with the launches of every other resident job.  Completion is found
by polling an event recorded after the job's launches.  The result is then
read (a 80-byte copy), the arena is released and the slot is reused.  The
lattices stay resident in HBM from admission to completion.

A job's result does not depend on which other jobs share the device.  Its
random numbers are indexed by (seed, site, sweep, trajectory) only, so a
result is bit-identical alone and in any mix (tests/test_gpu_serving.py).
"""
from __future__ import annotations

import time
from collections import deque
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

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.array([float("nan")])
        return {"completed": self.completed, "wall_s": self.wall_s,
                "jobs_per_s": self.completed / self.wall_s if self.wall_s > 0 else 0.0,
                "attempts_per_ns": self.attempts / (self.wall_s * 1e9) if self.wall_s > 0 else 0.0,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "max_resident_jobs": self.max_resident, "max_resident_bytes": self.max_resident_bytes}


class Server:
    def __init__(self, hbm_budget_bytes: int, slots: int = 8, n_therm: int = 100, keep_work: bool = False):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget_bytes)
        self.n_therm = n_therm
        self.keep_work = keep_work
        # default-priority streams only
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.free_slots = list(range(slots))
        self.waiting: deque[Request] = deque()
        self.resident: dict[int, tuple] = {}  # slot -> (request, job, event, bytes)
        self.used = 0
        self.stats = ServeStats()
        self._t0 = None

    # ------------------------------------------------------------------
    def now(self) -> float:
        return time.perf_counter() - self._t0

    def submit(self, req: Request) -> None:
        fp = ee.ee_job_footprint(req.spec.desc())
        if fp > self.budget:
            raise ValueError(f"request {req.rid} needs {fp} bytes, more than the whole budget")
        self.waiting.append(req)

    def _admit(self) -> None:
        while self.waiting and self.free_slots:
            req = self.waiting[0]
            fp = ee.ee_job_footprint(req.spec.desc())
            if self.used + fp > self.budget:
                return  # FCFS: wait for memory
            self.waiting.popleft()
            slot = self.free_slots.pop()
            stream = self.streams[slot]
            with self.torch.cuda.stream(stream):
                job = ee.Job(req.spec, stream=stream)
                job.thermalize(self.n_therm)
                job.run_protocol()
                ev = self.torch.cuda.Event()
                ev.record(stream)
            req.admitted = self.now()
            self.used += job.bytes
            self.resident[slot] = (req, job, ev, job.bytes)
            self.stats.max_resident = max(self.stats.max_resident, len(self.resident))
            self.stats.max_resident_bytes = max(self.stats.max_resident_bytes, self.used)

    def _reap(self) -> list[Request]:
        out = []
        for slot in list(self.resident):
            req, job, ev, nbytes = self.resident[slot]
            if not ev.query():
                continue
            req.result = job.estimate()  # estimator launch + 80-byte copy on this slot's stream
            if self.keep_work:
                req.work = job.work()
            req.done = self.now()
            job.close()
            del job
            self.used -= nbytes
            del self.resident[slot]
            self.free_slots.append(slot)
            self.stats.completed += 1
            self.stats.attempts += req.result.attempts
            self.stats.latencies.append(req.latency)
            out.append(req)
        return out

    def run(self, requests: list[Request], realtime: bool = True, idle_sleep: float = 1e-4) -> list[Request]:
        """Serve the requests (sorted by arrival).  realtime=False submits each
        request as soon as the previous one is submitted (a saturation run)."""
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
            self._admit()
            done = self._reap()
            finished.extend(done)
            if not done and realtime and pending and not self.waiting:
                dt = pending[0].arrival - self.now()
                if dt > 0:
                    time.sleep(min(dt, idle_sleep * 10))
            elif not done:
                time.sleep(idle_sleep)
        self.torch.cuda.synchronize()
        self.stats.wall_s = self.now()
        return finished


def requests_from_stream(stream) -> list[Request]:
    return [Request(i, spec, t) for i, (t, spec) in enumerate(stream)]
