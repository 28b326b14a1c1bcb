"""Python binding of the C ABI in include/ee.h (argument marshalling only).

Every step of the estimator runs in the gfx950 kernels of libee.so; PyTorch
is used only to allocate the device arena of a job and to supply the HIP
stream.  The functions below carry the C names; ``Job`` is a small
convenience owner of one arena.  If libee.so is missing or cannot be loaded
every call raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libee.so")

EE_OK, EE_EINVAL, EE_ENOMEM, EE_EHIP, EE_ESTATE, EE_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
EE_SPINS_INT8, EE_SPINS_BITPACKED = 0, 1
EE_FLAG_REVERSE = 1
EE_FLAG_SUBSETS = 2
EE_FLAG_WHOLE = 4
EE_LAUNCH_STREAMING = 1
EE_LAUNCH_MARCH = 2
EE_LAUNCH_TWO_PASS = 4


class ee_job_desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("lt", ctypes.c_int32), ("lx", ctypes.c_int32),
                ("ly", ctypes.c_int32), ("n_replicas", ctypes.c_int32), ("l", ctypes.c_int32),
                ("n_step", ctypes.c_int32), ("n_traj", ctypes.c_int32), ("beta", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("spin_format", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class ee_result(ctypes.Structure):
    _fields_ = [("dF", ctypes.c_double), ("dS", ctypes.c_double), ("dF_err", ctypes.c_double),
                ("w_mean", ctypes.c_double), ("w_var", ctypes.c_double), ("ess", ctypes.c_double),
                ("i_min", ctypes.c_int64), ("i_max", ctypes.c_int64), ("attempts", ctypes.c_int64),
                ("n_traj", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class ee_launch_cfg(ctypes.Structure):
    _fields_ = [("block_threads", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class EEError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


_lib = None
_SIGS = {
    "ee_job_footprint": [ctypes.POINTER(ee_job_desc), ctypes.POINTER(ctypes.c_size_t)],
    "ee_job_on_chip": [ctypes.POINTER(ee_job_desc), ctypes.POINTER(ctypes.c_int32)],
    "ee_job_create": [ctypes.POINTER(ee_job_desc), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                      ctypes.POINTER(ctypes.c_void_p)],
    "ee_thermalize": [ctypes.c_void_p, ctypes.c_int32],
    "ee_run_protocol": [ctypes.c_void_p],
    "ee_estimate": [ctypes.c_void_p, ctypes.POINTER(ee_result)],
    "ee_job_read_work": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32],
    "ee_job_read_spins": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t],
    "ee_job_reset": [ctypes.c_void_p],
    "ee_batch_run": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p],
    "ee_batch_run_cfg": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ee_launch_cfg),
                         ctypes.c_void_p],
    "ee_batch_run_noalloc": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ee_launch_cfg),
                             ctypes.c_void_p],
    "ee_job_set_launch": [ctypes.c_void_p, ctypes.POINTER(ee_launch_cfg)],
    "ee_batch_kernel_ms": [ctypes.POINTER(ctypes.c_double)],
    "ee_job_destroy": [ctypes.c_void_p],
    "ee_server_create": [ctypes.POINTER(ee_launch_cfg), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                         ctypes.POINTER(ctypes.c_void_p)],
    "ee_server_submit": [ctypes.c_void_p, ctypes.c_void_p],
    "ee_server_poll": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "ee_server_open_jobs": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)],
    "ee_server_stream": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)],
    "ee_server_destroy": [ctypes.c_void_p],
}
EXPORTED = list(_SIGS) + ["ee_last_error", "ee_version", "ee_build_id"]


def lib() -> ctypes.CDLL:
    """Load libee.so (raises if it is missing: no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.ee_last_error.restype = ctypes.c_char_p
        L.ee_last_error.argtypes = []
        L.ee_version.restype = ctypes.c_char_p
        L.ee_version.argtypes = []
        L.ee_build_id.restype = ctypes.c_char_p
        L.ee_build_id.argtypes = []
        from .build import source_hash
        built, here = L.ee_build_id().decode(), source_hash()
        if built != here:
            raise RuntimeError(f"{LIB_PATH} was built from other sources (build id {built}, sources {here}); "
                               f"run __graft_entry__.build() again")
        _lib = L
    return _lib


def _check(fn: str, status: int) -> None:
    if status != EE_OK:
        raise EEError(fn, status, lib().ee_last_error().decode())


def make_desc(dim, lt, lx, ly, n_replicas, beta, l, n_step, n_traj, seed, spin_format=EE_SPINS_INT8,
              flags=0) -> ee_job_desc:
    return ee_job_desc(dim, lt, lx, ly, n_replicas, l, n_step, n_traj, float(beta), int(seed),
                       int(spin_format), int(flags))


def ee_job_footprint(desc: ee_job_desc) -> int:
    out = ctypes.c_size_t()
    _check("ee_job_footprint", lib().ee_job_footprint(ctypes.byref(desc), ctypes.byref(out)))
    return int(out.value)


def ee_job_on_chip(desc: ee_job_desc) -> bool:
    out = ctypes.c_int32()
    _check("ee_job_on_chip", lib().ee_job_on_chip(ctypes.byref(desc), ctypes.byref(out)))
    return bool(out.value)


def ee_job_create(desc: ee_job_desc, arena_ptr: int, arena_bytes: int, stream: int) -> int:
    h = ctypes.c_void_p()
    _check("ee_job_create", lib().ee_job_create(ctypes.byref(desc), arena_ptr, arena_bytes, stream,
                                                ctypes.byref(h)))
    return h.value


def ee_thermalize(job: int, n_sweeps: int) -> None:
    _check("ee_thermalize", lib().ee_thermalize(job, n_sweeps))


def ee_run_protocol(job: int) -> None:
    _check("ee_run_protocol", lib().ee_run_protocol(job))


def ee_estimate(job: int) -> ee_result:
    r = ee_result()
    _check("ee_estimate", lib().ee_estimate(job, ctypes.byref(r)))
    return r


def ee_job_read_work(job: int, count: int):
    import numpy as np
    out = np.zeros(count, dtype=np.int64)
    _check("ee_job_read_work", lib().ee_job_read_work(job, out.ctypes.data, count))
    return out


def ee_job_read_spins(job: int, n_traj: int, sites_per_traj: int):
    import numpy as np
    out = np.zeros(n_traj * sites_per_traj, dtype=np.int8)
    _check("ee_job_read_spins", lib().ee_job_read_spins(job, out.ctypes.data, out.size))
    return out.reshape(n_traj, sites_per_traj)


def ee_job_reset(job: int) -> None:
    _check("ee_job_reset", lib().ee_job_reset(job))


def _cfg(cfg) -> ee_launch_cfg | None:
    if cfg is None:
        return None
    if isinstance(cfg, ee_launch_cfg):
        return cfg
    return ee_launch_cfg(int(cfg.get("block_threads", 0)), int(cfg.get("lds_bytes", 0)),
                         int(cfg.get("grid_blocks", 0)), int(cfg.get("use_graph", 1)), int(cfg.get("flags", 0)))


def ee_batch_run(jobs: list[int], n_therm: int, stream: int, cfg=None) -> None:
    arr = (ctypes.c_void_p * len(jobs))(*jobs)
    c = _cfg(cfg)
    _check("ee_batch_run_cfg", lib().ee_batch_run_cfg(arr, len(jobs), n_therm,
                                                       ctypes.byref(c) if c is not None else None, stream))


def ee_batch_run_noalloc(jobs: list[int], n_therm: int, stream: int, cfg=None) -> None:
    arr = (ctypes.c_void_p * len(jobs))(*jobs)
    c = _cfg(cfg)
    _check("ee_batch_run_noalloc", lib().ee_batch_run_noalloc(arr, len(jobs), n_therm,
                                                               ctypes.byref(c) if c is not None else None, stream))


def ee_job_set_launch(job: int, cfg) -> None:
    c = _cfg(cfg)
    _check("ee_job_set_launch", lib().ee_job_set_launch(job, ctypes.byref(c) if c is not None else None))


def ee_batch_kernel_ms() -> float:
    v = ctypes.c_double()
    _check("ee_batch_kernel_ms", lib().ee_batch_kernel_ms(ctypes.byref(v)))
    return float(v.value)


def ee_job_destroy(job: int) -> None:
    _check("ee_job_destroy", lib().ee_job_destroy(job))


def ee_server_create(cfg, n_therm: int, max_inflight: int = 2, chunk_units: int = 0) -> int:
    c = _cfg(cfg)
    h = ctypes.c_void_p()
    _check("ee_server_create", lib().ee_server_create(ctypes.byref(c) if c is not None else None, n_therm,
                                                      max_inflight, chunk_units, ctypes.byref(h)))
    return h.value


def ee_server_submit(srv: int, job: int) -> None:
    _check("ee_server_submit", lib().ee_server_submit(srv, job))


def ee_server_poll(srv: int, cap: int = 256) -> list[int]:
    arr = (ctypes.c_void_p * cap)()
    n = ctypes.c_int32()
    _check("ee_server_poll", lib().ee_server_poll(srv, arr, cap, ctypes.byref(n)))
    return [arr[i] for i in range(n.value)]


def ee_server_stream(srv: int) -> int:
    h = ctypes.c_void_p()
    _check("ee_server_stream", lib().ee_server_stream(srv, ctypes.byref(h)))
    return int(h.value or 0)


def ee_server_open_jobs(srv: int) -> int:
    n = ctypes.c_int32()
    _check("ee_server_open_jobs", lib().ee_server_open_jobs(srv, ctypes.byref(n)))
    return int(n.value)


def ee_server_destroy(srv: int) -> None:
    _check("ee_server_destroy", lib().ee_server_destroy(srv))


def ee_version() -> str:
    return lib().ee_version().decode()


# ---------------------------------------------------------------------------
# Convenience owner of one job's arena (torch is used for device memory only)
# ---------------------------------------------------------------------------

@dataclass
class JobSpec:
    """Problem statement of one job (Sec. 3 of the paper)."""
    dim: int
    lt: int
    lx: int
    ly: int
    n: int
    beta: float
    l: int  # noqa: E741
    n_step: int
    n_traj: int
    seed: int
    spin_format: int = EE_SPINS_INT8
    reverse: bool = False
    subsets: bool = False  # protocol 2 of App. B
    whole: bool = False  # whole-region protocol of Sec. 3: Delta F = (n-1) S_n(l)

    def desc(self) -> ee_job_desc:
        flags = ((EE_FLAG_REVERSE if self.reverse else 0) | (EE_FLAG_SUBSETS if self.subsets else 0)
                 | (EE_FLAG_WHOLE if self.whole else 0))
        return make_desc(self.dim, self.lt, self.lx, self.ly, self.n, self.beta, self.l, self.n_step,
                         self.n_traj, self.seed, self.spin_format, flags)

    @property
    def S(self) -> int:
        """Coupling unit beta/S: N, or N/ly for the subset protocol."""
        return self.n_step // self.ly if self.subsets else self.n_step

    @property
    def sites(self) -> int:
        return self.n * self.lt * self.ly * self.lx


def _stream_handle(stream) -> int:
    """A torch stream, a raw hipStream_t (int), or None (torch's current stream)."""
    if isinstance(stream, int):
        return stream
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Job:
    """One job: a torch-allocated device arena plus the C handle."""

    def __init__(self, spec: JobSpec, stream=None, device: str = "cuda"):
        import torch
        self.spec = spec
        self.desc = spec.desc()
        self.bytes = ee_job_footprint(self.desc)
        self.arena = torch.empty(self.bytes, dtype=torch.uint8, device=device)
        self.stream = _stream_handle(stream)
        self.handle = ee_job_create(self.desc, self.arena.data_ptr(), self.bytes, self.stream)

    def thermalize(self, n_sweeps: int) -> None:
        ee_thermalize(self.handle, n_sweeps)

    def run_protocol(self) -> None:
        ee_run_protocol(self.handle)

    def estimate(self) -> ee_result:
        return ee_estimate(self.handle)

    def work(self, count: int | None = None):
        return ee_job_read_work(self.handle, self.spec.n_traj if count is None else count)

    def spins(self, n_traj: int | None = None):
        return ee_job_read_spins(self.handle, self.spec.n_traj if n_traj is None else n_traj, self.spec.sites)

    def reset(self) -> None:
        ee_job_reset(self.handle)

    def set_launch(self, cfg) -> None:
        ee_job_set_launch(self.handle, cfg)

    def close(self) -> None:
        if self.handle:
            ee_job_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_run(jobs: list[Job], n_therm: int, stream=None, cfg=None) -> None:
    ee_batch_run([j.handle for j in jobs], n_therm, _stream_handle(stream), cfg)


def batch_run_noalloc(jobs: list[Job], n_therm: int, stream=None, cfg=None) -> None:
    ee_batch_run_noalloc([j.handle for j in jobs], n_therm, _stream_handle(stream), cfg)
