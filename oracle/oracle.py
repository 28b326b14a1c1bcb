"""ctypes front end of the C oracle (ee_oracle.c).  TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this module.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_build.ORACLE_SO):
            _build.build_oracle()
        L = ctypes.CDLL(_build.ORACLE_SO)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.eo_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.eo_philox4x32_10.restype = None
        L.eo_threshold.argtypes = [ctypes.c_double, ctypes.c_int64, ctypes.c_int32]
        L.eo_threshold.restype = ctypes.c_uint32
        L.eo_run.argtypes = [ctypes.c_int] * 5 + [ctypes.c_double] + [ctypes.c_int] * 3 + [
            ctypes.c_uint64] + [ctypes.c_int] * 5 + [ctypes.c_void_p, ctypes.c_void_p]
        L.eo_run.restype = ctypes.c_int
        L.eo_count_ramped_bonds.argtypes = [ctypes.c_int] * 6
        L.eo_count_ramped_bonds.restype = ctypes.c_int
        L.eo_energy_units.argtypes = [ctypes.c_int] * 9 + [ctypes.c_void_p, ctypes.c_void_p]
        L.eo_energy_units.restype = ctypes.c_int
        L.eo_estimate.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        L.eo_estimate.restype = ctypes.c_int
        L.eo_site_fields.argtypes = [ctypes.c_int] * 5 + [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32] + [
            ctypes.c_int] * 4 + [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.eo_site_fields.restype = ctypes.c_int
        _lib = L
    return _lib


def philox(ctr, key) -> tuple[int, int, int, int]:
    A = ctypes.c_uint32 * 4
    B = ctypes.c_uint32 * 2
    out = A()
    lib().eo_philox4x32_10(A(*ctr), B(*key), out)
    return tuple(int(v) for v in out)


def threshold(beta: float, K: int, N: int) -> int:
    return int(lib().eo_threshold(beta, K, N))


@dataclass
class Job:
    """Problem statement of one job (Sec. 3 and Sec. 4 conventions)."""
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
    reverse: bool = False
    subsets: bool = False  # protocol 2 of App. B: the Ly rows ramped one after the other
    whole: bool = False  # whole-region protocol (Sec. 3): all cut links of x < l ramped at once

    @property
    def nsites(self) -> int:
        return self.n * self.lt * self.ly * self.lx

    @property
    def flags(self) -> int:
        return (1 if self.reverse else 0) | (2 if self.subsets else 0) | (4 if self.whole else 0)

    @property
    def S(self) -> int:
        """Weight unit beta/S: S = N, or N/Ly for protocol 2."""
        return self.n_step // self.ly if self.subsets else self.n_step


def run(job: Job, n_therm: int, j0: int = 0, j1: int | None = None, n_step_run: int | None = None,
        want_spins: bool = False):
    """Run trajectories [j0, j1).  Returns (I[int64], spins[int8] or None)."""
    j1 = job.n_traj if j1 is None else j1
    n_step_run = job.n_step if n_step_run is None else n_step_run
    I = np.zeros(max(j1 - j0, 0), dtype=np.int64)
    spins = np.zeros((max(j1 - j0, 0), job.nsites), dtype=np.int8) if want_spins else None
    rc = lib().eo_run(job.dim, job.lt, job.lx, job.ly, job.n, job.beta, job.l, job.n_step,
                      job.n_traj, job.seed, job.flags, n_therm, j0, j1, n_step_run,
                      I.ctypes.data, spins.ctypes.data if spins is not None else None)
    if rc != 0:
        raise ValueError(f"eo_run failed ({rc}) for {job}")
    return I, spins


def site_fields(dim, lt, lx, ly, n, seed, g, j, r, t, y, x, U):
    """(v, w, decision) of one site in sweep g: the two 16-bit fields and the
    oracle's lazy Metropolis decision for threshold U."""
    v, w, d = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_int()
    rc = lib().eo_site_fields(dim, lt, lx, ly, n, seed, g, j, r, t, y, x, U, ctypes.byref(v), ctypes.byref(w),
                              ctypes.byref(d))
    if rc != 0:
        raise ValueError(rc)
    return int(v.value), int(w.value), int(d.value)


def count_ramped_bonds(dim, lt, lx, ly, n, l) -> int:
    return int(lib().eo_count_ramped_bonds(dim, lt, lx, ly, n, l))


def energy_units(job: Job, m: int, spins: np.ndarray) -> int:
    s = np.ascontiguousarray(spins, dtype=np.int8)
    out = ctypes.c_int64()
    rc = lib().eo_energy_units(job.dim, job.lt, job.lx, job.ly, job.n, job.l, job.n_step, m, job.flags,
                               s.ctypes.data, ctypes.addressof(out))
    if rc != 0:
        raise ValueError(rc)
    return int(out.value)


@dataclass
class Estimate:
    dF: float
    dS: float
    dF_err: float
    w_mean: float
    w_var: float
    ess: float
    i_min: int
    i_max: int


def estimate(I: np.ndarray, beta: float, N: int, n_rep: int) -> Estimate:
    I = np.ascontiguousarray(I, dtype=np.int64)
    out = np.zeros(8)
    imm = np.zeros(2, dtype=np.int64)
    rc = lib().eo_estimate(I.ctypes.data, len(I), beta, N, n_rep, out.ctypes.data, imm.ctypes.data)
    if rc != 0:
        raise ValueError(rc)
    return Estimate(out[0], out[1], out[2], out[3], out[4], out[5], int(imm[0]), int(imm[1]))


def attempts(job: Job, n_therm: int) -> int:
    return job.n_traj * job.nsites * (n_therm + job.n_step)


BETA_C_2D = 0.5 * math.log(1.0 + math.sqrt(2.0))
