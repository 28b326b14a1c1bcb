"""CPU checks of the C ABI: the library loads, exports every symbol that
include/ee.h declares, and validates job descriptions without a GPU."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

from paper_2304_03311_amd import ee

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ee.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ee_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = ee.lib()
    declared = _declared()
    assert "ee_job_create" in declared and "ee_batch_run" in declared
    out = subprocess.run(["nm", "-D", "--defined-only", ee.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for name in declared:
        assert name in exported, name
        assert hasattr(L, name)
    assert set(ee.EXPORTED) <= set(declared)


def test_struct_sizes_match_header():
    assert ctypes.sizeof(ee.ee_job_desc) == 56
    assert ctypes.sizeof(ee.ee_result) == 80
    assert ctypes.sizeof(ee.ee_launch_cfg) == 20


def _spec(**kw):
    base = dict(dim=2, lt=16, lx=16, ly=1, n=2, beta=0.44, l=4, n_step=10, n_traj=4, seed=1)
    base.update(kw)
    return ee.JobSpec(**base)


def test_footprint_of_valid_jobs():
    for kw in [{}, dict(dim=3, ly=8, lx=8, lt=8), dict(lx=6), dict(lx=2, l=1), dict(spin_format=1),
               dict(n=3), dict(n_traj=65535, n_step=1)]:
        nb = ee.ee_job_footprint(_spec(**kw).desc())
        assert nb > 0 and nb % 256 == 0


def test_bitpacked_footprint_is_smaller():
    a = ee.ee_job_footprint(_spec(lt=64, lx=64, n_traj=1024).desc())
    b = ee.ee_job_footprint(_spec(lt=64, lx=64, n_traj=1024, spin_format=1).desc())
    assert b < a


@pytest.mark.parametrize("kw", [
    dict(dim=4), dict(lt=15), dict(lx=7), dict(lx=0), dict(ly=2), dict(dim=3, ly=1), dict(dim=3, ly=3),
    dict(n=1), dict(beta=-0.1), dict(beta=float("nan")), dict(beta=float("inf")), dict(l=-1), dict(l=16),
    dict(n_step=0), dict(n_traj=0), dict(n_traj=70000), dict(spin_format=7),
])
def test_invalid_descriptions_are_rejected(kw):
    with pytest.raises(ee.EEError) as ei:
        ee.ee_job_footprint(_spec(**kw).desc())
    assert ei.value.status == ee.EE_EINVAL
    assert ee.lib().ee_last_error().decode() != ""


def test_unknown_flags_rejected():
    d = _spec().desc()
    d.flags = 6
    with pytest.raises(ee.EEError):
        ee.ee_job_footprint(d)


def test_too_large_for_lds_streams_in_int8_only():
    assert ee.ee_job_footprint(_spec(dim=3, lt=96, lx=96, ly=96).desc()) > 2 * 96 ** 3 * 4
    with pytest.raises(ee.EEError) as ei:
        ee.ee_job_footprint(_spec(dim=3, lt=96, lx=96, ly=96, spin_format=1).desc())
    assert ei.value.status == ee.EE_EUNSUPPORTED


def test_rows_wider_than_a_workgroup_stream_in_int8_only():
    # lx = 8200: 4100 sites of a colour per row = 1025 words, more than the
    # 1024 lanes of a workgroup; the trajectory itself (32 KiB) would fit LDS
    assert ee.ee_job_footprint(_spec(lt=2, lx=8200).desc()) > 0
    with pytest.raises(ee.EEError) as e:
        ee.ee_job_footprint(_spec(lt=2, lx=8200, spin_format=1).desc())
    assert e.value.status == ee.EE_EUNSUPPORTED
    # 1024 words per row still run on chip, also bit-packed
    assert ee.ee_job_footprint(_spec(lt=2, lx=8192, spin_format=1).desc()) > 0


def test_null_arguments():
    L = ee.lib()
    assert L.ee_job_footprint(None, None) == ee.EE_EINVAL
    assert L.ee_thermalize(None, 1) == ee.EE_EINVAL
    assert L.ee_run_protocol(None) == ee.EE_EINVAL
    assert L.ee_estimate(None, None) == ee.EE_EINVAL
    assert L.ee_batch_run(None, 0, 0, None) == ee.EE_EINVAL
    assert L.ee_job_destroy(None) == ee.EE_OK
    assert L.ee_batch_kernel_ms(None) == ee.EE_EINVAL


def test_create_rejects_small_or_misaligned_arena_without_touching_it():
    d = _spec().desc()
    need = ee.ee_job_footprint(d)
    h = ctypes.c_void_p()
    L = ee.lib()
    assert L.ee_job_create(ctypes.byref(d), ctypes.c_void_p(0x100000), need - 256, None, ctypes.byref(h)) == ee.EE_ENOMEM
    assert L.ee_job_create(ctypes.byref(d), ctypes.c_void_p(0x100010), need, None, ctypes.byref(h)) == ee.EE_EINVAL
    assert L.ee_job_create(ctypes.byref(d), None, need, None, ctypes.byref(h)) == ee.EE_EINVAL


def test_version():
    assert "gfx950" in ee.ee_version()
