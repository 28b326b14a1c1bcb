"""Host-side logic of the serving loop: the launch-shape map and which jobs
of the serving mix go to the on-chip server or the HBM-streaming path."""
from __future__ import annotations

from paper_2304_03311_amd import autotune, ee, serve, workloads


def test_shape_map_recognition():
    assert serve.is_shape_map(workloads.SERVE_LAUNCH)
    assert serve.is_shape_map({2: {"block_threads": 64}})
    assert serve.is_shape_map({(3, 24): {"block_threads": 192}})
    assert not serve.is_shape_map({"block_threads": 64, "lds_bytes": 4096})
    assert not serve.is_shape_map({})
    assert not serve.is_shape_map(None)
    assert not serve.is_shape_map({4: {"block_threads": 64}})
    assert not serve.is_shape_map({(3,): {"block_threads": 64}})


def test_extent_entries_take_precedence_over_the_dimension():
    m = workloads.SERVE_LAUNCH
    spec = lambda dim, L: ee.JobSpec(dim=dim, lt=L, lx=L, ly=L if dim == 3 else 1, n=2, beta=0.2, l=1,
                                     n_step=10, n_traj=4, seed=1)
    assert serve.launch_shape(m, spec(3, 24)) is m[(3, 24)]
    assert serve.launch_shape(m, spec(3, 16)) is m[(3, 16)]
    assert serve.launch_shape(m, spec(3, 32)) is m[3]
    assert serve.launch_shape(m, spec(2, 24)) is m[2]  # (2, 24) has no entry of its own
    assert serve.launch_shape({(3, 24): m[(3, 24)]}, spec(3, 32)) is None


def test_serving_mix_routes_jobs_and_every_on_chip_job_has_a_shape():
    """Every job of the 2000-request benchmark stream: on chip unless it is a
    3D lattice of L >= 48 (those stream from HBM), each on-chip job's
    trajectory fits one workgroup's LDS (the runtime raises a smaller LDS
    budget to one trajectory), and its shape has a multiple of 64 threads."""
    stream = workloads.serving_stream(2000, 200.0, seed=1, **workloads.SERVE_MIX)
    for _, s in stream:
        on_chip = ee.ee_job_on_chip(s.desc())
        assert on_chip == (not (s.dim == 3 and s.lx >= 48)), s
        if on_chip:
            shape = serve.launch_shape(workloads.SERVE_LAUNCH, s)
            assert shape is not None
            assert shape["block_threads"] % 64 == 0 and 64 <= shape["block_threads"] <= 1024
            assert autotune.traj_bytes(s) <= autotune.MAX_LDS, s
