"""The staged kernel's fallback paths, forced and checked against the oracle.

The staged kernel copies, per wave and node, slabs of the brick along the
rays' shared dominant axis into LDS. Two cases read the brick pool instead:
rays of one wave that share no dominant direction (a very wide-angle view
from inside the volume), and a slab whose single layer does not fit the
staging space (rays many voxels apart, 1 KiB of staging). The render
statistics show each path was taken; the images match the oracle within
1e-4 (with the early-termination bracket) and equal the gather kernel's
bit for bit. Retries of the slab size show up on an ordinary view. Every
case runs on both pool slot layouts (linear rows and 4^3 micro-blocks),
whose staging copies and pool reads address the slots differently."""
import numpy as np
import pytest

import gen
from tests.helpers import (ERT, LAYOUT_IDS, LAYOUTS, TOL, bracket_error, gpu_volume,
                           oracle_bracket, oracle_scene)

pytestmark = pytest.mark.gpu


def _render(h, views, params, gather=False):
    import torch

    from paper_1804_08197_amd import sg
    p = dict(params, gather=1) if gather else params
    out = [torch.full((v["height"], v["width"], 4), float("nan"), device="cuda") for v in views]
    st = sg.sg_render_views_stats(h, views, p, out)
    torch.cuda.synchronize()
    return [o.cpu().numpy().astype(np.float64) for o in out], st


def _check(h, sc, views, params):
    imgs, st = _render(h, views, params)
    gimgs, _ = _render(h, views, params, gather=True)
    for i, v in enumerate(views):
        best, needed = bracket_error(imgs[i], oracle_bracket(sc, v, params))
        assert best.max() <= TOL, "view %d: max abs err %g" % (i, best.max())
        assert np.array_equal(imgs[i], gimgs[i])
    assert 0 < st["loop_iterations"] and st["total_samples"] <= 64 * st["loop_iterations"]
    assert st["node_lanes"] <= 64 * st["node_visits"]
    return st


@pytest.mark.parametrize("layout", LAYOUTS, ids=LAYOUT_IDS)
def test_rays_without_a_shared_direction_read_the_pool(layout):
    from paper_1804_08197_amd import sg
    vol = gen.random_volume((36, 40, 44), 21, dtype=np.uint16)
    tf = gen.tf_hot(a_start=30)
    h = gpu_volume([vol], 16, 2, [tf], [(0, 65535)], layout=layout)
    try:
        sc = oracle_scene([vol], 16, 2, [tf], [(0, 65535)])
        c = np.array([22.0, 20.0, 18.0])
        # about 170 degrees across 16 pixels: neighbouring rays of a wave
        # point along different axes
        v = gen.view(gen.look_at(c + np.array([0.3, 0.2, 0.1]), c + np.array([5.0, 3.0, 1.0])),
                     16, 16, 12.0)
        st = _check(h, sc, [v], {"ert": ERT, "tau": 1.0})
        print("no shared direction:", st, flush=True)
        assert st["pool_samples"] > 0
    finally:
        sg.sg_volume_destroy(h)


@pytest.mark.parametrize("layout", LAYOUTS, ids=LAYOUT_IDS)
def test_slab_wider_than_the_staging_space_reads_the_pool(layout):
    from paper_1804_08197_amd import sg
    vol = gen.random_volume((100, 120, 140), 22, dtype=np.uint16)
    tf = gen.tf_hot(a_start=30)
    h = gpu_volume([vol], 64, 1, [tf], [(0, 65535)], layout=layout)
    try:
        sg.sg_set_launch_config(h, {"kernel": 0, "tile": 16, "block": 64, "stage_bytes": 1024,
                                    "persistent": 0})
        sc = oracle_scene([vol], 64, 1, [tf], [(0, 65535)])
        c = np.array([70.0, 60.0, 50.0])
        # each pixel spans about ten voxels: one layer of a wave's region
        # holds far more than the 512 voxels of 1 KiB
        v = gen.view(gen.look_at(c + np.array([-300.0, 180.0, 120.0]), c), 24, 20, 0.3)
        st = _check(h, sc, [v], {"ert": ERT, "lod": 0, "bias": 0})
        print("slab too wide:", st, flush=True)
        assert st["pool_samples"] > 0
    finally:
        sg.sg_volume_destroy(h)


@pytest.mark.parametrize("layout", LAYOUTS, ids=LAYOUT_IDS)
def test_ordinary_view_stages_everything_and_retries_slab_sizes(layout):
    from paper_1804_08197_amd import sg
    vol = gen.random_volume((48, 56, 64), 23, dtype=np.uint16)
    tf = gen.tf_hot(a_start=30)
    h = gpu_volume([vol], 32, 2, [tf], [(0, 65535)], layout=layout)
    try:
        sg.sg_set_launch_config(h, {"kernel": 0, "tile": 16, "block": 64, "stage_bytes": 8192,
                                    "persistent": 0})
        sc = oracle_scene([vol], 32, 2, [tf], [(0, 65535)])
        c = np.array([32.0, 28.0, 24.0])
        v = gen.view(gen.look_at(c + np.array([-70.0, 50.0, 35.0]), c), 96, 80, 0.5)
        st = _check(h, sc, [v], {"ert": ERT, "tau": 1.0})
        print("ordinary:", st, flush=True)
        assert st["pool_samples"] == 0 and st["slabs"] > 0 and st["slab_retries"] > 0
    finally:
        sg.sg_volume_destroy(h)


@pytest.mark.parametrize("layout", LAYOUTS, ids=LAYOUT_IDS)
def test_rows_wider_than_a_copy_pass_are_staged_chunk_by_chunk(layout):
    """uint16 bricks of 128 voxels: a region row can hold more than 64
    4-byte chunks (one copy pass), which the staging copies chunk by chunk.
    One-wave 8x8 views down z, 80-120 voxels above the volume, wide across
    x (tan 1 to 1.5) and narrow across y (tan 0.02), over a 130-voxel-wide
    volume with one level: the rays of one wave cross both x edges of the
    first brick within its first slab, so that slab's rows hold the whole
    brick width (65 chunks), a few rows and layers deep. The images match
    the oracle and the gather kernel's bit for bit."""
    from paper_1804_08197_amd import sg
    vol = gen.random_volume((40, 140, 130), 29, dtype=np.uint16)  # z, y, x
    tf = gen.tf_hot(a_start=30)
    h = gpu_volume([vol], 128, 1, [tf], [(0, 65535)], layout=layout)
    try:
        sg.sg_set_launch_config(h, {"kernel": 0, "tile": 16, "block": 32, "stage_bytes": 8192,
                                    "persistent": 0})
        sc = oracle_scene([vol], 128, 1, [tf], [(0, 65535)])
        c = np.array([65.0, 70.0, 20.0])
        views = [gen.view(gen.look_at(c + np.array([0.0, 0.0, 20.0 + d]), c, up=(0, 1, 0)), 8, 8,
                          0.02, tr) for d in (80.0, 100.0, 120.0) for tr in (1.0, 1.5)]
        st = _check(h, sc, views, {"ert": ERT, "tau": 1.0})
        print("wide rows:", st, flush=True)
        assert st["wide_slabs"] > 0 and st["slabs"] > 0
    finally:
        sg.sg_volume_destroy(h)
