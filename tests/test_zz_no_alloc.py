"""The allocation-free render (sg_render_views_noalloc, for callers that
cannot allocate) against sg_render_views through the C-ABI: two calls in a
row, the second on a smaller input (another volume, fewer and smaller
views), each bit-identical to the allocating entry point, in the direct
and the persistent launch; and its argument and state errors."""
import numpy as np
import pytest

import gen
from helpers import gpu_volume

pytestmark = pytest.mark.gpu


def _render(fn, h, views, params):
    import torch
    out = [torch.full((v["height"], v["width"], 4), float("nan"), device="cuda")
           for v in views]
    dep = [torch.full((v["height"], v["width"]), float("nan"), device="cuda") for v in views]
    fn(h, views, params, out, dep)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out], [d.cpu().numpy() for d in dep]


def _case(shape, dtype, brick, levels, views, seed, launch=None, layout=0):
    from paper_1804_08197_amd import sg
    print("noalloc case", shape, dtype.__name__, brick, levels, len(views), launch, layout,
          flush=True)
    vol = gen.random_volume(shape, seed, dtype=dtype)
    dom = (0, 255) if dtype == np.uint8 else (0, 65535)
    tf = gen.tf_hot(a_start=30)
    h = gpu_volume([vol], brick, levels, [tf], [dom], layout=layout)
    try:
        if launch is not None:
            sg.sg_set_launch_config(h, launch)
        sg.sg_volume_commit(h)
        params = {"ert": 0.99, "tau": 1.0}
        want = _render(sg.sg_render_views, h, views, params)
        got = _render(sg.sg_render_views_noalloc, h, views, params)
        for a, b in zip(got[0], want[0]):
            assert np.isfinite(a).all() and np.array_equal(a, b)
        for a, b in zip(got[1], want[1]):  # depth: +inf where no sample reached 0.5
            assert not np.isnan(a).any() and np.array_equal(a, b)
        assert any(np.any(r[..., 3] > 0) for r in got[0]), "want some content"
    finally:
        sg.sg_volume_destroy(h)


@pytest.mark.parametrize("layout", [0, 1], ids=["linear", "microblock"])
@pytest.mark.parametrize("launch", [None, {"kernel": 0, "tile": 8, "block": 32,
                                           "stage_bytes": 8192, "persistent": 1}])
def test_noalloc_render_equals_sg_render_views_twice(launch, layout):
    big = (40, 48, 56)  # z, y, x
    c = np.array([28.0, 24.0, 20.0])
    stereo = gen.stereo(c + np.array([-70.0, 45.0, 35.0]), c, 6.0, 96, 80, 0.55, 0.5)
    _case(big, np.uint16, 8, 3, stereo, 11, launch, layout)
    small = (22, 26, 30)
    c2 = np.array([15.0, 13.0, 11.0])
    mono = [gen.view(gen.look_at(c2 + np.array([30.0, -25.0, 20.0]), c2), 40, 30, 0.6)]
    _case(small, np.uint8, 4, 2, mono, 12, launch, layout)


def test_noalloc_render_rejects_what_it_cannot_hold():
    import torch

    from paper_1804_08197_amd import sg
    vol = gen.random_volume((20, 20, 20), 3, dtype=np.uint8)
    h = gpu_volume([vol], 4, 2, [gen.tf_hot(a_start=30)], [(0, 255)])
    try:
        c = np.array([10.0, 10.0, 10.0])
        v = gen.view(gen.look_at(c + np.array([40.0, 5.0, 5.0]), c), 16, 16, 0.5)
        out = [torch.empty(16, 16, 4, device="cuda") for _ in range(5)]
        # not committed yet (uploads and the table are pending)
        with pytest.raises(sg.SgError) as ex:
            sg.sg_render_views_noalloc(h, [v], {}, out[:1])
        assert ex.value.status == sg.SG_ERR_STATE
        sg.sg_volume_commit(h)
        with pytest.raises(sg.SgError) as ex:
            sg.sg_render_views_noalloc(h, [v] * 5, {}, out)
        assert ex.value.status == sg.SG_ERR_INVALID_ARG
        sg.sg_render_views_noalloc(h, [v], {}, out[:1])
        torch.cuda.synchronize()
    finally:
        sg.sg_volume_destroy(h)
    # cut maps beyond the scratch: 4 views of a 64^3-cell brick grid (4 MiB)
    h = sg.sg_volume_create((256, 256, 256), dtype=sg.SG_U8, brick=4, levels=1)
    try:
        sg.sg_set_transfer_function(h, 0, gen.tf_hot(a_start=30), 0, 255)
        sg.sg_volume_commit(h)
        c = np.array([128.0, 128.0, 128.0])
        v = gen.view(gen.look_at(c + np.array([500.0, 5.0, 5.0]), c), 8, 8, 0.5)
        out = [torch.empty(8, 8, 4, device="cuda") for _ in range(4)]
        with pytest.raises(sg.SgError) as ex:
            sg.sg_render_views_noalloc(h, [v] * 4, {}, out)
        assert ex.value.status == sg.SG_ERR_INVALID_ARG
        assert "scratch" in sg.sg_last_error()
    finally:
        sg.sg_volume_destroy(h)
