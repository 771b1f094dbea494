"""Sort-last split on one GPU: the region of interest clips each ray to one
octant of the volume (the share one GPU would own); the eight octant
renders of a view, composited front over back per pixel in the order the
ray enters the octants (sg_composite_over, checked against the same
composite done here on the host with the oracle's rays), equal the whole
render (the oracle pins the same identity in FP64; here the renders are
FP32, so up to rounding).
"""
import numpy as np
import pytest

import gen
import oracle as O
from tests.helpers import gpu_volume

pytestmark = pytest.mark.gpu


def test_octant_renders_composite_to_the_whole_frame():
    import torch

    from paper_1804_08197_amd import sg
    assert torch.cuda.is_available(), "GPU tests need a GPU (no CPU fallback exists)"
    vol = gen.blobs128()
    tf = gen.tf_identity()
    tf[:, 3] *= 0.25
    h = gpu_volume([vol], 32, 3, [tf], [(0, 255)])
    try:
        # level-0 bricks only (32^3), so every node lies inside one octant;
        # no early termination, so every octant is integrated to its end
        params = {"step": 0.5, "ert": 2.0, "tau": 1.0, "lod": 0, "skip_empty": 1, "bias": 0}
        views = [gen.view(gen.look_at((-150.0, 190.0, 110.0), (64, 64, 64)), 64, 56, 0.55),
                 gen.view(gen.look_at((210.0, -40.0, -90.0), (60, 70, 64)), 57, 61, 0.5)]

        def render(p):
            outs = [torch.full((v["height"], v["width"], 4), float("nan"), device="cuda")
                    for v in views]
            sg.sg_render_views(h, views, p, outs)
            torch.cuda.synchronize()
            return outs

        whole_d = render(params)
        whole = [o.cpu().numpy().astype(np.float64) for o in whole_d]
        boxes, parts_d = [], []
        for o in range(8):
            lo = [64.0 * ((o >> a) & 1) for a in range(3)]
            hi = [x + 64.0 for x in lo]
            boxes.append((lo, hi))
            parts_d.append(render(dict(params, roi=tuple(lo) + tuple(hi))))
        parts = [[x.cpu().numpy().astype(np.float64) for x in p] for p in parts_d]
        for i, v in enumerate(views):
            # on the device, through the C-ABI
            dev = torch.full((v["height"], v["width"], 4), float("nan"), device="cuda")
            sg.sg_composite_over(v, [p[i] for p in parts_d], [lo + hi for lo, hi in boxes], dev)
            torch.cuda.synchronize()
            dev = dev.cpu().numpy().astype(np.float64)
            err_dev = np.abs(dev - whole[i]).max()
            assert err_dev <= 2e-5, "view %d: device composite differs by %g" % (i, err_dev)
            comp = np.zeros_like(whole[i])
            for y in range(v["height"]):
                for x in range(v["width"]):
                    e, d = O.ray(v, x, y)
                    order = []
                    for o, (lo, hi) in enumerate(boxes):
                        hit, t0, t1 = O.box_interval(e, d, lo, hi)
                        if hit and t0 < t1:
                            order.append((t0, o))
                    c, T = np.zeros(4), 1.0
                    for _, o in sorted(order):
                        px = parts[o][i][y, x]
                        c += T * px
                        T *= 1.0 - px[3]
                    comp[y, x] = c
            err = np.abs(comp - whole[i]).max()
            assert err <= 2e-5, "view %d: composite differs by %g" % (i, err)
            assert np.abs(comp - dev).max() <= 2e-6
            assert whole[i][..., 3].max() > 0.3  # the rays do cross content
    finally:
        sg.sg_volume_destroy(h)


def test_slab_parts_with_a_lens_view_composite_to_the_whole_frame():
    """Three slabs of unequal width along x, a wrapped-space (lens) view and
    a view from inside the volume's bounding planes: the composite follows
    the renderer's own rays (lens included) and ignores parts a ray misses."""
    import torch

    from paper_1804_08197_amd import sg
    vol = gen.blobs128()
    tf = gen.tf_identity()
    tf[:, 3] *= 0.3
    h = gpu_volume([vol], 32, 3, [tf], [(0, 255)])
    try:
        params = {"step": 0.5, "ert": 2.0, "tau": 1.0, "lod": 0, "skip_empty": 1, "bias": 0}
        lens_view = dict(gen.view(gen.look_at((64.0, -170.0, 90.0), (64, 64, 64)), 48, 40, 0.6),
                         lens=(0.2, 0.1, 0.05, -0.03))
        side_view = gen.view(gen.look_at((64.0, 64.0, 300.0), (64, 64, 0), up=(0, 1, 0)), 33, 29,
                             0.4)
        boxes = [(0, 0, 0, 32, 128, 128), (32, 0, 0, 96, 128, 128), (96, 0, 0, 128, 128, 128)]
        for v in (lens_view, side_view):
            def render(p):
                o = torch.full((v["height"], v["width"], 4), float("nan"), device="cuda")
                sg.sg_render_views(h, [v], p, [o])
                return o
            whole = render(params)
            parts = [render(dict(params, roi=b)) for b in boxes]
            comp = torch.full_like(whole, float("nan"))
            sg.sg_composite_over(v, parts, boxes, comp)
            torch.cuda.synchronize()
            err = float((comp - whole).abs().max())
            assert err <= 2e-5, err
            assert float(whole[..., 3].max()) > 0.3
    finally:
        sg.sg_volume_destroy(h)
