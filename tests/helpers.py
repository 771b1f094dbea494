"""Shared helpers of the GPU tests: build a volume through the C-ABI, render,
and compare with the oracle under the early-termination bracket."""
from __future__ import annotations

import numpy as np

ERT = 0.99
BRACKET = 1e-5  # early-termination threshold bracket (several correct results)
TOL = 1e-4      # max abs RGBA error against the oracle
# pool slot layouts (sg_layout), as test parameters
LAYOUTS = [0, 1]
LAYOUT_IDS = ["linear", "microblock"]


def as_f64_tf(tf):
    """The table the GPU receives is float32; the oracle uses the same values."""
    return np.asarray(tf, dtype=np.float32).astype(np.float64)


def gpu_volume(channels, brick, levels, tfs, domains, device_upload=True, layout=0):
    import torch

    from paper_1804_08197_amd import sg, upload_volume
    vol0 = channels[0]
    nz, ny, nx = vol0.shape
    dtype = sg.SG_U8 if vol0.dtype == np.uint8 else sg.SG_U16
    h = sg.sg_volume_create((nx, ny, nz), channels=len(channels), dtype=dtype, brick=brick,
                            levels=levels, layout=layout)
    for c, v in enumerate(channels):
        data = torch.from_numpy(v).cuda() if device_upload else v
        upload_volume(h, data, brick, channel=c)
    for c, (tf, dom) in enumerate(zip(tfs, domains)):
        sg.sg_set_transfer_function(h, c, tf, dom[0], dom[1])
    return h


def oracle_scene(channels, brick, levels, tfs, domains):
    import oracle
    return oracle.Scene(channels, brick, levels, [as_f64_tf(t) for t in tfs], domains)


def render_gpu(h, views, params, depth=False, samples=False):
    import torch

    from paper_1804_08197_amd import sg
    rgba = [torch.full((v["height"], v["width"], 4), float("nan"), device="cuda") for v in views]
    dep = [torch.full((v["height"], v["width"]), float("nan"), device="cuda") for v in views] \
        if depth else None
    out = {}
    if samples:
        smp = [torch.full((v["height"], v["width"]), -1, dtype=torch.int32, device="cuda")
               for v in views]
        out["stats"] = sg.sg_render_views_stats(h, views, params, rgba, dep, smp)
        out["nsamp"] = [s.cpu().numpy() for s in smp]
    else:
        sg.sg_render_views(h, views, params, rgba, dep)
    torch.cuda.synchronize()
    out["rgba"] = [r.cpu().numpy().astype(np.float64) for r in rgba]
    if depth:
        out["depth"] = [d.cpu().numpy().astype(np.float64) for d in dep]
    return out


def oracle_bracket(scene, view, params, pixels=None, **kw):
    """Oracle renders at the termination threshold and +-BRACKET."""
    e = params.get("ert", ERT)
    return [scene.render(view, dict(params, ert=x), pixels=pixels, **kw)
            for x in (e, e - BRACKET, e + BRACKET)]


def bracket_error(gpu_rgba, refs):
    """Per pixel, the smallest max-abs error against any bracketed render;
    also the number of pixels that needed a bracketed render."""
    errs = np.stack([np.abs(gpu_rgba - r["rgba"]).max(axis=-1) for r in refs])
    best = errs.min(axis=0)
    needed = int(((errs[0] > TOL) & (best <= TOL)).sum())
    return best, needed
