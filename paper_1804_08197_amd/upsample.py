"""The learned-upsampler render path and its training loop.

Per frame (Sec 5.3: cast fewer rays, then resample): every eye is ray cast
at half resolution one pyramid level coarser, with first-hit depth; the
upsampler network (``upsampler.Upsampler``, HIP kernels on the matrix
cores) predicts the full-resolution frame and its squared error; when the
predicted PSNR of the frame is below a threshold the frame is ray cast at
full resolution instead (the fallback).

Training pairs are made by the ray caster itself: a random pose and a random
window of the full-resolution frame, rendered at full resolution on level 0
(the target) and at half resolution on level 1 (the input, with depth); the
window is an off-centre frustum, so only its rays are cast.

Orchestration only: every render, network pass and update runs in libsg.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import sg
from . import upsampler as up

DEPTH_ALPHA = 0.5


def render_params(base_params, lod):
    """(full-resolution, half-resolution) render parameters. Without LOD the
    target samples level 0 and the input level 1 everywhere; with the
    screen-space LOD both use it, and the half-resolution render, whose
    pixels span twice the angle, lands one level coarser on its own."""
    if lod:
        return (dict(base_params, lod=1, bias=0),
                dict(base_params, lod=1, bias=0, depth_alpha=DEPTH_ALPHA))
    return (dict(base_params, lod=0, bias=0),
            dict(base_params, lod=0, bias=1, depth_alpha=DEPTH_ALPHA))


def crop_view(view, x0, y0, w, h, scale=1):
    """The view restricted to full-resolution pixels [x0, x0+w) x [y0, y0+h)
    of `view`, rendered at w / scale x h / scale pixels."""
    W, H = view["width"], view["height"]
    sx = (view["tan_right"] - view["tan_left"]) / W
    sy = (view["tan_top"] - view["tan_bottom"]) / H
    return {"cam_to_world": view["cam_to_world"],
            "tan_left": view["tan_left"] + x0 * sx, "tan_right": view["tan_left"] + (x0 + w) * sx,
            "tan_top": view["tan_top"] - y0 * sy, "tan_bottom": view["tan_top"] - (y0 + h) * sy,
            "width": w // scale, "height": h // scale}


def half_view(view):
    return dict(view, width=view["width"] // 2, height=view["height"] // 2)


class Trainer:
    """Trains an upsampler on pairs rendered from a volume with >= 2 levels."""

    def __init__(self, vol, model: "up.Upsampler", depth_scale: float, base_params: dict,
                 crop=256, batch=16, lod=False):
        import torch
        if int(crop) < 2 or int(crop) % 2:
            raise ValueError("the crop must be even: the network upsamples by exactly 2")
        self.vol, self.model = vol, model
        self.depth_scale = float(depth_scale)
        self.p_full, self.p_half = render_params(base_params, lod)
        self.crop, self.batch = int(crop), int(batch)
        c2 = self.crop // 2
        self.rgba_lo = torch.empty(batch, c2, c2, 4, device="cuda")
        self.depth_lo = torch.empty(batch, c2, c2, device="cuda")
        self.target = torch.empty(batch, self.crop, self.crop, 4, device="cuda")

    def make_batch(self, rng, poses):
        """Render one batch of pairs: random poses (full-resolution view
        dicts) and random crop windows."""
        vf, vh = [], []
        for i in range(self.batch):
            v = poses[int(rng.integers(len(poses)))]
            if v["width"] < self.crop or v["height"] < self.crop:
                raise ValueError("a training pose is smaller than the crop")
            x0 = 2 * int(rng.integers(0, (v["width"] - self.crop) // 2 + 1))
            y0 = 2 * int(rng.integers(0, (v["height"] - self.crop) // 2 + 1))
            vf.append(crop_view(v, x0, y0, self.crop, self.crop))
            vh.append(crop_view(v, x0, y0, self.crop, self.crop, scale=2))
        sg.sg_render_views(self.vol, vf, self.p_full, list(self.target))
        sg.sg_render_views(self.vol, vh, self.p_half, list(self.rgba_lo), list(self.depth_lo))

    def step(self, rng, poses, lr, err_weight=1.0, want_loss=False):
        self.make_batch(rng, poses)
        return self.model.train_step(self.rgba_lo, self.depth_lo, self.depth_scale, self.target,
                                     lr, err_weight, want_loss=want_loss)


class UpsampledPath:
    """Frames through the upsampler, with the full-resolution fallback."""

    def __init__(self, vol, model: "up.Upsampler", depth_scale: float, base_params: dict,
                 width: int, height: int, n_views: int = 2, threshold_db: float = 40.0,
                 lod=False, launch_half=None, launch_full=None):
        """launch_half / launch_full: None, or the launch configuration
        (sg_set_launch_config) for the half-resolution render and for the
        full-resolution fallback render; the images are the same under any
        configuration, only their speed differs."""
        import torch
        if int(width) < 2 or int(height) < 2 or int(width) % 2 or int(height) % 2:
            raise ValueError("width and height must be even: the network writes rows of "
                             "2 x (width // 2) pixels")
        self.vol, self.model = vol, model
        self.depth_scale = float(depth_scale)
        self.p_full, self.p_half = render_params(base_params, lod)
        self.threshold_db = float(threshold_db)
        w2, h2 = width // 2, height // 2
        self.rgba_lo = torch.empty(n_views, h2, w2, 4, device="cuda")
        self.depth_lo = torch.empty(n_views, h2, w2, device="cuda")
        self.out = torch.empty(n_views, height, width, 4, device="cuda")
        # the half-resolution render's content mask (tile_any), which tells
        # the network which tiles hold anything but background
        self.content = torch.empty(n_views, (h2 + 7) // 8, (w2 + 7) // 8, dtype=torch.uint8,
                                   device="cuda")
        self.size = (int(width), int(height), int(n_views))
        self.launch_half, self.launch_full = launch_half, launch_full
        self._structs = None

    def _launch(self, cfg):
        if cfg is not None:
            sg.sg_set_launch_config(self.vol, cfg)

    def _half_views(self, views):
        return [dict(half_view(v), tile_any=self.content[i]) for i, v in enumerate(views)]

    def _check(self, views):
        w, h, n = self.size
        if len(views) != n or any(v["width"] != w or v["height"] != h for v in views):
            raise ValueError("this path renders %d views of %d x %d pixels" % (n, w, h))

    def predicted_psnr(self, views):
        """Half-resolution render and network pass; returns the predicted
        PSNR of the frame (all views together)."""
        self._check(views)
        self._launch(self.launch_half)
        sg.sg_render_views(self.vol, self._half_views(views), self.p_half,
                           list(self.rgba_lo), list(self.depth_lo))
        mse = self.model.forward(self.rgba_lo, self.depth_lo, self.depth_scale, self.out,
                                 predict=True, content=self.content)
        m = float(np.mean(mse))
        return math.inf if m <= 0 else 10.0 * math.log10(1.0 / m)

    def render(self, views):
        """One frame: the upsampled image, or the full-resolution render when
        the prediction falls below the threshold. Returns (images, fell_back)."""
        fell_back = self.predicted_psnr(views) < self.threshold_db
        if fell_back:
            self._launch(self.launch_full)
            sg.sg_render_views(self.vol, views, self.p_full, list(self.out))
        return self.out, fell_back

    def render_device(self, views, flag):
        """The same frame with the decision taken on the device, without a
        host round trip: flag (one-element int32 device tensor) receives 1
        when the frame fell back. Asynchronous; returns the images."""
        self._check(views)
        key = (id(self.launch_half), id(self.launch_full))
        if self._structs is None or self._structs[0] != key:
            # built once: per frame only the views are packed, once for
            # both renders (the half-resolution ones are a patched copy)
            lh = None if self.launch_half is None else sg.launch_config_struct(self.launch_half)
            lf = None if self.launch_full is None else sg.launch_config_struct(self.launch_full)
            self._structs = (key, sg.make_params(self.p_half), sg.make_params(self.p_full),
                             sg.pointer_array(list(self.rgba_lo)),
                             sg.pointer_array(list(self.depth_lo)),
                             sg.pointer_array(list(self.out)), lh, lf,
                             [self.content[i].data_ptr() for i in range(self.size[2])])
        _, ph, pf, lo, dlo, out, lh, lf, masks = self._structs
        full = sg.views_array(views)
        half = (sg.sg_view * len(full))()
        C.memmove(half, full, C.sizeof(full))
        for i in range(len(full)):
            half[i].width = full[i].width // 2
            half[i].height = full[i].height // 2
            half[i].tile_any = masks[i]
        if lh is not None:
            sg.sg_set_launch_config(self.vol, lh)
        sg.sg_render_views(self.vol, half, ph, lo, dlo)
        self.model.forward_flag(self.rgba_lo, self.depth_lo, self.depth_scale, self.out,
                                self.threshold_db, flag, content=self.content)
        if lf is not None:
            sg.sg_set_launch_config(self.vol, lf)
        sg.sg_render_views_if(self.vol, full, pf, out, flag)
        return self.out


def init_params(rng, scale=0.5):
    """He-style random initialisation; the last layer starts small so the
    network begins as bilinear upsampling."""
    out = []
    for i, (ci, co) in enumerate(up.LAYERS):
        fan = 9 * (5 if ci == 8 else ci)
        w = rng.normal(size=(9, ci, co)) * math.sqrt(2.0 / fan) * (0.1 if i == 3 else scale)
        if ci == 8:
            w[:, 5:, :] = 0.0
        out.append((w, np.zeros(co)))
    return up.pack(out)
