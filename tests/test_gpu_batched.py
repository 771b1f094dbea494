"""Batched uneven views: launch configurations, graphs and the autotuner.

Every launch configuration (kernel flavour, workgroup tile, XCD block, LDS
staging size, direct or persistent grid) must render the same image bit for
bit, so parity with the oracle carries over from the default configuration
(checked here on sampled pixels too). Render graphs replay equal to eager
renders, across re-posing and transfer-function edits; the autotuner's
choice is one of those configurations.
"""
import itertools
import math
import sys

import numpy as np
import pytest

import gen
from tests.helpers import ERT, TOL, bracket_error, gpu_volume, oracle_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU (no CPU fallback exists)"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def uneven_views(seed=1004, n=7):
    vs = gen.orbit_views((64, 64, 64), (1.5 * 221.7, 4 * 221.7), n, seed, (96, 700), (96, 700),
                         tan_top=math.tan(math.radians(30)))
    # degenerate sizes: a single pixel and a ragged sliver
    vs.append(dict(gen.view(gen.look_at((-300.0, 90.0, 40.0), (64, 64, 64)), 1, 1, 0.2)))
    vs.append(dict(gen.view(gen.look_at((40.0, -350.0, 120.0), (64, 64, 64)), 9, 203, 0.6)))
    return vs


@pytest.fixture(scope="module")
def blobs():
    from paper_1804_08197_amd import sg
    vol = gen.blobs128()
    tf = gen.tf_identity()
    h = gpu_volume([vol], 32, 3, [tf], [(0, 255)])
    yield h, vol, tf
    sg.sg_volume_destroy(h)


def render(h, views, params):
    import torch

    from paper_1804_08197_amd import sg
    outs = [torch.full((v["height"], v["width"], 4), float("nan"), device="cuda") for v in views]
    sg.sg_render_views(h, views, params, outs)
    torch.cuda.synchronize()
    return outs


CONFIGS = [dict(kernel=k, tile=t, block=b, stage_bytes=s, persistent=p)
           for k, t, b, s, p in itertools.product((0, 1), (8, 16, 32), (32, 64, 128),
                                                  (4096, 16384), (0, 1))
           if b >= t and not (k == 1 and s == 16384)]


def test_every_launch_config_renders_the_same_image(blobs):
    import torch

    from paper_1804_08197_amd import sg
    h, _, _ = blobs
    views = uneven_views()
    params = {"ert": ERT, "tau": 1.0}
    sg.sg_set_launch_config(h, None)
    ref = render(h, views, params)
    ref_stats = sg.sg_render_views_stats(h, views, params,
                                         [torch.empty_like(o) for o in ref])
    log("%d configurations, %d views" % (len(CONFIGS), len(views)))
    try:
        for cfg in CONFIGS:
            sg.sg_set_launch_config(h, cfg)
            assert sg.sg_get_launch_config(h) == cfg
            got = render(h, views, params)
            for i, (a, b) in enumerate(zip(ref, got)):
                assert torch.equal(a, b), (cfg, i)
        # instrumented persistent render counts the same samples
        sg.sg_set_launch_config(h, dict(kernel=0, tile=32, block=64, stage_bytes=8192,
                                        persistent=1))
        st = sg.sg_render_views_stats(h, views, params, [torch.empty_like(o) for o in ref])
        assert st["total_samples"] == ref_stats["total_samples"]
        assert st["microblocks"] == ref_stats["microblocks"]
    finally:
        sg.sg_set_launch_config(h, None)


def test_persistent_grid_parity_on_sampled_pixels(blobs):
    from paper_1804_08197_amd import sg
    h, vol, tf = blobs
    views = uneven_views(seed=2005, n=4)
    params = {"ert": ERT, "tau": 1.0}
    sg.sg_set_launch_config(h, dict(kernel=0, tile=16, block=128, stage_bytes=8192,
                                    persistent=1))
    try:
        got = render(h, views, params)
    finally:
        sg.sg_set_launch_config(h, None)
    sc = oracle_scene([vol], 32, 3, [tf], [(0, 255)])
    rng = np.random.default_rng(7)
    for i, v in enumerate(views):
        n = min(300, v["width"] * v["height"])
        pix = np.stack([rng.integers(0, v["width"], n), rng.integers(0, v["height"], n)], 1)
        refs = [sc.render(v, dict(params, ert=e), pixels=pix) for e in (ERT, ERT - 1e-5,
                                                                        ERT + 1e-5)]
        g = got[i].cpu().numpy().astype(np.float64)[pix[:, 1], pix[:, 0]]
        best, _ = bracket_error(g, refs)
        assert best.max() <= TOL


@pytest.mark.parametrize("persistent", [0, 1])
def test_graph_replays_on_microblock_slots(persistent):
    """A render graph over a volume with micro-block slots replays the eager
    render of the same volume, and that of the same data in linear slots."""
    import torch

    from paper_1804_08197_amd import sg
    vol = gen.random_volume((44, 52, 60), 123, dtype=np.uint16)
    tf = gen.tf_hot(a_start=30)
    hl = gpu_volume([vol], 16, 3, [tf], [(0, 65535)], layout=sg.SG_LAYOUT_LINEAR)
    hm = gpu_volume([vol], 16, 3, [tf], [(0, 65535)], layout=sg.SG_LAYOUT_MICROBLOCK)
    try:
        c = np.array([30.0, 26.0, 22.0])
        views = gen.stereo(c + np.array([-80.0, 50.0, 40.0]), c, 6.0, 72, 64, 0.55, 0.5)
        params = {"ert": ERT, "tau": 1.0}
        for h in (hl, hm):
            sg.sg_set_launch_config(h, dict(kernel=0, tile=16, block=32, stage_bytes=8192,
                                            persistent=persistent))
        ref = render(hl, views, params)
        outs = [torch.zeros(v["height"], v["width"], 4, device="cuda") for v in views]
        g = sg.RenderGraph(hm, views, params, outs)
        try:
            for rep in range(3):
                for o in outs:
                    o.fill_(float("nan"))
                g.launch()
                torch.cuda.synchronize()
                eager = render(hm, views, params)
                for a, b, e in zip(ref, outs, eager):
                    assert torch.equal(a, b), rep
                    assert torch.equal(a, e), rep
        finally:
            g.destroy()
    finally:
        sg.sg_volume_destroy(hl)
        sg.sg_volume_destroy(hm)


@pytest.mark.parametrize("persistent", [0, 1])
def test_graph_replays_equal_eager_renders(blobs, persistent):
    import torch

    from paper_1804_08197_amd import sg
    h, _, tf = blobs
    views = uneven_views(n=3)
    params = {"ert": ERT, "tau": 1.0}
    sg.sg_set_launch_config(h, dict(kernel=0, tile=16, block=64, stage_bytes=8192,
                                    persistent=persistent))
    try:
        outs = [torch.zeros(v["height"], v["width"], 4, device="cuda") for v in views]
        g = sg.RenderGraph(h, views, params, outs)
        try:
            ref = render(h, views, params)
            for rep in range(3):
                for o in outs:
                    o.fill_(float("nan"))
                g.launch()
                torch.cuda.synchronize()
                for a, b in zip(ref, outs):
                    assert torch.equal(a, b), rep
                # eager work on the same volume between replays
                render(h, uneven_views(seed=77, n=2), params)
            # re-posed views
            moved = uneven_views(seed=99, n=3)
            moved = [dict(m, width=v["width"], height=v["height"]) for m, v in zip(moved, views)]
            g.set_views(moved)
            g.launch()
            torch.cuda.synchronize()
            ref2 = render(h, moved, params)
            for a, b in zip(ref2, outs):
                assert torch.equal(a, b)
            # new table contents (same size and domain) are picked up
            sg.sg_set_transfer_function(h, 0, np.ascontiguousarray(tf[::-1]), 0, 255)
            g.launch()
            torch.cuda.synchronize()
            ref3 = render(h, moved, params)
            for a, b in zip(ref3, outs):
                assert torch.equal(a, b)
            # a different table size invalidates the graph
            sg.sg_set_transfer_function(h, 0, gen.tf_identity(128), 0, 255)
            with pytest.raises(sg.SgError) as ex:
                g.launch()
            assert ex.value.status == sg.SG_ERR_STATE
        finally:
            g.destroy()
            sg.sg_set_transfer_function(h, 0, tf, 0, 255)
    finally:
        sg.sg_set_launch_config(h, None)


def test_autotune_picks_a_valid_config_with_identical_output(blobs):
    import torch

    from paper_1804_08197_amd import sg
    h, _, _ = blobs
    views = uneven_views(n=5)
    params = {"ert": ERT, "tau": 1.0}
    sg.sg_set_launch_config(h, None)
    ref = render(h, views, params)
    outs = [torch.empty_like(o) for o in ref]
    try:
        cfg, ms = sg.sg_autotune(h, views, params, outs, repeats=1)
        log("autotuned %s: %.3f ms" % (cfg, ms))
        assert sg.sg_get_launch_config(h) == cfg
        assert ms > 0
        got = render(h, views, params)
        for a, b in zip(ref, got):
            assert torch.equal(a, b)
    finally:
        sg.sg_set_launch_config(h, None)


def test_bad_launch_configs_are_rejected(blobs):
    from paper_1804_08197_amd import sg
    h, _, _ = blobs
    for bad in (dict(tile=24), dict(block=16), dict(tile=32, block=32, stage_bytes=100),
                dict(persistent=2), dict(kernel=3), dict(tile=64, block=64)):
        with pytest.raises(sg.SgError) as ex:
            sg.sg_set_launch_config(h, bad)
        assert ex.value.status == sg.SG_ERR_INVALID_ARG
    assert sg.sg_get_launch_config(h) == sg.DEFAULT_LAUNCH


@pytest.mark.parametrize("launch", [None, (1, 8, 32, 8192, 0), (0, 16, 64, 8192, 1)])
def test_render_if_follows_the_device_flag(blobs, launch):
    """sg_render_views_if: a nonzero device flag renders exactly what
    sg_render_views renders; a zero flag leaves the outputs untouched."""
    import torch

    from paper_1804_08197_amd import sg
    h, _, _ = blobs
    try:
        if launch is not None:
            sg.sg_set_launch_config(h, dict(zip(sg.LAUNCH_FIELDS, launch)))
        vs = uneven_views(1010, 4)
        p = {"ert": ERT, "tau": 1.0}
        ref = render(h, vs, p)
        for on in (1, 0, 1):
            flag = torch.tensor([on], dtype=torch.int32, device="cuda")
            outs = [torch.full((v["height"], v["width"], 4), float("nan"), device="cuda")
                    for v in vs]
            sg.sg_render_views_if(h, vs, p, outs, flag)
            torch.cuda.synchronize()
            for o, r in zip(outs, ref):
                if on:
                    assert torch.equal(o, r)
                else:
                    assert torch.isnan(o).all()
        with pytest.raises(ValueError):
            sg.sg_render_views_if(h, vs, p, ref, None)
    finally:
        sg.sg_set_launch_config(h, None)


def test_small_calls_carry_their_views_inline_with_the_same_images(blobs):
    """Up to four views travel in the cut-map kernel's arguments, larger
    calls through a staged device table: both give the same images, and
    alternating the two routes leaves no stale view records behind."""
    h, vol, tf = blobs
    views = uneven_views(n=7)
    params = {"step": 0.5, "ert": ERT, "tau": 1.0, "lod": 1, "skip_empty": 1, "bias": 0}
    big = render(h, views, params)  # 9 views: staged table
    for n in (1, 2, 4):
        small = render(h, views[:n], params)  # inline records
        for i in range(n):
            assert np.array_equal(small[i].cpu().numpy(), big[i].cpu().numpy()), (n, i)
    # a staged call after inline ones, then an inline call of other views
    again = render(h, views, params)
    for i in range(len(views)):
        assert np.array_equal(again[i].cpu().numpy(), big[i].cpu().numpy()), i
    tail = render(h, views[5:9], params)
    for i in range(4):
        assert np.array_equal(tail[i].cpu().numpy(), big[5 + i].cpu().numpy()), i


@pytest.mark.parametrize("launch", [None, (1, 8, 32, 8192, 0), (0, 16, 64, 8192, 1),
                                    (1, 32, 64, 8192, 1)])
def test_content_mask_marks_the_blocks_with_content(blobs, launch):
    """tile_any: one byte per 8x8-pixel block, 1 exactly where a pixel of the
    block has a nonzero RGBA or (with depth output) a finite depth, in every
    launch configuration; ragged views included."""
    import torch

    from paper_1804_08197_amd import sg
    h, vol, tf = blobs
    views = uneven_views(n=5)
    params = {"step": 0.5, "ert": ERT, "tau": 1.0, "lod": 1, "skip_empty": 1, "bias": 0}
    sg.sg_set_launch_config(h, None if launch is None else
                            dict(zip(sg.LAUNCH_FIELDS, launch)))
    try:
        for with_depth in (False, True):
            masks = [torch.full(((v["height"] + 7) // 8, (v["width"] + 7) // 8), 7,
                                dtype=torch.uint8, device="cuda") for v in views]
            vs = [dict(v, tile_any=m) for v, m in zip(views, masks)]
            outs = [torch.full((v["height"], v["width"], 4), float("nan"), device="cuda")
                    for v in views]
            deps = [torch.full((v["height"], v["width"]), float("nan"), device="cuda")
                    for v in views] if with_depth else None
            sg.sg_render_views(h, vs, params, outs, deps)
            torch.cuda.synchronize()
            for i, v in enumerate(views):
                nz = (outs[i] != 0).any(-1)
                if with_depth:
                    nz |= torch.isfinite(deps[i])
                H8, W8 = masks[i].shape
                pad = torch.zeros(H8 * 8, W8 * 8, dtype=torch.bool, device="cuda")
                pad[:v["height"], :v["width"]] = nz
                want = pad.view(H8, 8, W8, 8).any(3).any(1).to(torch.uint8)
                assert torch.equal(masks[i], want), (launch, with_depth, i)
        # a nonzero background gives every block content
        v = views[0]
        m = torch.zeros(((v["height"] + 7) // 8, (v["width"] + 7) // 8), dtype=torch.uint8,
                        device="cuda")
        o = torch.empty(v["height"], v["width"], 4, device="cuda")
        sg.sg_render_views(h, [dict(v, tile_any=m)], dict(params, bg=(0, 0, 0.1, 1)),
                           [o])
        torch.cuda.synchronize()
        assert bool((m == 1).all())
    finally:
        sg.sg_set_launch_config(h, None)
