"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

RGBA within 1e-4 per pixel (with the early-termination bracket), LOD cuts
and empty flags bit-exact, skip / stereo / repeat invariants bit-identical,
and the two pool slot layouts (linear rows, 4^3 micro-blocks) render the
same images bit for bit.
"""
import math
import sys

import numpy as np
import pytest

import gen
from tests.helpers import (ERT, LAYOUT_IDS, LAYOUTS, TOL, bracket_error, gpu_volume,
                           oracle_bracket, oracle_scene, render_gpu)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU (no CPU fallback exists)"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check_views(h, sc, views, params, depth=False, samples=False, max_bracket_frac=0.01):
    g = render_gpu(h, views, params, depth=depth, samples=samples)
    worst = 0.0
    for i, v in enumerate(views):
        refs = oracle_bracket(sc, v, params, depth=depth, count=samples)
        best, needed = bracket_error(g["rgba"][i], refs)
        worst = max(worst, float(best.max()))
        assert best.max() <= TOL, "view %d: max abs err %g at %s" % (
            i, best.max(), np.unravel_index(best.argmax(), best.shape))
        assert needed <= max_bracket_frac * best.size + 2
        if samples:
            ns = g["nsamp"][i]
            ok = np.zeros(ns.shape, bool)
            for r in refs:
                ok |= ns == r["nsamp"]
            assert (~ok).sum() <= max(2, 1e-3 * ns.size), "sample counts differ at %d px" % (
                (~ok).sum())
        if depth:
            dg = g["depth"][i]
            okd = np.zeros(dg.shape, bool)
            for da in (0.5, 0.5 - 1e-5, 0.5 + 1e-5):
                r = sc.render(v, dict(params, depth_alpha=da), depth=True)["depth"]
                both_inf = np.isinf(dg) & np.isinf(r)
                fin = np.isfinite(dg) & np.isfinite(r)
                diff = np.abs(np.where(fin, dg, 0.0) - np.where(fin, r, 0.0))
                close = fin & (diff <= 1e-5 * np.abs(np.where(fin, r, 0.0)) + 1e-4)
                okd |= both_inf | close
            assert (~okd).sum() <= max(2, 1e-3 * dg.size)
    return g, worst


# ------------------------------------------------------------- blobs 128^3
@pytest.mark.parametrize("brick,levels", [(128, 1), (64, 1), (32, 2)])
def test_blobs128_full_image_parity(brick, levels):
    log("blobs128 parity brick=%d levels=%d" % (brick, levels))
    vol = gen.blobs128()
    tf = gen.tf_identity()
    h = gpu_volume([vol], brick, levels, [tf], [(0, 255)])
    from paper_1804_08197_amd import sg
    try:
        sc = oracle_scene([vol], brick, levels, [tf], [(0, 255)])
        v = gen.blobs128_view()
        params = {"ert": ERT, "lod": 0, "bias": 0, "step": 0.5}
        g, worst = check_views(h, sc, [v], params, samples=True)
        log("  worst err %.3g samples %d" % (worst, g["stats"]["total_samples"]))
        ref = sc.render(v, params, count=True, microblocks=True)
        assert g["stats"]["total_samples"] == pytest.approx(ref["total_samples"], rel=1e-3)
        mb = sum(int(m.sum()) for m in ref["microblocks"])
        assert g["stats"]["microblocks"] == pytest.approx(mb, rel=5e-3)
    finally:
        sg.sg_volume_destroy(h)


# ------------------------------------------------------ bricked LOD parity
@pytest.mark.parametrize("layout", LAYOUTS, ids=LAYOUT_IDS)
@pytest.mark.parametrize("dtype,shape,brick,levels,seed", [
    (np.uint16, (29, 38, 45), 8, 4, 1),
    (np.uint8, (40, 40, 40), 16, 3, 2),
    (np.uint16, (17, 50, 33), 4, 5, 3),
])
def test_bricked_lod_parity(dtype, shape, brick, levels, seed, layout):
    log("bricked parity %s %s brick=%d levels=%d layout=%d" % (
        np.dtype(dtype).name, shape, brick, levels, layout))
    from paper_1804_08197_amd import sg
    vol = gen.random_volume(shape, seed, dtype=dtype)
    vmax = 255 if dtype == np.uint8 else 65535
    tf = gen.tf_hot(a_start=60)
    tf[:, 3] *= 4.0
    h = gpu_volume([vol], brick, levels, [tf], [(0, vmax)], layout=layout)
    try:
        sc = oracle_scene([vol], brick, levels, [tf], [(0, vmax)])
        c = np.array(shape[::-1]) / 2.0
        views = gen.orbit_views(c, (20, 120), 3, seed, 61, 47, tan_top=0.6)
        views.append(gen.view(gen.look_at(c + 0.3, c + (5, -3, 7)), 53, 35, 0.9))  # inside
        for tau in (1.0, 3.5):
            for skip in (0, 1):
                params = {"ert": ERT, "tau": tau, "lod": 1, "skip_empty": skip}
                _, worst = check_views(h, sc, views, params, samples=True, depth=(tau == 1.0))
                log("  tau %.1f skip %d worst %.3g" % (tau, skip, worst))
    finally:
        sg.sg_volume_destroy(h)


def test_lod_cut_bit_exact_and_empty_flags():
    log("cut bit-exact")
    from paper_1804_08197_amd import sg
    rng = np.random.default_rng(5)
    vol = gen.random_volume((60, 52, 70), 9, dtype=np.uint16)
    tf = gen.tf_hot(a_start=100)
    h = gpu_volume([vol], 8, 4, [tf], [(0, 65535)])
    try:
        sc = oracle_scene([vol], 8, 4, [tf], [(0, 65535)])
        n_cmp = 0
        for i in range(40):
            eye = rng.uniform(-80, 150, 3)
            v = gen.view(gen.look_at(eye, rng.uniform(0, 60, 3)), int(rng.integers(8, 400)),
                         int(rng.integers(8, 400)), float(rng.uniform(0.1, 1.5)))
            params = {"tau": float(rng.uniform(0.3, 8)), "bias": int(rng.integers(0, 4)),
                      "lod": int(rng.integers(0, 5) > 0)}
            ids, emp = sg.sg_get_lod_cut(h, v, params)
            ref = sc.cut(v, params)
            assert np.array_equal(ids, ref), "cut differs for view %d" % i
            assert np.array_equal(emp, sc.empty(ref)), "empty flags differ for view %d" % i
            n_cmp += len(ids)
        assert n_cmp > 500
    finally:
        sg.sg_volume_destroy(h)


def test_skip_empty_bit_identical_and_deterministic():
    from paper_1804_08197_amd import sg
    vol = gen.random_volume((48, 44, 52), 12, dtype=np.uint16)
    tf = gen.tf_hot(a_start=120)
    h = gpu_volume([vol], 8, 3, [tf], [(0, 65535)])
    try:
        views = gen.orbit_views((26, 22, 24), (40, 120), 2, 13, 90, 70)
        p = {"ert": ERT, "tau": 1.5}
        a = render_gpu(h, views, dict(p, skip_empty=1))["rgba"]
        b = render_gpu(h, views, dict(p, skip_empty=0))["rgba"]
        c = render_gpu(h, views, dict(p, skip_empty=1))["rgba"]
        for x, y, z in zip(a, b, c):
            assert np.array_equal(x, y)
            assert np.array_equal(x, z)
        # a stereo pair in one call equals each eye rendered alone
        for i, v in enumerate(views):
            single = render_gpu(h, [v], dict(p, skip_empty=1))["rgba"][0]
            assert np.array_equal(single, a[i])
    finally:
        sg.sg_volume_destroy(h)


def test_empty_volume_returns_background_exactly():
    from paper_1804_08197_amd import sg
    vol = np.zeros((20, 30, 25), dtype=np.uint8)
    tf = gen.tf_hot()
    h = gpu_volume([vol], 8, 2, [tf], [(0, 255)])
    try:
        bg = (0.125, 0.25, 0.5, 0.75)
        views = [gen.view(gen.look_at((-20, 40, 30), (12, 15, 10)), 33, 21, 0.5),
                 gen.view(gen.look_at((12, 15, 10), (40, 40, 40)), 17, 9, 1.0),   # inside
                 gen.view(gen.look_at((-50, -50, -50), (-100, -90, -80)), 7, 5, 0.2)]  # misses
        for skip in (0, 1):
            out = render_gpu(h, views, {"bg": bg, "skip_empty": skip, "ert": ERT})["rgba"]
            for o in out:
                assert np.array_equal(o.astype(np.float32), np.broadcast_to(
                    np.array(bg, np.float32), o.shape))
    finally:
        sg.sg_volume_destroy(h)


def test_constant_medium_closed_form_on_gpu():
    from paper_1804_08197_amd import sg
    vol = np.full((24, 32, 28), 77, dtype=np.uint8)
    rgb, rho = np.array([0.3, 0.6, 0.9]), 0.037
    tf = gen.tf_constant(rgb, rho)
    h = gpu_volume([vol], 8, 3, [tf], [(0, 255)])
    try:
        import oracle
        views = [gen.view(gen.look_at((-20, 70, 50), (14, 16, 12)), 23, 17, 0.5),
                 gen.view(gen.look_at((10, 12, 9), (40, -3, 5)), 15, 19, 1.2)]
        rho32 = float(np.float32(rho))
        for bias in range(3):
            for lod in (0, 1):
                out = render_gpu(h, views, {"ert": 2.0, "bias": bias, "lod": lod, "tau": 2.0,
                                            "skip_empty": 0})["rgba"]
                for v, o in zip(views, out):
                    for y in range(v["height"]):
                        for x in range(v["width"]):
                            e, d = oracle.ray(v, x, y)
                            hit, tn, tfar = oracle.entry_exit((28, 32, 24), e, d)
                            A = 1 - math.exp(-rho32 * (tfar - tn)) if hit else 0.0
                            assert abs(o[y, x, 3] - A) < 2e-6
                            assert np.allclose(o[y, x, :3], np.float32(rgb) * A, atol=2e-6)
    finally:
        sg.sg_volume_destroy(h)


@pytest.mark.parametrize("layout", LAYOUTS, ids=LAYOUT_IDS)
def test_multichannel_parity(layout):
    log("multichannel parity layout=%d" % layout)
    from paper_1804_08197_amd import sg
    chans = [gen.random_volume((36, 40, 44), 20 + c, dtype=np.uint16) for c in range(3)]
    tfs = [gen.tf_tint(t, a_start=50, a_max=0.4) for t in gen.CELL_TINTS]
    doms = [(0, 65535)] * 3
    h = gpu_volume(chans, 8, 3, tfs, doms, layout=layout)
    try:
        sc = oracle_scene(chans, 8, 3, tfs, doms)
        views = gen.stereo((-40.0, 90.0, 60.0), (22, 20, 18), 5.0, 45, 39, 0.5, 0.55)
        _, worst = check_views(h, sc, views, {"ert": ERT, "tau": 1.0}, samples=True)
        log("  worst %.3g" % worst)
    finally:
        sg.sg_volume_destroy(h)


def test_host_and_device_uploads_agree():
    from paper_1804_08197_amd import sg
    vol = gen.random_volume((30, 26, 34), 31, dtype=np.uint16)
    tf = gen.tf_hot(a_start=30)
    hd = gpu_volume([vol], 8, 3, [tf], [(0, 65535)], device_upload=True)
    hh = gpu_volume([vol], 8, 3, [tf], [(0, 65535)], device_upload=False)
    try:
        v = [gen.view(gen.look_at((-30, 50, 40), (17, 13, 15)), 40, 33, 0.5)]
        a = render_gpu(hd, v, {"ert": ERT})["rgba"][0]
        b = render_gpu(hh, v, {"ert": ERT})["rgba"][0]
        assert np.array_equal(a, b)
    finally:
        sg.sg_volume_destroy(hd)
        sg.sg_volume_destroy(hh)


def test_edge_cases_tiny_images_and_no_termination():
    from paper_1804_08197_amd import sg
    vol = gen.random_volume((21, 19, 23), 41, dtype=np.uint8)
    tf = gen.tf_identity()
    tf[:, 3] *= 0.05
    h = gpu_volume([vol], 4, 3, [tf], [(0, 255)])
    try:
        sc = oracle_scene([vol], 4, 3, [tf], [(0, 255)])
        views = [gen.view(gen.look_at((-10, 30, 20), (11, 9, 10)), 1, 1, 0.3),
                 gen.view(gen.look_at((-10, 30, 20), (11, 9, 10)), 1, 37, 0.3),
                 gen.view(gen.look_at((40, -20, 5), (11, 9, 10)), 17, 1, 0.8)]
        for ert in (ERT, 5.0):
            check_views(h, sc, views, {"ert": ert, "tau": 2.0})
    finally:
        sg.sg_volume_destroy(h)


def test_error_paths_on_gpu():
    import torch

    from paper_1804_08197_amd import sg
    h = sg.sg_volume_create((16, 16, 16), brick=8, levels=2, dtype=sg.SG_U8)
    try:
        v = gen.view(gen.look_at((-10, 8, 8), (8, 8, 8)), 8, 8, 0.5)
        out = [torch.zeros(8, 8, 4, device="cuda")]
        with pytest.raises(sg.SgError) as ex:
            sg.sg_render_views(h, [v], {}, out)
        assert ex.value.status == sg.SG_ERR_STATE
        sg.sg_set_transfer_function(h, 0, gen.tf_identity(), 0, 255)
        sg.sg_render_views(h, [v], {}, out)
        bad = dict(v)
        bad["cam_to_world"] = v["cam_to_world"].copy()
        bad["cam_to_world"][0, 0] = float("nan")
        for vv, p in [(bad, {}), (v, {"bias": 2}), (v, {"step": 0.0}), (v, {"tau": -1}),
                      (v, {"timepoint": 1}), (v, {"flags": 64})]:
            with pytest.raises(sg.SgError) as ex:
                sg.sg_render_views(h, [vv], p, out)
            assert ex.value.status == sg.SG_ERR_INVALID_ARG
        sing = dict(v)
        sing["cam_to_world"] = np.zeros((4, 4))
        with pytest.raises(sg.SgError) as ex:
            sg.sg_render_views(h, [sing], {}, out)
        assert ex.value.status == sg.SG_ERR_INVALID_ARG
        with pytest.raises(sg.SgError):
            sg.sg_set_transfer_function(h, 0, gen.tf_identity(), 10, 5)
        with pytest.raises(sg.SgError):
            sg.sg_upload_bricks(h, 0, 0, 0, [[2, 0, 0]], np.zeros((1, 8, 8, 8), np.uint8))
        torch.cuda.synchronize()
    finally:
        sg.sg_volume_destroy(h)


@pytest.mark.parametrize("layout", LAYOUTS, ids=LAYOUT_IDS)
@pytest.mark.parametrize("dtype,shape,brick,levels,chans", [
    (np.uint16, (29, 38, 45), 8, 4, 1), (np.uint8, (40, 40, 40), 16, 3, 1),
    (np.uint8, (17, 50, 33), 2, 5, 1), (np.uint16, (36, 40, 44), 8, 3, 3),
    (np.uint8, (70, 66, 90), 32, 3, 2)])
def test_staged_and_gather_kernels_bit_identical(dtype, shape, brick, levels, chans, layout):
    """The LDS-staged kernel and the direct-gather kernel share every sample
    computation, so their images (and sample counts) must agree exactly."""
    log("staged vs gather %s %s brick=%d ch=%d layout=%d" % (
        np.dtype(dtype).name, shape, brick, chans, layout))
    from paper_1804_08197_amd import sg
    vols = [gen.random_volume(shape, 50 + c, dtype=dtype) for c in range(chans)]
    vmax = 255 if dtype == np.uint8 else 65535
    tfs = [gen.tf_hot(a_start=40)] if chans == 1 else \
        [gen.tf_tint(t, a_start=40, a_max=0.5) for t in gen.CELL_TINTS[:chans]]
    h = gpu_volume(vols, brick, levels, tfs, [(0, vmax)] * chans, layout=layout)
    try:
        c = np.array(shape[::-1]) / 2.0
        views = gen.orbit_views(c, (15, 150), 4, 7, 77, 45, tan_top=0.7)
        views.append(gen.view(gen.look_at(c, c + (3, 7, -2)), 64, 64, 1.2))  # inside
        views.append(gen.view(gen.look_at(c + (0, 0, 200.0), c, up=(0, 1, 0)), 40, 40, 0.3))
        for tau in (0.7, 2.0):
            for ert in (ERT, 5.0):
                p = {"ert": ert, "tau": tau}
                a = render_gpu(h, views, dict(p, gather=1), depth=True, samples=True)
                b = render_gpu(h, views, dict(p, gather=0), depth=True, samples=True)
                for i in range(len(views)):
                    assert np.array_equal(a["rgba"][i], b["rgba"][i]), "view %d tau %g" % (i, tau)
                    assert np.array_equal(a["depth"][i], b["depth"][i])
                    assert np.array_equal(a["nsamp"][i], b["nsamp"][i])
                for key in ("total_samples", "microblocks"):
                    assert a["stats"][key] == b["stats"][key]
    finally:
        sg.sg_volume_destroy(h)


@pytest.mark.parametrize("dtype,shape,brick,levels,chans", [
    (np.uint16, (29, 38, 45), 8, 4, 1), (np.uint8, (40, 40, 40), 16, 3, 1),
    (np.uint8, (17, 50, 33), 2, 5, 1), (np.uint16, (36, 40, 44), 4, 3, 3),
    (np.uint16, (70, 66, 90), 32, 3, 2), (np.uint8, (60, 70, 130), 128, 1, 1)])
def test_microblock_slots_render_the_linear_images(dtype, shape, brick, levels, chans):
    """The same data in linear and in micro-block slots (every brick edge,
    so stored edges of 4 to 130 voxels: multiples of 4 and not), rendered
    by both kernels under every optical model, with LOD, depth and sample
    counts: the images are equal bit for bit. Pins the slot addressing of
    the uploads, the pyramid, the aprons, the staging copies and the pool
    reads of the micro-block layout to the linear one."""
    log("layouts %s %s brick=%d ch=%d" % (np.dtype(dtype).name, shape, brick, chans))
    from paper_1804_08197_amd import sg
    vols = [gen.random_volume(shape, 90 + c, dtype=dtype) for c in range(chans)]
    vmax = 255 if dtype == np.uint8 else 65535
    tfs = [gen.tf_hot(a_start=40)] if chans == 1 else \
        [gen.tf_tint(t, a_start=40, a_max=0.5) for t in gen.CELL_TINTS[:chans]]
    hl = gpu_volume(vols, brick, levels, tfs, [(0, vmax)] * chans, layout=sg.SG_LAYOUT_LINEAR)
    hm = gpu_volume(vols, brick, levels, tfs, [(0, vmax)] * chans,
                    layout=sg.SG_LAYOUT_MICROBLOCK)
    try:
        c = np.array(shape[::-1]) / 2.0
        views = gen.orbit_views(c, (15, 150), 3, 11, 69, 41, tan_top=0.7)
        views.append(gen.view(gen.look_at(c, c + (3, 7, -2)), 64, 64, 1.2))  # inside
        for model in ("ea", "eo", "mip"):
            for gather in (0, 1):
                p = {"ert": ERT, "tau": 1.5, "model": model, "gather": gather}
                a = render_gpu(hl, views, p, depth=True, samples=True)
                b = render_gpu(hm, views, p, depth=True, samples=True)
                for i in range(len(views)):
                    assert np.array_equal(a["rgba"][i], b["rgba"][i]), (model, gather, i)
                    assert np.array_equal(a["depth"][i], b["depth"][i], equal_nan=True)
                    assert np.array_equal(a["nsamp"][i], b["nsamp"][i])
                for key in ("total_samples", "microblocks", "node_visits"):
                    assert a["stats"][key] == b["stats"][key], key
        for v in views[:2]:
            for L in range(levels):
                p = {"lod": 0, "bias": L}
                assert all(np.array_equal(x, y) for x, y in zip(sg.sg_get_lod_cut(hl, v, p),
                                                                 sg.sg_get_lod_cut(hm, v, p)))
    finally:
        sg.sg_volume_destroy(hl)
        sg.sg_volume_destroy(hm)
