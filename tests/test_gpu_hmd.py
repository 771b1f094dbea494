"""GPU parity of the head-mounted-display variants against the FP64 oracle.

Emission-only and maximum-intensity models (Sec 5.1), cut planes and region
of interest (Sec 6), per-pixel ray limits from opaque geometry (Sec 5.6) and
wrapped-space rays (Sec 5.3), through the C-ABI, in both kernels. RGBA within
1e-4 (emission-absorption with the early-termination bracket), skip flags
bit-exact, skip on / off bit-identical.
"""
import sys

import numpy as np
import pytest

import gen
from tests.helpers import (ERT, TOL, bracket_error, gpu_volume, oracle_bracket, oracle_scene,
                           render_gpu)

pytestmark = pytest.mark.gpu

DIMS_ZYX = (44, 40, 52)  # ragged against 16^3 bricks


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU (no CPU fallback exists)"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def views2():
    """Two uneven views with ragged tiles: a near one (three LOD levels in
    its cut) and a farther, tilted one."""
    a = gen.view(gen.look_at((-30.0, 70.0, 55.0), (26.0, 20.0, 22.0)), 83, 61, 0.55)
    b = gen.view(gen.look_at((90.0, -40.0, 10.0), (26.0, 20.0, 22.0), up=(0.2, 0.3, 1.0)),
                 50, 70, 0.5)
    return [a, b]


@pytest.fixture(scope="module")
def scene():
    from paper_1804_08197_amd import sg
    vol = gen.random_volume(DIMS_ZYX, 401, dtype=np.uint16)
    rng = np.random.default_rng(402)
    tf = gen.tf_random(rng, zero_below=60).astype(np.float32)
    tf[:, :3] *= 0.02
    tf[:90, :3] = 0.0  # dark below entry 90: emission-only skips
    h = gpu_volume([vol], 16, 3, [tf], [(0, 65535)])
    sc = oracle_scene([vol], 16, 3, [tf], [(0, 65535)])
    yield h, sc, vol
    sg.sg_volume_destroy(h)


def compare_plain(g, sc, views, params, limits=None, counts=True):
    """Models without early termination: one oracle render per view."""
    for i, v in enumerate(views):
        ref = sc.render(v, params, count=counts, limit=None if limits is None else limits[i])
        err = np.abs(g["rgba"][i] - ref["rgba"]).max(axis=-1)
        assert err.max() <= TOL, "view %d: err %g at %s" % (i, err.max(),
                                                            np.unravel_index(err.argmax(),
                                                                             err.shape))
        if counts and "nsamp" in g:
            bad = int((g["nsamp"][i] != ref["nsamp"]).sum())
            assert bad <= max(2, 1e-3 * err.size), "sample counts differ at %d px" % bad


@pytest.mark.parametrize("gather", [0, 1])
def test_emission_only_parity_and_dark_skip(scene, gather):
    import torch
    h, sc, _ = scene
    vs = views2()
    p = {"model": "eo", "lod": 1, "tau": 1.0, "gather": gather}
    g = render_gpu(h, vs, p, samples=True)
    compare_plain(g, sc, vs, p)
    assert all(np.all(r[..., 3] == 0) for r in g["rgba"])
    g0 = render_gpu(h, vs, dict(p, skip_empty=0), samples=True)
    for a, b in zip(g["rgba"], g0["rgba"]):
        assert np.array_equal(a, b)
    assert g["stats"]["total_samples"] < g0["stats"]["total_samples"]
    log("emission-only gather=%d: samples %d (no skip %d)" % (
        gather, g["stats"]["total_samples"], g0["stats"]["total_samples"]))


@pytest.mark.parametrize("gather", [0, 1])
def test_max_intensity_parity_and_skip(scene, gather):
    h, sc, _ = scene
    vs = views2()
    p = {"model": "mip", "lod": 1, "tau": 1.0, "gather": gather, "bg": (0.1, 0.0, 0.2, 0.5)}
    g = render_gpu(h, vs, p, samples=True)
    compare_plain(g, sc, vs, p)
    g0 = render_gpu(h, vs, dict(p, skip_empty=0), samples=True)
    for a, b in zip(g["rgba"], g0["rgba"]):
        assert np.array_equal(a, b)
    assert g["stats"]["total_samples"] < g0["stats"]["total_samples"]


def test_skip_flags_of_each_model_are_bit_exact(scene):
    from paper_1804_08197_amd import sg
    h, sc, _ = scene
    for v in views2():
        for model in ("ea", "eo", "mip"):
            p = {"model": model, "lod": 1, "tau": 1.0}
            ids, emp = sg.sg_get_lod_cut(h, v, p)
            cut = sc.cut(v, p)
            assert np.array_equal(ids, cut)
            assert np.array_equal(emp, sc.empty(cut, model)), model
    assert sc.empty(cut, "eo").any() and not sc.empty(cut, "mip").any()


def test_multichannel_emission_only_and_mip_parity():
    from paper_1804_08197_amd import sg
    rng = np.random.default_rng(410)
    vols = [gen.random_volume((30, 34, 38), 411 + c, dtype=np.uint8) for c in range(3)]
    tfs = [(gen.tf_random(rng) * 0.02).astype(np.float32) for _ in range(3)]
    h = gpu_volume(vols, 16, 2, tfs, [(0, 255)] * 3)
    try:
        sc = oracle_scene(vols, 16, 2, tfs, [(0, 255)] * 3)
        v = gen.view(gen.look_at((-25.0, 60.0, 45.0), (19.0, 17.0, 15.0)), 70, 45, 0.5)
        for model in ("eo", "mip"):
            for gather in (0, 1):
                p = {"model": model, "gather": gather}
                g = render_gpu(h, [v], p, samples=True)
                compare_plain(g, sc, [v], p)
    finally:
        sg.sg_volume_destroy(h)


@pytest.mark.parametrize("gather", [0, 1])
def test_cut_planes_and_roi_parity(scene, gather):
    h, sc, _ = scene
    vs = views2()
    n = gen.unit((0.6, -0.3, 0.74))
    c = np.array([26.0, 20.0, 22.0])
    cases = [
        {"planes": [(n[0], n[1], n[2], -float(n @ c))]},
        {"planes": [(1.0, 0.0, 0.0, -30.0), (0.0, -1.0, 0.0, 8.0)]},
        {"roi": (6.0, 4.5, 3.0, 40.0, 33.25, 30.0)},
        {"planes": [(-n[0], -n[1], -n[2], float(n @ c))], "roi": (0, 0, 0, 30, 30, 30)},
    ]
    for extra in cases:
        p = dict({"ert": ERT, "gather": gather}, **extra)
        g = render_gpu(h, vs, p)
        for i, v in enumerate(vs):
            best, _ = bracket_error(g["rgba"][i], oracle_bracket(sc, v, p))
            assert best.max() <= TOL, (extra, i, best.max())
    # clipping everything away leaves the background
    g = render_gpu(h, vs, {"ert": ERT, "roi": (1, 1, 1, 1, 1, 1), "bg": (0.25, 0.5, 0.75, 1.0)})
    for r in g["rgba"]:
        assert np.all(r == np.array([0.25, 0.5, 0.75, 1.0]))


@pytest.mark.parametrize("model", ["ea", "eo"])
def test_ray_limit_parity(scene, model):
    import torch
    h, sc, _ = scene
    vs = views2()
    rng = np.random.default_rng(420)
    limits, views = [], []
    for v in vs:
        lim = rng.uniform(20.0, 140.0, (v["height"], v["width"])).astype(np.float32)
        lim[rng.uniform(size=lim.shape) < 0.2] = np.inf
        lim[:4, :] = 1.0  # geometry in front of the volume
        limits.append(lim)
        views.append(dict(v, ray_limit=torch.from_numpy(lim).cuda()))
    p = {"ert": ERT, "model": model, "bg": (0.0, 0.1, 0.0, 0.3)}
    g = render_gpu(h, views, p)
    for i, v in enumerate(vs):
        refs = [sc.render(v, dict(p, ert=e), limit=limits[i].astype(np.float64))
                for e in (ERT, ERT - 1e-5, ERT + 1e-5)]
        best, _ = bracket_error(g["rgba"][i], refs)
        assert best.max() <= TOL, (i, best.max())
        bg = np.array([0.0, 0.1, 0.0, 0.3], dtype=np.float32).astype(np.float64)
        assert np.all(g["rgba"][i][:4] == bg)


@pytest.mark.parametrize("gather", [0, 1])
def test_wrapped_space_rays_parity(scene, gather):
    h, sc, _ = scene
    vs = [dict(v, lens=(0.25, 0.06, 0.03, -0.02)) for v in views2()]
    p = {"ert": ERT, "gather": gather}
    g = render_gpu(h, vs, p, samples=True)
    for i, v in enumerate(vs):
        refs = oracle_bracket(sc, v, p, count=True)
        best, _ = bracket_error(g["rgba"][i], refs)
        assert best.max() <= TOL
        ok = np.zeros(best.shape, bool)
        for r in refs:
            ok |= g["nsamp"][i] == r["nsamp"]
        assert (~ok).sum() <= max(2, 1e-3 * ok.size)


def test_all_variants_together_in_one_stereo_call(scene):
    """Lens, ray limit, cut plane and ROI on a stereo pair in one launch; each
    eye equals its own single-view render."""
    import torch
    from paper_1804_08197_amd import sg
    h, sc, _ = scene
    pair = gen.stereo(np.array([-20.0, 60.0, 50.0]), np.array([26.0, 20.0, 22.0]), 8.0, 64, 72,
                      0.6, 0.54)
    lim = torch.full((72, 64), 95.0, device="cuda")
    pair = [dict(v, lens=(0.2, 0.0, 0.0, 0.0), ray_limit=lim) for v in pair]
    p = {"ert": ERT, "planes": [(0.0, 0.0, 1.0, -30.0)], "roi": (2, 2, 2, 50, 38, 42)}
    g = render_gpu(h, pair, p)
    for i, v in enumerate(pair):
        refs = oracle_bracket(sc, v, p, limit=np.full((72, 64), 95.0))
        best, _ = bracket_error(g["rgba"][i], refs)
        assert best.max() <= TOL
        one = render_gpu(h, [v], p)
        assert np.array_equal(one["rgba"][0], g["rgba"][i])


def test_bad_clip_and_model_arguments_are_rejected(scene):
    from paper_1804_08197_amd import sg
    h, _, _ = scene
    import torch
    v = views2()[0]
    out = [torch.empty(v["height"], v["width"], 4, device="cuda")]
    for p in ({"model": 3}, {"planes": [(0.0, 0.0, 0.0, 1.0)]}, {"roi": (5, 0, 0, 4, 1, 1)},
              {"planes": [(1.0, 0.0, 0.0, float("nan"))]}, {"n_planes": 5}):
        with pytest.raises(sg.SgError) as ex:
            sg.sg_render_views(h, [v], p, out)
        assert ex.value.status == sg.SG_ERR_INVALID_ARG
    with pytest.raises(sg.SgError):
        sg.sg_render_views(h, [dict(v, lens=(float("inf"), 0, 0, 0))], {}, out)
