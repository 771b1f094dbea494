"""Pins of the oracle's head-mounted-display variants (CPU only).

* wrapped-space rays (Sec 5.3): a radial lens map of the pixel tangents;
* ray clipping: cut planes and region of interest (Sec 6), termination at
  the distance of opaque geometry (Sec 5.6);
* optical models (Sec 5.1): emission-only and maximum intensity projection
  next to emission-absorption, with the zero alpha of Sec 5.6.

Each check is against a closed form, a library routine, brute force or an
invariant, never against the oracle's own formula retyped.
"""
import math

import numpy as np
import pytest
from scipy import integrate, ndimage, optimize

import gen
import oracle as O

O.build()

NO_ERT = 2.0


def params(**kw):
    p = {"step": 0.5, "ert": NO_ERT, "tau": 1.0, "bg": (0, 0, 0, 0), "bias": 0, "lod": 1,
         "skip_empty": 1}
    p.update(kw)
    return p


def _profile_volume(seed=30, n=40):
    rng = np.random.default_rng(seed)
    prof = rng.integers(0, 65535, n).astype(np.uint16)
    return np.broadcast_to(prof[None, None, :], (6, 6, n)).copy(), prof


# ------------------------------------------------------- emission-only model
@pytest.mark.parametrize("B,levels", [(32, 1), (8, 3)])
def test_emission_only_constant_medium_closed_form(B, levels):
    """Constant emission rgb over a chord of length L integrates to rgb L,
    alpha stays 0 and the background shows through unattenuated."""
    vol = np.full((24, 32, 28), 77, dtype=np.uint8)
    rgb = np.array([0.003, 0.006, 0.009])
    tf = gen.tf_constant(rgb, 0.5)
    sc = O.Scene([vol], B, levels, [tf], [(0, 255)])
    v = gen.view(gen.look_at((-20, 70, 50), (14, 16, 12)), 13, 11, 0.5)
    bg = (0.1, 0.2, 0.3, 0.4)
    for lod in (0, 1):
        for bias in range(levels):
            out = sc.render(v, params(model="eo", lod=lod, bias=bias, bg=bg, ert=0.99))["rgba"]
            for y in range(v["height"]):
                for x in range(v["width"]):
                    e, d = O.ray(v, x, y)
                    hit, tn, tf_ = O.entry_exit((28, 32, 24), e, d)
                    L = (tf_ - tn) if hit else 0.0
                    assert np.allclose(out[y, x, :3], rgb * L + np.array(bg[:3]), atol=1e-12)
                    assert out[y, x, 3] == bg[3]


def test_emission_only_converges_to_the_emission_integral():
    """The emission-only integral of Sec 5.1 (I = integral of tau[f] along the
    chord), computed with scipy.integrate.quad on the trilinear field, is
    approached at second order as the step shrinks."""
    vol, prof = _profile_volume()
    tf = gen.tf_identity()
    tf[:, 1] = np.sqrt(tf[:, 1]) * 0.01
    lo, hi = 0.0, 65535.0
    sc = O.Scene([vol], 64, 1, [tf], [(lo, hi)])
    e = np.array([-3.0, 3.0, 3.0])
    v = gen.view(gen.look_at(e, (20.0, 3.0, 3.0)), 1, 1, 0.01)

    def g(t):
        val = ndimage.map_coordinates(prof.astype(np.float64), [[e[0] + t - 0.5]], order=1,
                                      mode="nearest")[0]
        return np.interp((val - lo) / (hi - lo) * 255, np.arange(256), tf[:, 1])

    ref = integrate.quad(g, 3.0, 43.0, points=list(np.arange(3.5, 43.0, 1.0)), limit=400,
                         epsabs=1e-14)[0]
    errs = [abs(sc.render(v, params(model="eo", step=s, skip_empty=0))["rgba"][0, 0, 1] - ref)
            for s in (0.5, 0.25, 0.125, 0.0625)]
    assert errs[-1] < 2e-5
    for a, b in zip(errs, errs[1:]):
        assert a / b > 3.0


def test_emission_only_skip_of_dark_nodes_is_bit_identical():
    vol = gen.random_volume((20, 24, 28), 41, dtype=np.uint16)
    tf = gen.tf_random(np.random.default_rng(42)) * 0.01
    tf[:100, :3] = 0.0  # no emission below entry 100
    tf[:, 3] = 0.3  # extinction everywhere: the emission-absorption test finds no empty node
    sc = O.Scene([vol], 4, 3, [tf], [(0, 65535)])
    v = gen.view(gen.look_at((-30, 50, 40), (14, 12, 10)), 24, 20, 0.4)
    cut = sc.cut(v, params())
    dark = sc.empty(cut, "eo")
    assert dark.any() and not dark.all()
    assert not sc.empty(cut, "ea").any()
    a = sc.render(v, params(model="eo", skip_empty=0), count=True)
    b = sc.render(v, params(model="eo", skip_empty=1), count=True)
    assert np.array_equal(a["rgba"], b["rgba"])
    assert b["total_samples"] < a["total_samples"]


def test_emission_only_channels_add():
    """Two channels emit the sum of their single-channel images."""
    rng = np.random.default_rng(43)
    v0 = gen.random_volume((16, 16, 16), 44, dtype=np.uint8)
    v1 = gen.random_volume((16, 16, 16), 45, dtype=np.uint8)
    t0, t1 = gen.tf_random(rng) * 0.01, gen.tf_random(rng) * 0.01
    view = gen.view(gen.look_at((-20, 30, 25), (8, 8, 8)), 9, 7, 0.5)
    p = params(model="eo", skip_empty=0)
    both = O.Scene([v0, v1], 8, 2, [t0, t1], [(0, 255)] * 2).render(view, p)["rgba"]
    a = O.Scene([v0], 8, 2, [t0], [(0, 255)]).render(view, p)["rgba"]
    b = O.Scene([v1], 8, 2, [t1], [(0, 255)]).render(view, p)["rgba"]
    assert np.allclose(both[..., :3], a[..., :3] + b[..., :3], atol=1e-12)
    assert np.all(both[..., 3] == 0)


# ------------------------------------------------ maximum intensity projection
def test_mip_single_bright_voxel_hand_computed():
    """The centre ray meets the tent of a lone 255 voxel with samples of
    density 1/4, 3/4, 3/4, 1/4 of it: the maximum is 3/4 of 255, which the
    identity table maps to 0.75."""
    vol = np.zeros((9, 9, 9), dtype=np.uint8)
    vol[4, 4, 4] = 255
    sc = O.Scene([vol], 16, 1, [gen.tf_identity()], [(0, 255)])
    v = gen.view(gen.look_at((40.0, 4.5, 4.5), (4.5, 4.5, 4.5)), 3, 5, 0.01)
    out = sc.render(v, params(model="mip", skip_empty=0), count=True)
    assert np.allclose(out["rgba"][2, 1, :3], 0.75, atol=1e-15)
    assert out["rgba"][2, 1, 3] == 0.0
    assert out["nsamp"][2, 1] == 18


def test_mip_equals_max_of_library_samples():
    """Maximum of the trilinear samples (scipy) mapped through the table
    (numpy.interp), on a ray along a 1D profile."""
    vol, prof = _profile_volume(seed=50)
    rng = np.random.default_rng(51)
    tf = gen.tf_random(rng)
    lo, hi = 1000.0, 64000.0
    sc = O.Scene([vol], 64, 1, [tf], [(lo, hi)])
    e = np.array([-7.25, 3.0, 3.0])
    v = gen.view(gen.look_at(e, (20.0, 3.0, 3.0)), 1, 1, 0.01)
    out = sc.render(v, params(model="mip", skip_empty=0), count=True)
    t = 7.25 + 0.25 + 0.5 * np.arange(80)
    vals = ndimage.map_coordinates(prof.astype(np.float64), [e[0] + t - 0.5], order=1,
                                   mode="nearest")
    u = (vals.max() - lo) / (hi - lo) * 255
    ref = [np.interp(u, np.arange(256), tf[:, k]) for k in range(3)]
    assert out["nsamp"][0, 0] == 80
    assert np.allclose(out["rgba"][0, 0, :3], ref, atol=1e-12)


def test_mip_node_skip_is_bit_identical_and_bounded():
    """Passing over nodes whose stored maximum cannot raise the running
    maximum changes no pixel; every pixel is at most the table's colour at
    the volume maximum when the table is monotone."""
    vol = gen.random_volume((24, 28, 32), 52, dtype=np.uint16)
    tf = gen.tf_identity()
    sc = O.Scene([vol], 4, 3, [tf], [(0, 65535)])
    v = gen.view(gen.look_at((-30, 60, 40), (16, 14, 12)), 26, 22, 0.45)
    a = sc.render(v, params(model="mip", skip_empty=0), count=True)
    b = sc.render(v, params(model="mip", skip_empty=1), count=True)
    assert np.array_equal(a["rgba"], b["rgba"])
    assert b["total_samples"] < a["total_samples"]
    assert a["rgba"][..., :3].max() <= vol.max() / 65535 + 1e-12
    assert np.all(a["rgba"][..., 3] == 0)


# --------------------------------------------------------------- clipping
def _march_inside(e, d, t_max, keep, n=400001):
    t = np.linspace(0.0, t_max, n)
    pts = e[None, :] + t[:, None] * d[None, :]
    k = keep(pts)
    if not k.any():
        return None
    return t[k].min(), t[k].max()


def test_clip_interval_against_brute_force_marching():
    """Planes, region of interest and ray limit: the clipped interval equals
    the set of ray points passing every membership test, found by marching."""
    rng = np.random.default_rng(60)
    dims = np.array([40.0, 30.0, 20.0])
    checked = 0
    for _ in range(150):
        e = rng.uniform(-20, 60, 3)
        d = gen.unit(rng.uniform(0, 1, 3) * dims - e)
        hit, tn, tf_ = O.entry_exit(tuple(int(x) for x in dims), e, d)
        if not hit:
            continue
        planes = []
        for _ in range(rng.integers(0, 3)):
            n = gen.unit(rng.normal(size=3))
            c = rng.uniform(0, 1, 3) * dims
            planes.append((n[0], n[1], n[2], -float(n @ c)))
        roi = None
        if rng.uniform() < 0.5:
            a, b = rng.uniform(0, 1, 3) * dims, rng.uniform(0, 1, 3) * dims
            roi = np.concatenate([np.minimum(a, b), np.maximum(a, b)])
        limit = rng.uniform(tn, tf_ + 10) if rng.uniform() < 0.5 else np.inf
        ok, t0, t1 = O.clip(params(planes=planes, roi=roi), e, d, tn, tf_, limit)

        def keep(p):
            k = np.all((p >= 0) & (p <= dims), axis=1)
            for q in planes:
                k &= p @ np.array(q[:3]) + q[3] <= 0
            if roi is not None:
                k &= np.all((p >= roi[:3]) & (p <= roi[3:]), axis=1)
            return k

        t_max = min(tf_ + 1.0, limit)
        ref = _march_inside(e, d, t_max, keep)
        step = t_max / 400000
        if ref is None or ref[1] - ref[0] < 4 * step:
            assert not ok or t1 - t0 < 4 * step
            continue
        assert ok
        assert abs(t0 - ref[0]) <= 2 * step and abs(t1 - ref[1]) <= 2 * step
        checked += 1
    assert checked > 40


def test_cut_plane_constant_medium_closed_form():
    """Constant medium cut by the plane x <= 12 (normal +x): a ray along +x
    entering at x = 0 integrates 12 voxel lengths."""
    vol = np.full((16, 16, 40), 50, dtype=np.uint8)
    rho = 0.05
    tf = gen.tf_constant((0.2, 0.4, 0.6), rho)
    sc = O.Scene([vol], 8, 2, [tf], [(0, 255)])
    v = gen.view(gen.look_at((-10.0, 8.0, 8.0), (20.0, 8.0, 8.0)), 1, 1, 0.01)
    for lod in (0, 1):
        out = sc.render(v, params(planes=[(1.0, 0.0, 0.0, -12.0)], lod=lod))["rgba"]
        A = 1 - math.exp(-rho * 12.0)
        assert abs(out[0, 0, 3] - A) < 1e-12
        # the mirrored plane keeps x >= 12: 28 lengths
        out = sc.render(v, params(planes=[(-1.0, 0.0, 0.0, 12.0)], lod=lod))["rgba"]
        assert abs(out[0, 0, 3] - (1 - math.exp(-rho * 28.0))) < 1e-12
    # a plane parallel to the ray keeps all of it or none
    keep = sc.render(v, params(planes=[(0.0, 1.0, 0.0, -9.0)]))["rgba"]
    none = sc.render(v, params(planes=[(0.0, 1.0, 0.0, -7.0)]))["rgba"]
    assert abs(keep[0, 0, 3] - (1 - math.exp(-rho * 40.0))) < 1e-12
    assert none[0, 0, 3] == 0.0


def test_ray_inside_a_brick_face_is_counted_once():
    """An axis-parallel ray lying in the face shared by four bricks crosses
    the medium once (cells are half-open), at every level of detail."""
    vol = np.full((16, 16, 40), 50, dtype=np.uint8)
    rho = 0.05
    sc = O.Scene([vol], 8, 2, [gen.tf_constant((0.2, 0.4, 0.6), rho)], [(0, 255)])
    for eye in [(-10.0, 8.0, 8.0), (-10.0, 16.0, 0.0), (-10.0, 8.0, 3.0)]:
        v = gen.view(gen.look_at(eye, (20.0, eye[1], eye[2])), 1, 1, 0.01)
        for lod in (0, 1):
            for bias in (0, 1):
                out = sc.render(v, params(lod=lod, bias=bias), count=True)
                assert abs(out["rgba"][0, 0, 3] - (1 - math.exp(-rho * 40.0))) < 1e-12
                assert out["nsamp"][0, 0] == 80 // 2 ** bias


def test_roi_and_ray_limit_constant_medium_closed_form():
    vol = np.full((16, 16, 40), 50, dtype=np.uint8)
    rho = 0.05
    tf = gen.tf_constant((0.2, 0.4, 0.6), rho)
    sc = O.Scene([vol], 8, 2, [tf], [(0, 255)])
    v = gen.view(gen.look_at((-10.0, 8.0, 8.0), (20.0, 8.0, 8.0)), 1, 1, 0.01)
    out = sc.render(v, params(roi=(5, 2, 2, 17.5, 14, 14)))["rgba"]
    assert abs(out[0, 0, 3] - (1 - math.exp(-rho * 12.5))) < 1e-12
    # opaque geometry 21 units from the eye: the ray (entering at t = 10)
    # integrates 11 lengths and stops
    lim = np.array([[21.0]])
    out = sc.render(v, params(), limit=lim, count=True)
    assert abs(out["rgba"][0, 0, 3] - (1 - math.exp(-rho * 11.0))) < 1e-12
    assert out["nsamp"][0, 0] == 22
    # geometry in front of the volume hides it
    out = sc.render(v, params(bg=(0.5, 0.5, 0.5, 1.0)), limit=np.array([[5.0]]))["rgba"]
    assert np.array_equal(out[0, 0], [0.5, 0.5, 0.5, 1.0])


# --------------------------------------------------------- wrapped-space rays
def _cam_tangent(view, d):
    """Tangent-plane coordinates of a world direction in the view's camera."""
    m = np.asarray(view["cam_to_world"], dtype=np.float64).reshape(4, 4)
    c = m[:3, :3].T @ d
    return -c[0] / c[2], -c[1] / c[2]


def test_lens_with_zero_coefficients_is_rectilinear():
    vol = gen.random_volume((16, 16, 16), 70, dtype=np.uint8)
    sc = O.Scene([vol], 8, 2, [gen.tf_identity()], [(0, 255)])
    v = gen.view(gen.look_at((-20, 30, 25), (8, 8, 8)), 11, 9, 0.6)
    w = dict(v, lens=(0.0, 0.0, 0.3, -0.2))
    p = params(ert=0.99)
    assert np.array_equal(sc.render(v, p)["rgba"], sc.render(w, p)["rgba"])


def test_lens_rays_invert_to_the_uniform_pixel_grid():
    """Inverting the radial lens map numerically (scipy brentq) on each wrapped
    ray's tangent recovers the pixel centre of the uniform grid; the lens
    centre stays fixed and rays spread outwards for k1 > 0."""
    k1, k2, cx, cy = 0.22, 0.05, 0.1, -0.05
    v = gen.view(gen.look_at((-20, 30, 25), (8, 8, 8)), 31, 27, 0.9)
    w = dict(v, lens=(k1, k2, cx, cy))
    for x, y in [(0, 0), (30, 26), (15, 13), (3, 20), (27, 4)]:
        sx0 = v["tan_left"] + (x + 0.5) / v["width"] * (v["tan_right"] - v["tan_left"])
        sy0 = v["tan_top"] - (y + 0.5) / v["height"] * (v["tan_top"] - v["tan_bottom"])
        e, d = O.ray(w, x, y)
        tx, ty = _cam_tangent(v, d)
        rt = math.hypot(tx - cx, ty - cy)
        r0 = optimize.brentq(lambda r: r * (1 + k1 * r * r + k2 * r ** 4) - rt, 0.0, rt + 1e-12,
                             xtol=1e-15)
        ux, uy = (tx - cx) / rt * r0 + cx, (ty - cy) / rt * r0 + cy
        assert abs(ux - sx0) < 1e-10 and abs(uy - sy0) < 1e-10
        assert rt >= math.hypot(sx0 - cx, sy0 - cy) - 1e-15


def test_lens_pixel_equals_rectilinear_ray_through_its_tangent():
    """A wrapped pixel renders what a one-pixel rectilinear view pointed at
    the same tangent renders."""
    vol = gen.random_volume((24, 24, 24), 71, dtype=np.uint16)
    sc = O.Scene([vol], 8, 3, [gen.tf_hot()], [(0, 65535)])
    v = gen.view(gen.look_at((-25, 40, 30), (12, 12, 12)), 21, 17, 0.7)
    w = dict(v, lens=(0.3, 0.0, 0.0, 0.0))
    p = params(ert=0.99, lod=0)
    img = sc.render(w, p)["rgba"]
    for x, y in [(0, 0), (20, 16), (10, 8), (4, 13)]:
        e, d = O.ray(w, x, y)
        tx, ty = _cam_tangent(v, d)
        h = 1e-9
        one = gen.view(v["cam_to_world"], 1, 1, ty + h, tan_right=tx + h, tan_left=tx - h,
                       tan_bottom=ty - h)
        ref = sc.render(one, p)["rgba"][0, 0]
        assert np.allclose(img[y, x], ref, atol=1e-9)
