"""Pins of the FP64 oracle against facts fixed by the paper and mathematics.

Each test checks one oracle step against something other than the oracle
itself: a closed form, a library routine (scipy / numpy), brute force, or an
invariant the method guarantees. They run on the CPU.
"""
import math

import numpy as np
import pytest
from scipy import integrate, ndimage

import gen
import oracle as O

O.build()

NO_ERT = 2.0  # a threshold alpha never reaches


def params(**kw):
    p = {"step": 0.5, "ert": NO_ERT, "tau": 1.0, "bg": (0, 0, 0, 0), "bias": 0, "lod": 1,
         "skip_empty": 1}
    p.update(kw)
    return p


# ---------------------------------------------------------------- O2 pyramid
@pytest.mark.parametrize("shape", [(8, 8, 8), (5, 7, 9), (1, 3, 2), (17, 4, 11)])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_pyramid_matches_padded_block_mean(shape, dtype):
    rng = np.random.default_rng(3)
    vmax = np.iinfo(dtype).max
    v = rng.integers(0, vmax + 1, shape, dtype=dtype)
    got = O.downsample(v)
    # independent: pad odd axes by edge replication, then sum 2x2x2 blocks
    pad = [(0, s % 2) for s in shape]
    p = np.pad(v.astype(np.int64), pad, mode="edge")
    m = [s // 2 for s in p.shape]
    blocks = p.reshape(m[0], 2, m[1], 2, m[2], 2).sum(axis=(1, 3, 5))
    assert np.array_equal(got.astype(np.int64), (blocks + 4) // 8)


def test_pyramid_dims_are_ceil_halves():
    assert O.level_dims((2048, 2048, 2048), 5) == (64, 64, 64)
    assert O.level_dims((1024, 1024, 512), 4) == (64, 64, 32)
    assert O.level_dims((5, 9, 1), 2) == (2, 3, 1)
    assert O.brick_grid((2048, 2048, 2048), 64, 0) == (32, 32, 32)
    assert O.brick_grid((1024, 1024, 512), 64, 4) == (1, 1, 1)
    # 37,449 bricks for the 2048^3 / 64^3 / 6-level pyramid
    total = sum(np.prod(O.brick_grid((2048,) * 3, 64, L)) for L in range(6))
    assert total == 37449


# ------------------------------------------------- O3 brick region / apron
def test_brick_region_is_clamped_window():
    rng = np.random.default_rng(5)
    lvl = rng.integers(0, 65535, (13, 10, 21), dtype=np.uint16)
    B = 8
    for b in [(0, 0, 0), (2, 1, 1), (1, 0, 1)]:
        reg = O.brick_region(lvl, B, b)
        x = np.clip(np.arange(B * b[0] - 1, B * b[0] + B + 1), 0, 20)
        y = np.clip(np.arange(B * b[1] - 1, B * b[1] + B + 1), 0, 9)
        z = np.clip(np.arange(B * b[2] - 1, B * b[2] + B + 1), 0, 12)
        assert np.array_equal(reg, lvl[np.ix_(z, y, x)])
        mn, mx = O.brick_minmax(lvl, B, b)
        assert (mn, mx) == (float(reg.min()), float(reg.max()))


def test_apron_sampling_equals_whole_level_sampling():
    """Sampling a node through its stored brick (core + apron) gives the same
    value as sampling the whole level, anywhere inside the node box."""
    rng = np.random.default_rng(7)
    vol = rng.integers(0, 255, (19, 23, 29), dtype=np.uint8)
    lv = O.pyramid(vol, 3)
    B = 8
    dims0 = (29, 23, 19)
    n_pts = 0
    for L in range(3):
        grid = O.brick_grid(dims0, B, L)
        for bz in range(grid[2]):
            for by in range(grid[1]):
                for bx in range(grid[0]):
                    b = (bx, by, bz)
                    lo, hi = O.node_box(dims0, B, L, b)
                    reg = O.brick_region(lv[L], B, b).astype(np.float64)
                    pts = lo + rng.uniform(0, 1, (300, 3)) * (hi - lo)
                    for p in pts:
                        q = p / 2 ** L - 0.5 - (np.array(b) * B - 1)  # local stored index
                        local = ndimage.map_coordinates(reg, [[q[2]], [q[1]], [q[0]]], order=1,
                                                        mode="nearest")[0]
                        assert abs(local - O.sample(lv[L], L, p)) <= 1e-9
                        n_pts += 1
    assert n_pts > 1000


# ------------------------------------------------------------- O5 trilinear
@pytest.mark.parametrize("L", [0, 1, 2])
def test_trilinear_matches_scipy_map_coordinates(L):
    rng = np.random.default_rng(11 + L)
    vol = rng.integers(0, 65535, (12, 9, 15), dtype=np.uint16)
    lv = O.pyramid(vol, 3)[L].astype(np.float64)
    dims0 = np.array([15, 9, 12], dtype=np.float64)
    pts = rng.uniform(-3, 1, (500, 3)) * 0 + rng.uniform(-0.2, 1.2, (500, 3)) * dims0
    for p in pts:
        q = p / 2 ** L - 0.5
        ref = ndimage.map_coordinates(lv, [[q[2]], [q[1]], [q[0]]], order=1, mode="nearest")[0]
        got = O.sample(O.pyramid(vol, 3)[L], L, p)
        assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref))


def test_trilinear_reproduces_voxel_values_at_centres():
    vol = np.arange(4 * 5 * 6, dtype=np.uint16).reshape(4, 5, 6)
    for (i, j, k) in [(0, 0, 0), (5, 4, 3), (2, 3, 1)]:
        assert O.sample(vol, 0, (i + 0.5, j + 0.5, k + 0.5)) == vol[k, j, i]


# ------------------------------------------------------------------- O4 TF
def test_tf_matches_numpy_interp():
    rng = np.random.default_rng(2)
    tf = rng.uniform(0, 1, (256, 4))
    lo, hi = 100.0, 60000.0
    for v in np.concatenate([rng.uniform(-1000, 70000, 400), [lo, hi, 100.0001, 59999.9]]):
        u = (v - lo) / (hi - lo) * 255
        ref = np.array([np.interp(u, np.arange(256), tf[:, c]) for c in range(4)])
        assert np.allclose(O.tf_eval(tf, lo, hi, v), ref, rtol=0, atol=1e-13)


def test_identity_tf_is_identity():
    tf = gen.tf_identity()
    for v in [0.0, 63.75, 127.5, 200.25, 255.0]:
        assert np.allclose(O.tf_eval(tf, 0, 255, v), v / 255.0, atol=1e-15)


# ------------------------------------------------------------- O6 / O7 rays
def test_centre_ray_of_odd_symmetric_view_is_forward():
    eye = np.array([30.0, 4.5, 4.5])
    v = gen.view(gen.look_at(eye, (4.5, 4.5, 4.5)), 5, 7, 0.3, 0.2)
    e, d = O.ray(v, 2, 3)
    assert np.array_equal(e, eye)
    assert np.array_equal(d, [-1.0, 0.0, 0.0])


def test_ray_angles_and_top_row():
    m = gen.look_at((0, 0, 0), (0, 1, 0))
    v = gen.view(m, 64, 48, 0.4, 0.7)
    for (x, y) in [(0, 0), (63, 47), (10, 40), (31, 0)]:
        e, d = O.ray(v, x, y)
        assert abs(np.linalg.norm(d) - 1) < 1e-15
        tx = -0.7 + (x + 0.5) / 64 * 1.4
        ty = 0.4 - (y + 0.5) / 48 * 0.8
        # angle to the optical axis (world +y) from the image-plane tangents
        ang = math.atan(math.hypot(tx, ty))
        assert abs(math.acos(np.clip(d[1], -1, 1)) - ang) < 1e-12
        # row 0 is the top: positive component along the camera up (+z)
        assert (d[2] > 0) == (ty > 0)
        # right half of the image is towards camera right
        assert (np.dot(d, m[:3, 0]) > 0) == (tx > 0)


def _march(dims, e, d, t_max, n=200001):
    t = np.linspace(0, t_max, n)
    p = e[None, :] + t[:, None] * d[None, :]
    ins = np.all((p >= 0) & (p <= np.asarray(dims, dtype=np.float64)), axis=1)
    return t, ins


def test_entry_exit_against_brute_force_marching():
    rng = np.random.default_rng(4)
    dims = (30, 20, 10)
    for _ in range(200):
        e = rng.uniform(-40, 70, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        hit, tn, tf = O.entry_exit(dims, e, d)
        t, ins = _march(dims, e, d, 200.0)
        dt = t[1] - t[0]
        if not ins.any():
            assert not hit or tf - tn < 2 * dt
            continue
        assert hit
        assert abs(t[ins][0] - tn) <= dt and abs(t[ins][-1] - tf) <= dt


def test_entry_exit_axis_parallel_rays():
    dims = (8, 8, 8)
    # eye inside the slab in y, z: unbounded there, bounded by x
    hit, tn, tf = O.entry_exit(dims, (20.0, 4.0, 4.0), (-1.0, 0.0, 0.0))
    assert hit and tn == 12.0 and tf == 20.0
    # eye exactly on a face plane counts as inside the slab
    hit, tn, tf = O.entry_exit(dims, (20.0, 8.0, 0.0), (-1.0, 0.0, 0.0))
    assert hit and (tn, tf) == (12.0, 20.0)
    # outside the slab: miss
    hit, _, _ = O.entry_exit(dims, (20.0, 8.5, 4.0), (-1.0, 0.0, 0.0))
    assert not hit
    # eye inside the volume: entry at t = 0
    hit, tn, tf = O.entry_exit(dims, (2.0, 3.0, 4.0), (0.0, 0.0, 1.0))
    assert hit and tn == 0.0 and tf == 4.0
    # pointing away
    hit, _, _ = O.entry_exit(dims, (20.0, 4.0, 4.0), (1.0, 0.0, 0.0))
    assert not hit


# ---------------------------------------------------------------- O8 LOD cut
def _brute_cut(dims0, B, levels, view, tau, bias, lod):
    e = np.asarray(view["cam_to_world"])[:3, 3]
    K = O.lod_k(view, tau)
    grids = [O.brick_grid(dims0, B, L) for L in range(levels)]

    def acc(L, b):
        return O.node_accept(dims0, B, e, K, bias, L, b) if lod else L == bias

    out = []
    for L in range(bias, levels):
        g = grids[L]
        for bz in range(g[2]):
            for by in range(g[1]):
                for bx in range(g[0]):
                    if not acc(L, (bx, by, bz)):
                        continue
                    anc_rejected = all(not acc(A, (bx >> (A - L), by >> (A - L), bz >> (A - L)))
                                       for A in range(L + 1, levels))
                    if anc_rejected:
                        out.append(O.node_id(L, bx, by, bz))
    return np.sort(np.array(out, dtype=np.uint64))


def test_cut_equals_brute_force_enumeration_on_tiny_trees():
    rng = np.random.default_rng(10)
    dims0, B, levels = (8, 8, 8), 2, 3
    for i in range(2000):
        eye = rng.uniform(-20, 28, 3)
        v = gen.view(gen.look_at(eye, rng.uniform(0, 8, 3)), int(rng.integers(1, 40)),
                     int(rng.integers(1, 40)), float(rng.uniform(0.05, 2.0)))
        tau = float(rng.uniform(0.2, 8))
        bias = int(rng.integers(0, levels))
        lod = bool(rng.integers(0, 4))
        got = O.lod_cut(dims0, B, levels, v, tau, bias, lod)
        assert np.array_equal(got, _brute_cut(dims0, B, levels, v, tau, bias, lod)), i


def test_cut_equals_brute_force_ragged_dims():
    rng = np.random.default_rng(12)
    dims0, B, levels = (13, 7, 10), 2, 4
    for i in range(300):
        eye = rng.uniform(-10, 25, 3)
        v = gen.view(gen.look_at(eye, (6, 3, 5)), 30, 20, float(rng.uniform(0.1, 1.0)))
        tau = float(rng.uniform(0.5, 6))
        got = O.lod_cut(dims0, B, levels, v, tau, 0, True)
        assert np.array_equal(got, _brute_cut(dims0, B, levels, v, tau, 0, True)), i


def _cover_count(dims0, B, cut):
    cnt = np.zeros(dims0[::-1], dtype=np.int32)
    for L, bx, by, bz in O.node_decode(cut):
        lo, hi = O.node_box(dims0, B, int(L), (int(bx), int(by), int(bz)))
        lo, hi = lo.astype(int), hi.astype(int)
        cnt[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += 1
    return cnt


@pytest.mark.parametrize("dims0,B,levels", [((64, 48, 40), 4, 4), ((37, 29, 23), 8, 3),
                                             ((16, 16, 16), 2, 4)])
def test_cut_partitions_the_volume(dims0, B, levels):
    rng = np.random.default_rng(21)
    for _ in range(40):
        eye = rng.uniform(-30, 90, 3)
        v = gen.view(gen.look_at(eye, np.asarray(dims0) / 2), 200, 160, 0.6)
        cut = O.lod_cut(dims0, B, levels, v, float(rng.uniform(0.3, 30)), 0, True)
        assert np.all(_cover_count(dims0, B, cut) == 1)


def test_accept_threshold_matches_angular_size_definition():
    """A node whose closest face is at distance D along x is accepted exactly
    when its voxel edge 2^L subtends no more than tau pixels: 2^L <= tau
    theta D with theta = (tan_top - tan_bottom) / H."""
    dims0, B = (256, 256, 256), 16
    H, tt = 100, 0.5
    theta = 2 * tt / H
    for L, tau in [(1, 1.0), (2, 1.0), (3, 2.5), (4, 0.7)]:
        D = 2 ** L / (tau * theta)  # exact threshold distance
        b = (0, 0, 0)
        lo, hi = O.node_box(dims0, B, L, b)
        for dist, expect in [(D * (1 + 1e-9), True), (D * (1 - 1e-9), False)]:
            eye = np.array([hi[0] + dist, 5.0, 5.0])
            v = gen.view(gen.look_at(eye, (0, 5, 5)), 80, H, tt)
            K = O.lod_k(v, tau)
            assert O.node_accept(dims0, B, eye, K, 0, L, b) == expect
    # eye inside the node box: distance 0, refine (unless at the bias level)
    v = gen.view(gen.look_at((5, 5, 5), (0, 0, 0)), 8, 8, 0.5)
    K = O.lod_k(v, 1.0)
    assert not O.node_accept(dims0, B, (5.0, 5.0, 5.0), K, 0, 3, (0, 0, 0))
    assert O.node_accept(dims0, B, (5.0, 5.0, 5.0), K, 3, 3, (0, 0, 0))


def test_cut_far_eye_is_top_level_and_near_eye_refines():
    dims0, B, levels = (128, 128, 128), 8, 5
    far = gen.view(gen.look_at((1e7, 64, 64), (64, 64, 64)), 64, 64, 0.5)
    cut = O.lod_cut(dims0, B, levels, far, 1.0, 0, True)
    assert set(O.node_decode(cut)[:, 0]) == {levels - 1}
    near = gen.view(gen.look_at((64, 64, 64), (0, 0, 0)), 64, 64, 1.0)
    cut = O.lod_cut(dims0, B, levels, near, 1.0, 0, True)
    lv = O.node_decode(cut)
    # the eye's own node is at level 0, coarser levels further away
    assert any((r[0] == 0 and r[1] * 8 <= 64 < r[1] * 8 + 8) for r in lv)
    assert lv[:, 0].max() > 0


# ----------------------------------------------------------- O9 empty flags
def test_empty_flags_conservative_and_exact():
    rng = np.random.default_rng(8)
    vol = np.zeros((16, 16, 16), dtype=np.uint8)
    vol[2:5, 3:6, 1:4] = 200  # one bright region inside brick (0,0,0)
    vol[12, 12, 12] = 30
    tf = np.zeros((256, 4))
    tf[100:, 3] = 0.5  # transparent below entry 100
    tf[:, :3] = rng.uniform(0, 1, (256, 3))
    sc = O.Scene([vol], 8, 2, [tf], [(0, 255)])
    ids = np.array([O.node_id(0, x, y, z) for z in range(2) for y in range(2) for x in range(2)],
                   dtype=np.uint64)
    emp = sc.empty(ids)
    exp = [not (x == 0 and y == 0 and z == 0) for z in range(2) for y in range(2)
           for x in range(2)]
    assert list(emp) == exp
    # guard band: a max two entries below the first opaque entry is not empty
    vol2 = np.zeros((8, 8, 8), dtype=np.uint8)
    vol2[0, 0, 0] = 98
    sc2 = O.Scene([vol2], 8, 1, [tf], [(0, 255)])
    assert not sc2.empty(np.array([O.node_id(0, 0, 0, 0)], dtype=np.uint64))[0]
    vol2[0, 0, 0] = 97
    sc2 = O.Scene([vol2], 8, 1, [tf], [(0, 255)])
    assert sc2.empty(np.array([O.node_id(0, 0, 0, 0)], dtype=np.uint64))[0]


# ---------------------------------------------------------------- rendering
def test_empty_volume_returns_background_exactly():
    vol = np.zeros((20, 24, 28), dtype=np.uint16)
    tf = gen.tf_hot()
    for skip in (0, 1):
        for lod in (0, 1):
            sc = O.Scene([vol], 4, 3, [tf], [(0, 65535)])
            v = gen.view(gen.look_at((-30, 50, 40), (14, 12, 10)), 33, 21, 0.4)
            bg = (0.1, 0.25, 0.5, 0.75)
            out = sc.render(v, params(bg=bg, skip_empty=skip, lod=lod, ert=0.99))["rgba"]
            assert np.array_equal(out, np.broadcast_to(np.array(bg), out.shape))


@pytest.mark.parametrize("B,levels", [(32, 1), (8, 3), (4, 4)])
def test_constant_medium_closed_form_every_lod(B, levels):
    """A constant volume gives A = 1 - exp(-rho L) and C = rgb A along every
    ray (L = chord length) for every cut, level and bricking."""
    vol = np.full((24, 32, 28), 77, dtype=np.uint8)
    rgb, rho = np.array([0.3, 0.6, 0.9]), 0.037
    tf = gen.tf_constant(rgb, rho)
    sc = O.Scene([vol], B, levels, [tf], [(0, 255)])
    views = [gen.view(gen.look_at((-20, 70, 50), (14, 16, 12)), 23, 17, 0.5),
             gen.view(gen.look_at((10, 12, 9), (40, -3, 5)), 15, 19, 1.2)]  # eye inside
    for v in views:
        for bias in range(levels):
            for lod in (0, 1):
                for tau in (0.5, 4.0):
                    p = params(bias=bias, lod=lod, tau=tau, skip_empty=0)
                    out = sc.render(v, p)["rgba"]
                    for y in range(v["height"]):
                        for x in range(v["width"]):
                            e, d = O.ray(v, x, y)
                            hit, tn, tf_ = O.entry_exit((28, 32, 24), e, d)
                            A = 1 - math.exp(-rho * (tf_ - tn)) if hit else 0.0
                            assert abs(out[y, x, 3] - A) < 1e-12
                            assert np.allclose(out[y, x, :3], rgb * A, atol=1e-12)


def test_constant_medium_early_termination_closed_form():
    vol = np.full((200, 16, 16), 10, dtype=np.uint8)  # long in z
    rho = 0.2
    tf = gen.tf_constant((1.0, 0.5, 0.25), rho)
    sc = O.Scene([vol], 16, 1, [tf], [(0, 255)])
    v = gen.view(gen.look_at((8.0, 8.0, 500.0), (8.0, 8.0, 0.0), up=(0, 1, 0)), 3, 3, 0.001)
    out = sc.render(v, params(ert=0.99), count=True)
    # centre ray runs along -z through 200 voxels; steps of 0.5
    k = math.ceil(math.log(100.0) / (rho * 0.5))  # first k with 1-exp(-rho k/2) >= 0.99
    A = 1 - math.exp(-rho * 0.5 * k)
    assert out["nsamp"][1, 1] == k
    assert abs(out["rgba"][1, 1, 3] - A) < 1e-12
    assert np.allclose(out["rgba"][1, 1, :3], np.array([1, 0.5, 0.25]) * A, atol=1e-12)


def test_single_bright_voxel_hand_computed():
    """One voxel of 255 in a zero 9^3 volume, identity transfer function,
    eye on the +x axis through the voxel centre. The centre ray meets the
    tent of the voxel at 4 samples with densities 1/4, 3/4, 3/4, 1/4."""
    vol = np.zeros((9, 9, 9), dtype=np.uint8)
    vol[4, 4, 4] = 255
    sc = O.Scene([vol], 16, 1, [gen.tf_identity()], [(0, 255)])
    v = gen.view(gen.look_at((40.0, 4.5, 4.5), (4.5, 4.5, 4.5)), 3, 5, 0.01)
    out = sc.render(v, params(ert=0.99, skip_empty=0), count=True)
    # the closed form written out by hand: 18 samples on the chord, four of
    # them inside the tent; colour = density under the identity table
    C, T = 0.0, 1.0
    for r in (0.25, 0.75, 0.75, 0.25):
        a = 1 - math.exp(-r * 0.5)
        C += T * a * r
        T *= 1 - a
    assert out["nsamp"][2, 1] == 18
    assert abs(out["rgba"][2, 1, 3] - (1 - T)) < 1e-15
    assert np.allclose(out["rgba"][2, 1, :3], C, atol=1e-15)
    assert abs((1 - T) - (1 - math.exp(-1.0))) < 1e-15


def _profile_volume():
    """Volume varying along x only (a 1D profile), constant in y and z."""
    rng = np.random.default_rng(30)
    prof = rng.integers(0, 65535, 40).astype(np.uint16)
    return np.broadcast_to(prof[None, None, :], (6, 6, 40)).copy(), prof


def test_compositing_equals_explicit_sum_and_back_to_front():
    """Front-to-back recursion equals the explicit sum T_k a_k c_k and the
    back-to-front 'over' recursion, with sample values from scipy and the
    table from numpy.interp (no early termination)."""
    vol, prof = _profile_volume()
    rng = np.random.default_rng(31)
    tf = gen.tf_random(rng)
    lo, hi = 1000.0, 64000.0
    sc = O.Scene([vol], 64, 1, [tf], [(lo, hi)])
    e = np.array([-7.25, 3.0, 3.0])
    v = gen.view(gen.look_at(e, (20.0, 3.0, 3.0)), 1, 1, 0.01)
    out = sc.render(v, params(skip_empty=0), count=True)
    # samples: chord [7.25, 47.25], steps 0.5 at midpoints
    t = 7.25 + 0.25 + 0.5 * np.arange(80)
    xs = e[0] + t
    vals = ndimage.map_coordinates(prof.astype(np.float64), [xs - 0.5], order=1, mode="nearest")
    u = (vals - lo) / (hi - lo) * 255
    c = np.stack([np.interp(u, np.arange(256), tf[:, k]) for k in range(4)], axis=1)
    a = 1 - np.exp(-c[:, 3] * 0.5)
    T = np.concatenate([[1.0], np.cumprod(1 - a)[:-1]])
    explicit = (T * a)[:, None] * c[:, :3]
    Cb = np.zeros(3)
    for k in reversed(range(80)):  # back to front: C <- a c + (1 - a) C
        Cb = a[k] * c[k, :3] + (1 - a[k]) * Cb
    assert out["nsamp"][0, 0] == 80
    assert np.allclose(out["rgba"][0, 0, :3], explicit.sum(0), atol=1e-12, rtol=0)
    assert np.allclose(out["rgba"][0, 0, :3], Cb, atol=1e-12, rtol=0)
    assert abs(out["rgba"][0, 0, 3] - (1 - np.prod(1 - a))) < 1e-12


def test_midpoint_rule_converges_to_emission_absorption_integral():
    """As the step shrinks the result approaches Eq. 2 of Sec 5.1 with the
    associated colour c = rho tau (computed by scipy.integrate.quad on the
    trilinear field), at second order."""
    vol, prof = _profile_volume()
    tf = gen.tf_identity()
    tf[:, 3] *= 0.2
    tf[:, 0] = np.sqrt(tf[:, 0])
    lo, hi = 0.0, 65535.0
    sc = O.Scene([vol], 64, 1, [tf], [(lo, hi)])
    e = np.array([-3.0, 3.0, 3.0])
    v = gen.view(gen.look_at(e, (20.0, 3.0, 3.0)), 1, 1, 0.01)

    def field(t):
        x = e[0] + t
        val = ndimage.map_coordinates(prof.astype(np.float64), [[x - 0.5]], order=1,
                                      mode="nearest")[0]
        u = (val - lo) / (hi - lo) * 255
        return np.interp(u, np.arange(256), tf[:, 0]), np.interp(u, np.arange(256), tf[:, 3])

    breaks = list(np.arange(3.5, 43.0, 1.0))
    tau_of = lambda s: integrate.quad(lambda t: field(t)[1], 3.0, s, points=[b for b in breaks if b < s], limit=200)[0]
    ref = integrate.quad(lambda t: field(t)[0] * field(t)[1] * math.exp(-tau_of(t)), 3.0, 43.0,
                         points=breaks, limit=400, epsabs=1e-13)[0]
    errs = []
    for step in (0.5, 0.25, 0.125, 0.0625):
        out = sc.render(v, params(step=step, skip_empty=0))
        errs.append(abs(out["rgba"][0, 0, 0] - ref))
    assert errs[-1] < 1e-4
    for a, b in zip(errs, errs[1:]):
        assert a / b > 3.0  # second order: ~4x per halving


def test_skip_empty_is_bit_identical():
    rng = np.random.default_rng(40)
    vol = gen.random_volume((40, 36, 44), 41, dtype=np.uint16)
    tf = gen.tf_hot(a_start=120)
    sc = O.Scene([vol], 8, 3, [tf], [(0, 65535)])
    for i in range(3):
        eye = rng.uniform(-60, 100, 3)
        v = gen.view(gen.look_at(eye, (22, 18, 20)), 31, 27, 0.5)
        p = params(ert=0.99, tau=float(rng.uniform(0.5, 3)))
        cut = sc.cut(v, p)
        emp = sc.empty(cut)
        assert emp.any() and not emp.all()
        a = sc.render(v, dict(p, skip_empty=1))["rgba"]
        b = sc.render(v, dict(p, skip_empty=0))["rgba"]
        assert np.array_equal(a, b)


def test_sort_last_split_and_composite_identity():
    """Rendering two halves of the cut separately and compositing them front
    over back (in the order the ray crosses the split plane) reproduces the
    full render."""
    vol = gen.random_volume((32, 32, 32), 50, dtype=np.uint8)
    tf = gen.tf_identity()
    tf[:, 3] *= 0.1
    sc = O.Scene([vol], 8, 3, [tf], [(0, 255)])
    v = gen.view(gen.look_at((-30, 45, 20), (16, 16, 16)), 21, 19, 0.6)
    p = params(skip_empty=0)
    cut = sc.cut(v, p)
    boxes = [O.node_box(sc.dims, 8, int(r[0]), tuple(int(x) for x in r[1:]))
             for r in O.node_decode(cut)]
    left = np.array([b[1][0] <= 16 for b in boxes])
    full = sc.render(v, p)["rgba"]
    f = sc.render(v, p, cut=cut[left], empty=np.zeros(left.sum(), bool))["rgba"]
    b = sc.render(v, p, cut=cut[~left], empty=np.zeros((~left).sum(), bool))["rgba"]
    # eye has x < 16: the left half is in front for every ray
    comp = f + (1 - f[..., 3:4]) * b
    assert np.allclose(comp, full, atol=1e-12, rtol=0)


def test_one_nonzero_channel_reduces_to_single_channel():
    rng = np.random.default_rng(60)
    a = gen.random_volume((20, 22, 24), 61, dtype=np.uint16)
    b = gen.random_volume((20, 22, 24), 62, dtype=np.uint16)
    tf = gen.tf_random(rng)
    zero = tf.copy()
    zero[:, 3] = 0.0
    v = gen.view(gen.look_at((-20, 40, 30), (12, 11, 10)), 17, 13, 0.5)
    p = params(ert=0.99)
    single = O.Scene([a], 8, 2, [tf], [(0, 65535)]).render(v, p)["rgba"]
    multi = O.Scene([b, a], 8, 2, [zero, tf], [(0, 65535), (0, 65535)]).render(v, p)["rgba"]
    assert np.allclose(single, multi, atol=1e-14, rtol=0)


def test_multichannel_additive_extinction():
    """Two channels with constant values: rho = rho1 + rho2 and the colour
    is the extinction-weighted mean."""
    a = np.full((10, 10, 10), 50, dtype=np.uint8)
    b = np.full((10, 10, 10), 90, dtype=np.uint8)
    t1 = gen.tf_constant((1.0, 0.0, 0.0), 0.05)
    t2 = gen.tf_constant((0.0, 0.0, 1.0), 0.15)
    sc = O.Scene([a, b], 4, 2, [t1, t2], [(0, 255), (0, 255)])
    v = gen.view(gen.look_at((5.0, 5.0, 40.0), (5.0, 5.0, 0.0), up=(0, 1, 0)), 1, 1, 0.01)
    out = sc.render(v, params(skip_empty=0))["rgba"][0, 0]
    A = 1 - math.exp(-0.2 * 10)
    assert abs(out[3] - A) < 1e-12
    assert np.allclose(out[:3], np.array([0.25, 0.0, 0.75]) * A, atol=1e-12)


def test_depth_is_first_sample_reaching_half_alpha():
    vol = np.zeros((64, 8, 8), dtype=np.uint8)
    vol[:24] = 255  # bright for z < 24, the far side from the eye
    tf = gen.tf_constant((1, 1, 1), 0.0)
    tf[200:, 3] = 0.3
    sc = O.Scene([vol], 8, 1, [tf], [(0, 255)])
    v = gen.view(gen.look_at((4.0, 4.0, 100.0), (4.0, 4.0, 0.0), up=(0, 1, 0)), 1, 1, 0.01)
    out = sc.render(v, params(ert=0.99, skip_empty=0), depth=True)
    # entry at z = 64 (t = 36); the trilinear edge between centres 23.5 and
    # 24.5 gives value 255 * clip(24.5 - z, 0, 1) at z = 100 - t
    t = 36.0 + 0.25 + 0.5 * np.arange(128)
    val = 255 * np.clip(24.5 - (100.0 - t), 0, 1)
    rho = np.interp(val, np.arange(256), tf[:, 3])
    A = 1 - np.exp(-np.cumsum(rho * 0.5))
    k = int(np.argmax(A >= 0.5))
    assert k > 80
    assert out["depth"][0, 0] == t[k]
