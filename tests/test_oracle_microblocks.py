"""Pin of the oracle's micro-block counter (the traffic the method needs).

The oracle counts, per channel and level, the distinct 4^3 voxel blocks
that the trilinear stencils of the samples it takes read. That count is the
algorithmic byte figure of the ray caster's memory roofline, so it is
pinned here against an enumeration written from the definitions alone:
rays through pixel centres (Sec 5.1), the node intervals of the cut taken
front to back with the ray restarted in every block (Sec 5.2), samples at
the midpoints of steps of 0.5 x 2^L level-0 units (the last one partial),
and for each sample the eight voxels of its trilinear stencil
(Sec 5.1, hardware-style trilinear filtering: voxel centres at +1/2,
indices clamped to the level), each mapped to its block by integer
division by 4. Early termination and skipping are switched off, so the set
of samples depends on geometry only. Runs on the CPU.
"""
import math

import numpy as np
import pytest

import gen
import oracle as O

O.build()

NO_ERT = 2.0


def _ray(view, x, y):
    """Eye and unit direction of pixel (x, y): centre tangents, camera -z."""
    m = np.asarray(view["cam_to_world"], dtype=np.float64).reshape(4, 4)
    sx = view["tan_left"] + (x + 0.5) / view["width"] * (view["tan_right"] - view["tan_left"])
    sy = view["tan_top"] - (y + 0.5) / view["height"] * (view["tan_top"] - view["tan_bottom"])
    w = m[:3, :3] @ np.array([sx, sy, -1.0])
    return m[:3, 3].copy(), w / np.linalg.norm(w)


def _box(e, d, lo, hi):
    """Parameter interval of the ray inside the box [lo, hi] (or None)."""
    t0, t1 = -np.inf, np.inf
    for i in range(3):
        if d[i] == 0.0:
            if not (lo[i] <= e[i] <= hi[i]):
                return None
            continue
        a, b = (lo[i] - e[i]) / d[i], (hi[i] - e[i]) / d[i]
        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
    return (t0, t1) if t0 < t1 else None


def _level_dims(dims0, L):
    n = list(dims0)
    for _ in range(L):
        n = [(v + 1) // 2 for v in n]
    return n


def _enumerate(dims0, B, view, cut_ids, step, pixels):
    """(sample count, {(L, bx, by, bz)} blocks) from the definitions."""
    blocks = set()
    count = 0
    lv = [int(i) >> 60 for i in cut_ids]
    bb = [((int(i) >> 40) & 0xFFFFF, (int(i) >> 20) & 0xFFFFF, int(i) & 0xFFFFF)
          for i in cut_ids]
    for (x, y) in pixels:
        e, d = _ray(view, x, y)
        whole = _box(e, d, np.zeros(3), np.asarray(dims0, dtype=np.float64))
        if whole is None:
            continue
        tn, tf = max(whole[0], 0.0), whole[1]
        if not tn < tf:
            continue
        segs = []
        for L, b in zip(lv, bb):
            w = B * 2 ** L
            lo = np.array([w * b[i] for i in range(3)], dtype=np.float64)
            hi = np.array([min(w * (b[i] + 1), dims0[i]) for i in range(3)], dtype=np.float64)
            iv = _box(e, d, lo, hi)
            if iv is None:
                continue
            t0, t1 = max(iv[0], tn), min(iv[1], tf)
            if t0 < t1:
                segs.append((t0, t1, L))
        segs.sort()
        for t0, t1, L in segs:
            D = step * 2.0 ** L
            n = math.ceil((t1 - t0) / D)
            nl = _level_dims(dims0, L)
            for k in range(n):
                s = min(D, (t1 - t0) - k * D)
                p = e + (t0 + k * D + 0.5 * s) * d
                count += 1
                q = p / 2.0 ** L - 0.5
                i0 = np.floor(q).astype(np.int64)
                for dz in (0, 1):
                    for dy in (0, 1):
                        for dx in (0, 1):
                            v = [min(max(i0[0] + dx, 0), nl[0] - 1),
                                 min(max(i0[1] + dy, 0), nl[1] - 1),
                                 min(max(i0[2] + dz, 0), nl[2] - 1)]
                            blocks.add((L, v[0] // 4, v[1] // 4, v[2] // 4))
    return count, blocks


def _oracle_blocks(out, channels, levels):
    per_channel = []
    for c in range(channels):
        s = set()
        for L in range(levels):
            bm = out["microblocks"][c * levels + L]
            for z, y, x in zip(*np.nonzero(bm)):
                s.add((L, int(x), int(y), int(z)))
        per_channel.append(s)
    return per_channel


CASES = [
    # dims (x, y, z), brick, levels, eye, lod, bias, channels, tau (pixels)
    ((29, 22, 17), 8, 3, (-9.0, 40.0, 30.0), 1, 0, 1, 1.0),
    ((29, 22, 17), 8, 3, (60.0, -25.0, 8.0), 0, 0, 1, 1.0),
    ((29, 22, 17), 8, 3, (60.0, -25.0, 8.0), 0, 1, 2, 1.0),
    ((13, 31, 9), 4, 4, (6.0, 15.0, 4.0), 1, 0, 1, 6.0),   # eye inside the volume
    ((13, 31, 9), 4, 4, (-30.0, 70.0, -20.0), 1, 1, 1, 1.0),
    # level dims divisible by 4: the stencils at the far faces clamp into
    # the last block
    ((32, 24, 16), 8, 3, (50.0, 45.0, 30.0), 0, 0, 1, 1.0),
    ((32, 24, 16), 8, 3, (50.0, 45.0, 30.0), 0, 1, 1, 1.0),
]


@pytest.mark.parametrize("dims0,B,levels,eye,lod,bias,channels,tau", CASES)
def test_microblocks_equal_brute_force_stencil_enumeration(dims0, B, levels, eye, lod, bias,
                                                           channels, tau):
    rng = np.random.default_rng(sum(dims0) + B + channels)
    vols = [rng.integers(0, 256, dims0[::-1], dtype=np.uint8) for _ in range(channels)]
    tfs = [gen.tf_random(rng) for _ in range(channels)]
    sc = O.Scene(vols, B, levels, tfs, [(0, 255)] * channels)
    centre = [0.5 * v for v in dims0]
    view = gen.view(gen.look_at(eye, centre), 23, 19, math.tan(math.radians(35)))
    p = {"step": 0.5, "ert": NO_ERT, "tau": tau, "bias": bias, "lod": lod, "skip_empty": 0}
    cut = sc.cut(view, p)
    if lod:
        assert len({int(i) >> 60 for i in cut}) >= 2, "want a cut that mixes levels"
    pixels = [(x, y) for y in range(view["height"]) for x in range(view["width"])]
    out = sc.render(view, p, microblocks=True)
    count, blocks = _enumerate(dims0, B, view, cut, p["step"], pixels)
    assert out["total_samples"] == count
    assert count > 0
    for c, got in enumerate(_oracle_blocks(out, channels, levels)):
        assert got == blocks, "channel %d: %d extra, %d missing" % (
            c, len(got - blocks), len(blocks - got))


def test_microblocks_hand_count_axis_aligned_ray():
    """One ray along +x at y = 4.6, z = 3.6 through a 16 x 8 x 8 level-0
    volume (one brick, dense): samples at x = 0.25, 0.75, ..., 15.75 give
    stencil x-voxels 0..15 (blocks 0..3), y-voxels 4, 5 (block 1) and
    z-voxels 3, 4 (blocks 0, 1): 4 x 1 x 2 = 8 blocks, 32 samples."""
    vol = np.zeros((8, 8, 16), np.uint8)
    sc = O.Scene([vol], 16, 1, [gen.tf_identity()], [(0, 255)])
    m = np.eye(4)
    # camera -z looks along world +x; camera y is world y
    m[:3, :3] = [[0.0, 0.0, -1.0], [0.0, 1.0, 0.0], [1.0, 0.0, 0.0]]
    m[:3, 3] = (-10.0, 4.6, 3.6)
    view = gen.view(m, 1, 1, 1e-3)
    e, d = _ray(view, 0, 0)
    assert np.allclose(d, (1.0, 0.0, 0.0)) and np.allclose(e, (-10.0, 4.6, 3.6))
    p = {"step": 0.5, "ert": NO_ERT, "tau": 1.0, "bias": 0, "lod": 0, "skip_empty": 0}
    out = sc.render(view, p, microblocks=True)
    assert out["total_samples"] == 32
    bm = out["microblocks"][0]
    assert bm.shape == (2, 2, 4)  # (z, y, x) blocks of a 16 x 8 x 8 level
    want = np.zeros_like(bm)
    want[0:2, 1, 0:4] = 1
    assert np.array_equal(bm, want)
