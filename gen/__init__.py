"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds none of the ray caster's arithmetic: it only produces
volumes, camera poses and transfer-function tables. The paper's datasets
(Drosophila brain, mouse vasculature, zebrafish musculature, multi-TB
volumes) are not available, so these workloads stand in for them:

* ``blobs128``: a 128^3 uint8 volume of 8 Gaussian blobs plus uniform noise
  (the small plain-ray-cast workload).
* ``tubes``: a 2048^3 uint16 volume of 400 branching Gaussian tubes over a
  Poisson(200) background (the bricked stereo workload), evaluated by the
  HIP/CPU generator in ``gen/gen.hip``.
* ``cells``: 3 channels of 1024x1024x512 uint16 moving Gaussian cells over a
  smooth background, per timepoint (the multichannel time-series workload).
* small random volumes for the parity tests.

Camera conventions: world units are level-0 voxels with the volume box at
[0, dims]; a camera looks down its own -z axis; ``cam_to_world`` is a
row-major 4x4 matrix whose last column is the eye position.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

# ------------------------------------------------------------------ cameras


def look_at(eye, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Row-major camera-to-world matrix looking from ``eye`` at ``target``."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    if np.linalg.norm(r) < 1e-9:  # looking along up: pick another up
        r = np.cross(f, np.array([0.0, 1.0, 0.0]))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    m = np.eye(4)
    m[:3, 0], m[:3, 1], m[:3, 2], m[:3, 3] = r, u, -f, eye
    return m


def view(cam_to_world, width, height, tan_top, tan_right=None, tan_left=None,
         tan_bottom=None) -> dict:
    if tan_right is None:
        tan_right = tan_top * width / height
    return {"cam_to_world": np.asarray(cam_to_world, dtype=np.float64).reshape(4, 4),
            "tan_left": -tan_right if tan_left is None else tan_left,
            "tan_right": tan_right,
            "tan_bottom": -tan_top if tan_bottom is None else tan_bottom,
            "tan_top": tan_top, "width": int(width), "height": int(height)}


def stereo(head, target, ipd, width, height, tan_top, tan_right, up=(0, 0, 1)):
    """Left and right eye views: parallel axes, eyes at head -/+ ipd/2 along
    the head's right vector (an HMD pair)."""
    m = look_at(head, target, up)
    r = m[:3, 0]
    out = []
    for s in (-0.5, 0.5):
        mm = m.copy()
        mm[:3, 3] = np.asarray(head, dtype=np.float64) + s * ipd * r
        out.append(view(mm, width, height, tan_top, tan_right))
    return out


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


# ---------------------------------------------------------- transfer tables


def tf_identity(n=256) -> np.ndarray:
    """Linear ramp: entry k = k/(n-1) in every channel (Sec 8 linear map)."""
    k = np.arange(n, dtype=np.float64) / (n - 1)
    return np.stack([k, k, k, k], axis=1)


def tf_hot(n=256, a_start=5, a_max=0.25) -> np.ndarray:
    """'Hot' palette with an extinction ramp that is zero below a_start."""
    k = np.arange(n, dtype=np.float64)
    s = k / (n - 1)
    rgb = np.stack([np.minimum(1.0, 3 * s), np.clip(3 * s - 1, 0, 1), np.clip(3 * s - 2, 0, 1)],
                   axis=1)
    a = np.where(k < a_start, 0.0, a_max * (k - a_start) / (n - 1 - a_start))
    return np.concatenate([rgb, a[:, None]], axis=1)


def tf_tint(tint, n=256, a_start=12, a_max=0.15) -> np.ndarray:
    k = np.arange(n, dtype=np.float64)
    s = k / (n - 1)
    rgb = np.outer(s, np.asarray(tint, dtype=np.float64))
    a = np.where(k < a_start, 0.0, a_max * (k - a_start) / (n - 1 - a_start))
    return np.concatenate([rgb, a[:, None]], axis=1)


def tf_constant(rgb, rho, n=256) -> np.ndarray:
    out = np.zeros((n, 4))
    out[:, :3] = rgb
    out[:, 3] = rho
    return out


def tf_random(rng, n=256, zero_below=0) -> np.ndarray:
    t = rng.uniform(0, 1, (n, 4))
    t[:, 3] *= 0.3
    t[:zero_below, 3] = 0.0
    return t


# ------------------------------------------------------------------ volumes


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def blobs(shape_zyx, n_blobs, seed, sigma=(6.0, 20.0), amp=(100.0, 255.0), noise=16.0,
          dtype=np.uint8, vmax=255):
    """Sum of isotropic Gaussian blobs at voxel centres plus uniform noise.

    Blob parameters are drawn first (centre, sigma, amplitude per blob), then
    the noise array in [z, y, x] order; values are rounded and clipped.
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape_zyx
    dims = np.array([nx, ny, nz], dtype=np.float64)
    cen = rng.uniform(0, 1, (n_blobs, 3)) * dims
    sig = rng.uniform(sigma[0], sigma[1], n_blobs)
    am = rng.uniform(amp[0], amp[1], n_blobs)
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                          indexing="ij")
    f = np.zeros(shape_zyx, dtype=np.float64)
    for c, s, a in zip(cen, sig, am):
        r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
        f += a * np.exp(-r2 / (2 * s * s))
    f += rng.uniform(0, noise, shape_zyx)
    return np.clip(np.rint(f), 0, vmax).astype(dtype)


def blobs128() -> np.ndarray:
    """The 128^3 uint8 plain-ray-cast volume (seed 1001)."""
    return blobs((128, 128, 128), 8, 1001)


def blobs128_view() -> dict:
    """256x256, 60-degree FOV, eye at 2.5 volume diagonals from the centre."""
    c = np.array([64.0, 64.0, 64.0])
    eye = c + 2.5 * (128 * math.sqrt(3)) * unit((1.0, 0.7, 0.4))
    return view(look_at(eye, c), 256, 256, math.tan(math.radians(30)))


def random_volume(shape_zyx, seed, dtype=np.uint16, n_blobs=12):
    """Small structured volume (blobs over noise) for parity tests."""
    vmax = 255 if dtype == np.uint8 else 65535
    sc = vmax / 255.0
    nz, ny, nx = shape_zyx
    smin = max(1.0, min(shape_zyx) / 16)
    return blobs(shape_zyx, n_blobs, seed, sigma=(smin, 3 * smin),
                 amp=(60 * sc, 255 * sc), noise=20 * sc, dtype=dtype, vmax=vmax)


def orbit_views(center, radius_range, n, seed, width, height, tan_top=math.tan(math.radians(30)),
                stereo_ipd=None):
    """Seeded poses on a sphere around ``center`` (direction uniform on S^2,
    redrawn near the poles), looking at the centre."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        if abs(v[2]) > 0.99:
            continue
        r = rng.uniform(*radius_range)
        eye = np.asarray(center, dtype=np.float64) + r * v
        w = width if np.isscalar(width) else int(rng.integers(width[0], width[1] + 1))
        h = height if np.isscalar(height) else int(rng.integers(height[0], height[1] + 1))
        if stereo_ipd is None:
            out.append(view(look_at(eye, center), w, h, tan_top))
        else:
            out.append(stereo(eye, center, stereo_ipd, w, h, tan_top, tan_top * w / h))
    return out


# --------------------------------------------------- tube volume (2048^3)

TUBES_DIMS = (2048, 2048, 2048)
TUBES_BRICK = 64
TUBES_LEVELS = 6


def tube_geometry(seed=1002, n_filaments=400, dims=TUBES_DIMS, step=4.0, noise=0.15,
                  length=(256.0, 2048.0), p_branch=0.004, max_branches=8, radius=(1.0, 6.0),
                  intensity=(2000.0, 60000.0)):
    """Branching random-walk filaments as polyline segments.

    Returns float64 arrays p0 (M,3), p1 (M,3), radius (M,), intensity (M,)
    and int64 branch id (M,). Each filament draws its root, heading, radius
    and intensity; each branch walks ``length`` voxels in steps of 4 with a
    Gaussian heading perturbation and may spawn side branches.
    """
    rng = np.random.default_rng(seed)
    dims = np.asarray(dims, dtype=np.float64)
    P0, P1, R, I, BID = [], [], [], [], []
    bid = 0
    for _ in range(n_filaments):
        root = rng.uniform(0, 1, 3) * dims
        h = rng.normal(size=3)
        h /= np.linalg.norm(h)
        r = rng.uniform(*radius)
        amp = rng.uniform(*intensity)
        queue = [(root, h)]
        spawned = 0
        while queue:
            p, d = queue.pop(0)
            n_steps = int(rng.uniform(*length) / step)
            g = rng.normal(size=(n_steps, 3))
            u = rng.uniform(size=n_steps)
            pts = [p]
            for s in range(n_steps):
                gp = g[s] - np.dot(g[s], d) * d
                d = d + noise * gp
                d /= np.linalg.norm(d)
                p = p + step * d
                pts.append(p)
                if u[s] < p_branch and spawned < max_branches:
                    nd = d + 0.6 * rng.normal(size=3)
                    queue.append((p, nd / np.linalg.norm(nd)))
                    spawned += 1
            pts = np.array(pts)
            P0.append(pts[:-1])
            P1.append(pts[1:])
            R.append(np.full(len(pts) - 1, r))
            I.append(np.full(len(pts) - 1, amp))
            BID.append(np.full(len(pts) - 1, bid, dtype=np.int64))
            bid += 1
    return (np.concatenate(P0), np.concatenate(P1), np.concatenate(R), np.concatenate(I),
            np.concatenate(BID))


def bin_primitives(lo, hi, dims, brick):
    """CSR lists of primitive indices per level-0 brick for boxes [lo, hi].

    Primitives are kept in index order inside each list (so segments of one
    branch stay contiguous)."""
    nb = [(d + brick - 1) // brick for d in dims]
    blo = np.clip(np.floor(lo / brick).astype(np.int64), 0, np.array(nb) - 1)
    bhi = np.clip(np.floor(hi / brick).astype(np.int64), 0, np.array(nb) - 1)
    inside = np.all(hi >= 0, axis=1) & np.all(lo < np.asarray(dims, dtype=np.float64), axis=1)
    ids, cells = [], []
    for i in np.nonzero(inside)[0]:
        for z in range(blo[i, 2], bhi[i, 2] + 1):
            for y in range(blo[i, 1], bhi[i, 1] + 1):
                for x in range(blo[i, 0], bhi[i, 0] + 1):
                    ids.append(i)
                    cells.append((z * nb[1] + y) * nb[0] + x)
    ids = np.asarray(ids, dtype=np.int64)
    cells = np.asarray(cells, dtype=np.int64)
    order = np.lexsort((ids, cells))
    ids, cells = ids[order], cells[order]
    counts = np.bincount(cells, minlength=nb[0] * nb[1] * nb[2])
    offsets = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    return offsets, ids


def poisson_cdf(lam, kmax):
    """CDF table of Poisson(lam) for k = 0..kmax (inverse-transform sampling)."""
    k = np.arange(kmax + 1)
    logp = -lam + k * math.log(lam) - np.array([math.lgamma(i + 1) for i in k])
    return np.cumsum(np.exp(logp))


# ------------------------------------------------ cell volume (3 x 1 GiB)

CELLS_DIMS = (1024, 1024, 512)
CELLS_BRICK = 64
CELLS_LEVELS = 5


def cell_tracks(channel, timepoint, dims=CELLS_DIMS, n_cells=200, seed=1003,
                sigma=(4.0, 12.0), amp=(5000.0, 40000.0)):
    """Cell centres at a timepoint (damped random walk, reflecting walls),
    with per-cell sigma and amplitude; plus 4 static background Gaussians."""
    rng = np.random.default_rng(seed + channel)
    dims = np.asarray(dims, dtype=np.float64)
    pos = rng.uniform(0, 1, (n_cells, 3)) * dims
    sig = rng.uniform(*sigma, n_cells)
    am = rng.uniform(*amp, n_cells)
    bg_c = rng.uniform(0, 1, (4, 3)) * dims
    bg_a = rng.uniform(500.0, 1500.0, 4)
    vel = np.zeros((n_cells, 3))
    for _ in range(timepoint):
        vel = 0.9 * vel + rng.normal(size=(n_cells, 3))
        pos = pos + vel
        for a in range(3):
            lo = pos[:, a] < 0
            pos[lo, a] = -pos[lo, a]
            vel[lo, a] = -vel[lo, a]
            hi = pos[:, a] > dims[a]
            pos[hi, a] = 2 * dims[a] - pos[hi, a]
            vel[hi, a] = -vel[hi, a]
    return pos, sig, am, bg_c, bg_a


def cells_stereo():
    """The time series' stereo pair: 1440x1600 per eye, vertical half-FOV 50
    degrees, horizontal 0.9 tan 50; longest edge 1024 voxels = 1 m, so the
    64 mm IPD is 65.536 voxels; head 1.25 m from the centre."""
    c = np.array([512.0, 512.0, 256.0])
    head = c + 1280.0 * unit((0.3, -1.0, 0.45))
    t = math.tan(math.radians(50.0))
    return stereo(head, c, 65.536, 1440, 1600, t, 0.9 * t)


CELL_TINTS = ((1.0, 0.2, 0.2), (0.2, 1.0, 0.2), (0.3, 0.3, 1.0))
CELL_DOMAIN = (0.0, 50000.0)
TUBE_DOMAIN = (0.0, 65535.0)
