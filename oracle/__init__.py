"""FP64 CPU oracle for the bricked multiresolution volume ray caster.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The GPU library
never imports, links or calls it, and it shares no code with the GPU library.

The arithmetic lives in ``sgo.c`` (plain C99, double precision, built with
``-O2 -ffp-contract=off``). This module only marshals numpy arrays into it;
every function cites the passage of the paper (arXiv 1804.08197) it follows
in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgo.c")
_LIB = os.path.join(_HERE, "libsgoracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-std=c99", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class View(C.Structure):
    _fields_ = [("cam_to_world", C.c_double * 16),
                ("tan_left", C.c_double), ("tan_right", C.c_double),
                ("tan_bottom", C.c_double), ("tan_top", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32), ("lens", C.c_double * 4)]


class _Scene(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("brick", C.c_int32), ("levels", C.c_int32),
                ("channels", C.c_int32), ("bpv", C.c_int32), ("tf_n", C.c_int32),
                ("lvl", C.POINTER(C.c_void_p)), ("tf", C.POINTER(C.c_double)),
                ("tf_lo", C.POINTER(C.c_double)), ("tf_hi", C.POINTER(C.c_double))]


class Params(C.Structure):
    _fields_ = [("step", C.c_double), ("ert", C.c_double), ("tau", C.c_double),
                ("bg", C.c_double * 4), ("depth_alpha", C.c_double),
                ("bias", C.c_int32), ("lod_on", C.c_int32), ("skip_empty", C.c_int32),
                ("pad", C.c_int32), ("model", C.c_int32), ("n_planes", C.c_int32),
                ("planes", (C.c_double * 4) * 4), ("roi_on", C.c_int32), ("pad2", C.c_int32),
                ("roi", C.c_double * 6)]


MODELS = {"ea": 0, "eo": 1, "mip": 2}


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        i3 = C.POINTER(C.c_int32)
        d3 = C.POINTER(C.c_double)
        vp = C.c_void_p
        L.sgo_level_dims.argtypes = [i3, C.c_int32, i3]
        L.sgo_brick_grid.argtypes = [i3, C.c_int32, C.c_int32, i3]
        L.sgo_node_id.argtypes = [C.c_int32] * 4
        L.sgo_node_id.restype = C.c_uint64
        L.sgo_node_box.argtypes = [i3, C.c_int32, C.c_int32, i3, d3, d3]
        L.sgo_box_outside_view.argtypes = [C.POINTER(View), d3, d3]
        L.sgo_box_outside_view.restype = C.c_int32
        L.sgo_downsample.argtypes = [vp, C.c_int32, i3, vp]
        L.sgo_brick_region.argtypes = [vp, C.c_int32, i3, C.c_int32, i3, vp]
        L.sgo_brick_minmax.argtypes = [vp, C.c_int32, i3, C.c_int32, i3, d3, d3]
        L.sgo_tf_eval.argtypes = [d3, C.c_int32, C.c_double, C.c_double, C.c_double, d3]
        L.sgo_sample.argtypes = [vp, C.c_int32, i3, C.c_int32, d3]
        L.sgo_sample.restype = C.c_double
        L.sgo_ray.argtypes = [C.POINTER(View), C.c_int32, C.c_int32, d3, d3]
        L.sgo_box_interval.argtypes = [d3, d3, d3, d3, d3, d3]
        L.sgo_box_interval.restype = C.c_int32
        L.sgo_entry_exit.argtypes = [i3, d3, d3, d3, d3]
        L.sgo_entry_exit.restype = C.c_int32
        L.sgo_lod_k.argtypes = [C.POINTER(View), C.c_double]
        L.sgo_lod_k.restype = C.c_double
        L.sgo_node_accept.argtypes = [i3, C.c_int32, d3, C.c_double, C.c_int32, C.c_int32, i3]
        L.sgo_node_accept.restype = C.c_int32
        L.sgo_lod_cut.argtypes = [i3, C.c_int32, C.c_int32, C.POINTER(View), C.c_double,
                                  C.c_int32, C.c_int32, C.POINTER(C.c_uint64), C.c_int64]
        L.sgo_lod_cut.restype = C.c_int64
        L.sgo_lod_cut_resident.argtypes = [i3, C.c_int32, C.c_int32, C.POINTER(View),
                                           C.c_double, C.c_int32, C.c_int32,
                                           C.POINTER(C.c_uint64), C.c_int64,
                                           C.POINTER(C.c_uint64), C.c_int64,
                                           C.POINTER(C.c_uint64), C.c_int64,
                                           C.POINTER(C.c_int64)]
        L.sgo_lod_cut_resident.restype = C.c_int64
        L.sgo_nodes_empty.argtypes = [C.POINTER(_Scene), C.POINTER(C.c_uint64), C.c_int64,
                                      C.POINTER(C.c_uint8)]
        L.sgo_nodes_empty_model.argtypes = [C.POINTER(_Scene), C.c_int32,
                                            C.POINTER(C.c_uint64), C.c_int64,
                                            C.POINTER(C.c_uint8)]
        L.sgo_clip.argtypes = [C.POINTER(Params), d3, d3, C.c_double, d3, d3]
        L.sgo_clip.restype = C.c_int32
        L.sgo_render.argtypes = [C.POINTER(_Scene), C.POINTER(View), C.POINTER(Params),
                                 C.POINTER(C.c_uint64), C.c_int64, C.POINTER(C.c_uint8),
                                 C.c_int64, i3, d3, d3, d3, C.POINTER(C.c_int64),
                                 C.POINTER(C.c_void_p), C.c_int32]
        L.sgo_render.restype = C.c_int64
        L.sgo_max_threads.restype = C.c_int32
        _lib = L
    return _lib


def _i3(v):
    return (C.c_int32 * 3)(*[int(x) for x in v])


def _d3(v):
    return (C.c_double * 3)(*[float(x) for x in v])


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _bpv(a: np.ndarray) -> int:
    if a.dtype == np.uint8:
        return 1
    if a.dtype == np.uint16:
        return 2
    raise TypeError("volumes are uint8 or uint16")


def make_view(v: dict) -> View:
    """Oracle view from a plain dict (cam_to_world 4x4, tangents, size)."""
    out = View()
    m = np.asarray(v["cam_to_world"], dtype=np.float64).reshape(16)
    for i in range(16):
        out.cam_to_world[i] = float(m[i])
    out.tan_left, out.tan_right = float(v["tan_left"]), float(v["tan_right"])
    out.tan_bottom, out.tan_top = float(v["tan_bottom"]), float(v["tan_top"])
    out.width, out.height = int(v["width"]), int(v["height"])
    lens = v.get("lens") or (0.0, 0.0, 0.0, 0.0)
    for i in range(4):
        out.lens[i] = float(lens[i])
    return out


def make_params(p: dict) -> Params:
    out = Params()
    out.step = float(p.get("step", 0.5))
    out.ert = float(p.get("ert", 0.99))
    out.tau = float(p.get("tau", 1.0))
    bg = p.get("bg", (0.0, 0.0, 0.0, 0.0))
    for i in range(4):
        out.bg[i] = float(bg[i])
    out.depth_alpha = float(p.get("depth_alpha", 0.5))
    out.bias = int(p.get("bias", 0))
    out.lod_on = int(p.get("lod", 1))
    out.skip_empty = int(p.get("skip_empty", 1))
    model = p.get("model", 0)
    out.model = MODELS[model] if isinstance(model, str) else int(model)
    planes = p.get("planes") or ()
    if len(planes) > 4:
        raise ValueError("at most 4 cut planes")
    out.n_planes = len(planes)
    for j, q in enumerate(planes):
        for i in range(4):
            out.planes[j][i] = float(q[i])
    roi = p.get("roi")
    out.roi_on = int(roi is not None)
    if roi is not None:
        for i in range(6):
            out.roi[i] = float(np.asarray(roi, dtype=np.float64).reshape(6)[i])
    return out


# ---------------------------------------------------------------- steps
def level_dims(dims0, L):
    out = (C.c_int32 * 3)()
    lib().sgo_level_dims(_i3(dims0), int(L), out)
    return tuple(out)


def brick_grid(dims0, B, L):
    out = (C.c_int32 * 3)()
    lib().sgo_brick_grid(_i3(dims0), int(B), int(L), out)
    return tuple(out)


def node_id(L, bx, by, bz) -> int:
    return int(lib().sgo_node_id(L, bx, by, bz))


def node_decode(ids):
    ids = np.asarray(ids, dtype=np.uint64)
    return np.stack([(ids >> np.uint64(60)).astype(np.int64),
                     ((ids >> np.uint64(40)) & np.uint64(0xFFFFF)).astype(np.int64),
                     ((ids >> np.uint64(20)) & np.uint64(0xFFFFF)).astype(np.int64),
                     (ids & np.uint64(0xFFFFF)).astype(np.int64)], axis=-1)


def node_box(dims0, B, L, b):
    lo, hi = (C.c_double * 3)(), (C.c_double * 3)()
    lib().sgo_node_box(_i3(dims0), int(B), int(L), _i3(b), lo, hi)
    return np.array(lo[:]), np.array(hi[:])


def box_outside_view(view: dict, lo, hi) -> bool:
    """Does box [lo, hi] lie outside every ray of the view (Sec 5.2)?"""
    v = make_view(view)
    return bool(lib().sgo_box_outside_view(C.byref(v), _d3(lo), _d3(hi)))


def downsample(vol: np.ndarray) -> np.ndarray:
    """Next pyramid level. vol is indexed [z, y, x]."""
    vol = np.ascontiguousarray(vol)
    nz, ny, nx = vol.shape
    out = np.empty(((nz + 1) // 2, (ny + 1) // 2, (nx + 1) // 2), dtype=vol.dtype)
    lib().sgo_downsample(vol.ctypes.data, _bpv(vol), _i3((nx, ny, nz)), out.ctypes.data)
    return out


def pyramid(vol: np.ndarray, levels: int):
    out = [np.ascontiguousarray(vol)]
    for _ in range(1, levels):
        out.append(downsample(out[-1]))
    return out


def brick_region(level: np.ndarray, B: int, b):
    nz, ny, nx = level.shape
    out = np.empty((B + 2,) * 3, dtype=level.dtype)
    lib().sgo_brick_region(level.ctypes.data, _bpv(level), _i3((nx, ny, nz)), int(B),
                           _i3(b), out.ctypes.data)
    return out


def brick_minmax(level: np.ndarray, B: int, b):
    nz, ny, nx = level.shape
    mn, mx = C.c_double(), C.c_double()
    lib().sgo_brick_minmax(level.ctypes.data, _bpv(level), _i3((nx, ny, nz)), int(B),
                           _i3(b), C.byref(mn), C.byref(mx))
    return mn.value, mx.value


def tf_eval(tf: np.ndarray, lo: float, hi: float, v: float) -> np.ndarray:
    tf = np.ascontiguousarray(tf, dtype=np.float64)
    out = (C.c_double * 4)()
    lib().sgo_tf_eval(_ptr(tf, C.c_double), tf.shape[0], float(lo), float(hi), float(v), out)
    return np.array(out[:])


def sample(level: np.ndarray, L: int, p) -> float:
    nz, ny, nx = level.shape
    return float(lib().sgo_sample(level.ctypes.data, _bpv(level), _i3((nx, ny, nz)), int(L),
                                  _d3(p)))


def ray(view: dict, x: int, y: int):
    e, d = (C.c_double * 3)(), (C.c_double * 3)()
    v = make_view(view)
    lib().sgo_ray(C.byref(v), int(x), int(y), e, d)
    return np.array(e[:]), np.array(d[:])


def box_interval(e, d, lo, hi):
    t0, t1 = C.c_double(), C.c_double()
    hit = lib().sgo_box_interval(_d3(e), _d3(d), _d3(lo), _d3(hi), C.byref(t0), C.byref(t1))
    return bool(hit), t0.value, t1.value


def entry_exit(dims0, e, d):
    t0, t1 = C.c_double(), C.c_double()
    hit = lib().sgo_entry_exit(_i3(dims0), _d3(e), _d3(d), C.byref(t0), C.byref(t1))
    return bool(hit), t0.value, t1.value


def clip(params: dict, e, d, t0, t1, limit=np.inf):
    """O16: the ray interval [t0, t1] clipped by cut planes, ROI and a ray limit."""
    p = make_params(params)
    a, b = C.c_double(t0), C.c_double(t1)
    ok = lib().sgo_clip(C.byref(p), _d3(e), _d3(d), float(limit), C.byref(a), C.byref(b))
    return bool(ok), a.value, b.value


def lod_k(view: dict, tau: float) -> float:
    v = make_view(view)
    return float(lib().sgo_lod_k(C.byref(v), float(tau)))


def node_accept(dims0, B, e, K, bias, L, b) -> bool:
    return bool(lib().sgo_node_accept(_i3(dims0), int(B), _d3(e), float(K), int(bias),
                                      int(L), _i3(b)))


def lod_cut(dims0, B, levels, view: dict, tau=1.0, bias=0, lod=True) -> np.ndarray:
    v = make_view(view)
    n = lib().sgo_lod_cut(_i3(dims0), int(B), int(levels), C.byref(v), float(tau), int(bias),
                          int(bool(lod)), None, 0)
    if n < 0:
        raise ValueError("bad LOD arguments")
    out = np.zeros(max(n, 1), dtype=np.uint64)
    m = lib().sgo_lod_cut(_i3(dims0), int(B), int(levels), C.byref(v), float(tau), int(bias),
                          int(bool(lod)), _ptr(out, C.c_uint64), n)
    assert m == n
    return out[:n]


def lod_cut_resident(dims0, B, levels, view: dict, resident, tau=1.0, bias=0, lod=True):
    """O18: (cut, requested) when only the node identifiers in `resident`
    are in the cache (every top-level node must be)."""
    v = make_view(view)
    res = np.unique(np.asarray(resident, dtype=np.uint64))
    res = np.ascontiguousarray(res if len(res) else np.zeros(1, np.uint64)[:0])
    nreq = C.c_int64()
    args = (_i3(dims0), int(B), int(levels), C.byref(v), float(tau), int(bias), int(bool(lod)),
            _ptr(res, C.c_uint64) if len(res) else (C.c_uint64 * 1)(), len(res))
    n = lib().sgo_lod_cut_resident(*args, None, 0, None, 0, C.byref(nreq))
    if n == -2:
        raise ValueError("a top-level node is not resident")
    if n < 0:
        raise ValueError("bad LOD arguments")
    out = np.zeros(max(n, 1), dtype=np.uint64)
    req = np.zeros(max(nreq.value, 1), dtype=np.uint64)
    m = lib().sgo_lod_cut_resident(*args, _ptr(out, C.c_uint64), n, _ptr(req, C.c_uint64),
                                   nreq.value, C.byref(nreq))
    assert m == n
    return out[:n], req[:nreq.value]


class Scene:
    """Volume pyramid(s) plus transfer functions, held as numpy arrays.

    ``channels`` is a list of level-0 arrays indexed [z, y, x] (uint8 or
    uint16); ``tfs`` a list of (N, 4) float64 tables and ``domains`` a list
    of (lo, hi) raw-value windows, one per channel.
    """

    def __init__(self, channels, brick: int, levels: int, tfs, domains, pyramids=None):
        self.channels = [np.ascontiguousarray(c) for c in channels]
        nz, ny, nx = self.channels[0].shape
        self.dims = (nx, ny, nz)
        self.brick, self.levels = int(brick), int(levels)
        self.levels_arr = pyramids if pyramids is not None else \
            [pyramid(c, self.levels) for c in self.channels]
        self.set_tfs(tfs, domains)
        ptrs = []
        for c in range(len(self.channels)):
            for L in range(self.levels):
                ptrs.append(self.levels_arr[c][L].ctypes.data)
        self._ptrs = (C.c_void_p * len(ptrs))(*ptrs)
        self._bpv = _bpv(self.channels[0])

    def set_tfs(self, tfs, domains):
        self.tf = np.ascontiguousarray(np.stack([np.asarray(t, dtype=np.float64) for t in tfs]))
        self.tf_lo = np.ascontiguousarray([float(d[0]) for d in domains], dtype=np.float64)
        self.tf_hi = np.ascontiguousarray([float(d[1]) for d in domains], dtype=np.float64)

    def _struct(self) -> _Scene:
        s = _Scene()
        for i in range(3):
            s.dims[i] = self.dims[i]
        s.brick, s.levels = self.brick, self.levels
        s.channels, s.bpv, s.tf_n = len(self.channels), self._bpv, self.tf.shape[1]
        s.lvl = C.cast(self._ptrs, C.POINTER(C.c_void_p))
        s.tf = _ptr(self.tf, C.c_double)
        s.tf_lo = _ptr(self.tf_lo, C.c_double)
        s.tf_hi = _ptr(self.tf_hi, C.c_double)
        return s

    def cut(self, view: dict, params: dict) -> np.ndarray:
        p = make_params(params)
        return lod_cut(self.dims, self.brick, self.levels, view, p.tau, p.bias, bool(p.lod_on))

    def empty(self, ids: np.ndarray, model=0) -> np.ndarray:
        """Skip flags of the cut nodes for an optical model (O9, O17)."""
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        out = np.zeros(max(len(ids), 1), dtype=np.uint8)
        s = self._struct()
        m = MODELS[model] if isinstance(model, str) else int(model)
        lib().sgo_nodes_empty_model(C.byref(s), m, _ptr(ids, C.c_uint64), len(ids),
                                    _ptr(out, C.c_uint8))
        return out[:len(ids)].astype(bool)

    def render(self, view: dict, params: dict, pixels=None, depth=False, count=False,
               microblocks=False, threads=0, cut=None, empty=None, limit=None):
        """Render a view (all pixels, or the (x, y) rows of ``pixels``).

        ``limit`` is an optional (H, W) array of ray limits (distance along
        the ray of opaque geometry, +inf where there is none).

        Returns a dict with ``rgba`` (H, W, 4) or (npix, 4) float64 and,
        on request, ``depth``, ``nsamp``, per-level micro-block bitmaps and
        the total sample count.
        """
        v = make_view(view)
        p = make_params(params)
        if cut is None:
            cut = self.cut(view, params)
        cut = np.ascontiguousarray(cut, dtype=np.uint64)
        if empty is None:
            empty = self.empty(cut, p.model) if p.skip_empty else np.zeros(len(cut), bool)
        lim = None
        if limit is not None:
            lim = np.ascontiguousarray(limit, dtype=np.float64).reshape(v.height, v.width)
        emp = np.ascontiguousarray(empty, dtype=np.uint8)
        if pixels is None:
            npix = v.width * v.height
            pix_ptr = None
        else:
            pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
            npix = pix.shape[0]
            pix_ptr = _ptr(pix, C.c_int32)
        rgba = np.zeros((npix, 4), dtype=np.float64)
        dep = np.zeros(npix, dtype=np.float64) if depth else None
        ns = np.zeros(npix, dtype=np.int64) if count else None
        mbs = None
        mb_ptr = None
        if microblocks:
            mbs = []
            for c in range(len(self.channels)):
                for L in range(self.levels):
                    n = level_dims(self.dims, L)
                    mbs.append(np.zeros(((n[2] + 3) // 4, (n[1] + 3) // 4, (n[0] + 3) // 4),
                                        dtype=np.uint8))
            mb_ptr = (C.c_void_p * len(mbs))(*[m.ctypes.data for m in mbs])
        s = self._struct()
        total = lib().sgo_render(
            C.byref(s), C.byref(v), C.byref(p), _ptr(cut, C.c_uint64), len(cut),
            _ptr(emp, C.c_uint8) if len(emp) else None, npix, pix_ptr,
            _ptr(lim, C.c_double) if lim is not None else None, _ptr(rgba, C.c_double), _ptr(dep, C.c_double) if dep is not None else None,
            _ptr(ns, C.c_int64) if ns is not None else None,
            C.cast(mb_ptr, C.POINTER(C.c_void_p)) if mb_ptr is not None else None, int(threads))
        if total < 0:
            raise ValueError("oracle render: bad arguments")
        out = {"total_samples": int(total)}
        if pixels is None:
            out["rgba"] = rgba.reshape(v.height, v.width, 4)
            if dep is not None:
                out["depth"] = dep.reshape(v.height, v.width)
            if ns is not None:
                out["nsamp"] = ns.reshape(v.height, v.width)
        else:
            out["rgba"] = rgba
            if dep is not None:
                out["depth"] = dep
            if ns is not None:
                out["nsamp"] = ns
        if mbs is not None:
            out["microblocks"] = mbs
        return out


def max_threads() -> int:
    return int(lib().sgo_max_threads())
