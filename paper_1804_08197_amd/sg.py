"""ctypes binding of ``include/sg.h`` (argument marshalling only).

Every function has the name of the C entry point it calls. Device buffers
are passed as torch tensors (``data_ptr()``) and streams as torch streams or
raw ``hipStream_t`` integers; the work itself runs in ``libsg.so``. There is
no fallback: if the library is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsg.so")

SG_OK = 0
SG_ERR_INVALID_ARG = -1
SG_ERR_OUT_OF_MEMORY = -2
SG_ERR_DEVICE = -3
SG_ERR_STATE = -4
SG_ERR_UNSUPPORTED = -5
SG_U8, SG_U16 = 1, 2
SG_LAYOUT_LINEAR, SG_LAYOUT_MICROBLOCK = 0, 1
SG_LOD, SG_SKIP_EMPTY, SG_GATHER = 1, 2, 4
SG_MODEL_EMISSION_ABSORPTION, SG_MODEL_EMISSION_ONLY, SG_MODEL_MAX_INTENSITY = 0, 1, 2
MODELS = {"ea": SG_MODEL_EMISSION_ABSORPTION, "eo": SG_MODEL_EMISSION_ONLY,
          "mip": SG_MODEL_MAX_INTENSITY}
SG_ABI_VERSION = 5


class SgError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__("%s: %s (%s)" % (where, detail, _status_name(status)))
        self.status = status


class sg_volume_desc(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("channels", C.c_int32), ("timepoints", C.c_int32),
                ("dtype", C.c_int32), ("brick", C.c_int32), ("levels", C.c_int32),
                ("device", C.c_int32), ("cache_slots", C.c_int32), ("layout", C.c_int32)]


class sg_view(C.Structure):
    _fields_ = [("cam_to_world", C.c_double * 16), ("tan_left", C.c_double),
                ("tan_right", C.c_double), ("tan_bottom", C.c_double), ("tan_top", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32), ("lens", C.c_double * 4),
                ("ray_limit", C.c_void_p), ("tile_any", C.c_void_p)]


class sg_render_params(C.Structure):
    _fields_ = [("step_voxels", C.c_double), ("ert_alpha", C.c_double),
                ("lod_tau_px", C.c_double), ("background", C.c_double * 4),
                ("depth_alpha", C.c_double), ("lod_bias", C.c_int32), ("timepoint", C.c_int32),
                ("flags", C.c_uint32), ("model", C.c_int32), ("n_planes", C.c_int32),
                ("roi_on", C.c_int32), ("planes", (C.c_double * 4) * 4), ("roi", C.c_double * 6)]


class sg_render_stats(C.Structure):
    _fields_ = [("samples", C.POINTER(C.c_void_p)), ("total_samples", C.c_uint64),
                ("microblocks", C.c_uint64), ("node_visits", C.c_uint64), ("slabs", C.c_uint64),
                ("staged_bytes", C.c_uint64), ("node_lanes", C.c_uint64),
                ("loop_iterations", C.c_uint64), ("pool_samples", C.c_uint64),
                ("slab_retries", C.c_uint64), ("alive_lanes", C.c_uint64),
                ("wide_slabs", C.c_uint64)]


class sg_cache_info(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("resident", C.c_int64), ("uploads", C.c_int64),
                ("evictions", C.c_int64), ("frame", C.c_int64)]


class sg_launch_config(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("tile", C.c_int32), ("block", C.c_int32),
                ("stage_bytes", C.c_int32), ("persistent", C.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError("libsg.so is not built (run __graft_entry__.build()); there is no "
                      "fallback implementation")
# torch ships its own HIP runtime (libamdhip64.so, found through its RPATH).
# It must be loaded before libsg.so: the library then binds to that same
# runtime (same soname) and shares torch's devices, streams and memory.
# Loaded the other way round, the process would hold two HIP runtimes and
# the library would receive pointers and streams it cannot use.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)
_P = C.c_void_p
_lib.sg_volume_create.argtypes = [C.POINTER(sg_volume_desc), C.POINTER(_P)]
_lib.sg_volume_destroy.argtypes = [_P]
_lib.sg_upload_bricks.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  C.POINTER(C.c_int32), _P, C.c_int32, _P]
_lib.sg_build_lod.argtypes = [_P, C.c_int32, C.c_int32, _P]
_lib.sg_volume_commit.argtypes = [_P, _P]
_lib.sg_set_transfer_function.argtypes = [_P, C.c_int32, C.POINTER(C.c_float), C.c_int32,
                                          C.c_double, C.c_double]
_lib.sg_render_views.argtypes = [_P, C.c_int32, C.POINTER(sg_view),
                                 C.POINTER(sg_render_params), C.POINTER(_P), C.POINTER(_P), _P]
_lib.sg_render_views_stats.argtypes = [_P, C.c_int32, C.POINTER(sg_view),
                                       C.POINTER(sg_render_params), C.POINTER(_P),
                                       C.POINTER(_P), C.POINTER(sg_render_stats), _P]
_lib.sg_get_lod_cut.argtypes = [_P, C.POINTER(sg_view), C.POINTER(sg_render_params),
                                C.POINTER(C.c_uint64), C.POINTER(C.c_int32),
                                C.POINTER(C.c_uint8), _P]
_lib.sg_volume_memory.argtypes = [_P, C.POINTER(C.c_uint64)]
_lib.sg_set_kernel_timing.argtypes = [_P, C.c_int32]
_lib.sg_get_kernel_timing.argtypes = [_P, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
_lib.sg_set_launch_config.argtypes = [_P, C.POINTER(sg_launch_config)]
_lib.sg_get_launch_config.argtypes = [_P, C.POINTER(sg_launch_config)]
_lib.sg_autotune.argtypes = [_P, C.c_int32, C.POINTER(sg_view), C.POINTER(sg_render_params),
                             C.POINTER(_P), C.c_int32, C.POINTER(sg_launch_config),
                             C.POINTER(C.c_double), _P]
_lib.sg_render_graph_create.argtypes = [_P, C.c_int32, C.POINTER(sg_view),
                                        C.POINTER(sg_render_params), C.POINTER(_P),
                                        C.POINTER(_P), C.POINTER(_P)]
_lib.sg_render_graph_set_views.argtypes = [_P, C.POINTER(sg_view), _P]
_lib.sg_render_graph_launch.argtypes = [_P, _P]
_lib.sg_render_graph_destroy.argtypes = [_P]
_lib.sg_cache_put.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                              C.POINTER(C.c_int32), _P, C.c_int32, _P]
_lib.sg_render_views_if.argtypes = [_P, C.c_int32, C.POINTER(sg_view), C.POINTER(sg_render_params),
                                    C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), _P, _P]
_lib.sg_composite_over.argtypes = [C.POINTER(sg_view), C.c_int32, C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_double), _P, _P]
_lib.sg_cache_put_scattered.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                        C.POINTER(C.c_int32), C.POINTER(C.c_void_p), _P]
_lib.sg_cache_requests.argtypes = [_P, C.POINTER(C.c_uint64), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), _P]
_lib.sg_cache_get_info.argtypes = [_P, C.POINTER(sg_cache_info)]
_lib.sg_cache_resident.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32)]
_lib.sg_render_views_noalloc.argtypes = [_P, C.c_int32, C.POINTER(sg_view),
                                         C.POINTER(sg_render_params), C.POINTER(_P),
                                         C.POINTER(_P), _P]
_lib.sg_pyramid_level.argtypes = [C.c_int32, C.POINTER(C.c_int32), _P, _P, _P]
_lib.sg_brick_regions.argtypes = [C.c_int32, C.POINTER(C.c_int32), _P, C.c_int32, C.c_int32,
                                  C.POINTER(C.c_int32), _P, _P]
_lib.sg_status_string.argtypes = [C.c_int]
_lib.sg_status_string.restype = C.c_char_p
_lib.sg_last_error.restype = C.c_char_p
_lib.sg_abi_version.restype = C.c_int32
for _f in ("sg_volume_create", "sg_volume_destroy", "sg_upload_bricks", "sg_build_lod",
           "sg_volume_commit", "sg_set_transfer_function", "sg_render_views",
           "sg_render_views_stats", "sg_get_lod_cut", "sg_volume_memory",
           "sg_set_kernel_timing", "sg_get_kernel_timing", "sg_set_launch_config",
           "sg_get_launch_config", "sg_autotune", "sg_render_graph_create",
           "sg_render_graph_set_views", "sg_render_graph_launch", "sg_render_graph_destroy",
           "sg_cache_put", "sg_cache_put_scattered", "sg_cache_requests", "sg_cache_get_info",
           "sg_cache_resident", "sg_render_views_if", "sg_pyramid_level", "sg_brick_regions",
           "sg_render_views_noalloc"):
    getattr(_lib, _f).restype = C.c_int


def lib():
    return _lib


def _status_name(s: int) -> str:
    return _lib.sg_status_string(int(s)).decode()


def _check(status: int, where: str):
    if status != SG_OK:
        raise SgError(status, where, _lib.sg_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(x):
    """Device or host address of a torch tensor / numpy array / int."""
    if x is None:
        return None
    if isinstance(x, int):
        return C.c_void_p(x)
    if isinstance(x, np.ndarray):
        return C.c_void_p(x.ctypes.data)
    return C.c_void_p(x.data_ptr())


def make_view(v) -> sg_view:
    if isinstance(v, sg_view):
        return v
    o = sg_view()
    o.cam_to_world[:] = np.asarray(v["cam_to_world"], dtype=np.float64).reshape(16).tolist()
    o.tan_left, o.tan_right = float(v["tan_left"]), float(v["tan_right"])
    o.tan_bottom, o.tan_top = float(v["tan_bottom"]), float(v["tan_top"])
    o.width, o.height = int(v["width"]), int(v["height"])
    lens = v.get("lens")
    if lens:
        o.lens[:] = [float(x) for x in lens]
    lim = _ptr(v.get("ray_limit"))
    o.ray_limit = lim.value if lim is not None else None
    ta = _ptr(v.get("tile_any"))
    o.tile_any = ta.value if ta is not None else None
    return o


def make_params(p=None) -> sg_render_params:
    if isinstance(p, sg_render_params):
        return p
    p = dict(p or {})
    o = sg_render_params()
    o.step_voxels = float(p.get("step", 0.5))
    o.ert_alpha = float(p.get("ert", 0.99))
    o.lod_tau_px = float(p.get("tau", 1.0))
    bg = p.get("bg", (0.0, 0.0, 0.0, 0.0))
    for i in range(4):
        o.background[i] = float(bg[i])
    o.depth_alpha = float(p.get("depth_alpha", 0.5))
    o.lod_bias = int(p.get("bias", 0))
    o.timepoint = int(p.get("timepoint", 0))
    flags = 0
    if p.get("lod", 1):
        flags |= SG_LOD
    if p.get("skip_empty", 1):
        flags |= SG_SKIP_EMPTY
    if p.get("gather", 0):
        flags |= SG_GATHER
    o.flags = int(p.get("flags", flags))
    model = p.get("model", SG_MODEL_EMISSION_ABSORPTION)
    o.model = MODELS[model] if isinstance(model, str) else int(model)
    planes = list(p.get("planes") or ())
    o.n_planes = int(p.get("n_planes", len(planes)))
    for j, q in enumerate(planes[:4]):
        for i in range(4):
            o.planes[j][i] = float(q[i])
    roi = p.get("roi")
    o.roi_on = int(p.get("roi_on", roi is not None))
    if roi is not None:
        r = np.asarray(roi, dtype=np.float64).reshape(6)
        for i in range(6):
            o.roi[i] = float(r[i])
    return o


# ------------------------------------------------------------ entry points
def sg_abi_version() -> int:
    return int(_lib.sg_abi_version())


def sg_status_string(s: int) -> str:
    return _status_name(s)


def sg_last_error() -> str:
    return _lib.sg_last_error().decode()


def sg_volume_create(dims, channels=1, timepoints=1, dtype=SG_U16, brick=64, levels=1,
                     device=0, cache_slots=0, layout=SG_LAYOUT_LINEAR):
    d = sg_volume_desc()
    for i in range(3):
        d.dims[i] = int(dims[i])
    d.channels, d.timepoints, d.dtype = int(channels), int(timepoints), int(dtype)
    d.brick, d.levels, d.device = int(brick), int(levels), int(device)
    d.cache_slots, d.layout = int(cache_slots), int(layout)
    h = C.c_void_p()
    _check(_lib.sg_volume_create(C.byref(d), C.byref(h)), "sg_volume_create")
    return h


def sg_volume_destroy(vol):
    _check(_lib.sg_volume_destroy(vol), "sg_volume_destroy")


def sg_upload_bricks(vol, channel, timepoint, level, coords, src, src_on_device=None,
                     stream=None):
    coords = np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 3)
    if src_on_device is None:
        src_on_device = not isinstance(src, np.ndarray) and getattr(src, "is_cuda", False)
    if isinstance(src, np.ndarray):
        src = np.ascontiguousarray(src)
    _check(_lib.sg_upload_bricks(vol, int(channel), int(timepoint), int(level), len(coords),
                                 coords.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(src),
                                 int(bool(src_on_device)), _stream(stream)),
           "sg_upload_bricks")


def sg_build_lod(vol, channel, timepoint, stream=None):
    _check(_lib.sg_build_lod(vol, int(channel), int(timepoint), _stream(stream)), "sg_build_lod")


def sg_volume_commit(vol, stream=None):
    _check(_lib.sg_volume_commit(vol, _stream(stream)), "sg_volume_commit")


def sg_set_transfer_function(vol, channel, rgba, domain_lo, domain_hi):
    t = np.ascontiguousarray(rgba, dtype=np.float32).reshape(-1, 4)
    _check(_lib.sg_set_transfer_function(vol, int(channel),
                                         t.ctypes.data_as(C.POINTER(C.c_float)), t.shape[0],
                                         float(domain_lo), float(domain_hi)),
           "sg_set_transfer_function")


def _views(views):
    """An sg_view array from view dicts (or the prebuilt array itself)."""
    if isinstance(views, C.Array):
        return views
    return (sg_view * len(views))(*[make_view(v) for v in views])


def _ptrs(tensors):
    """A device-pointer array from tensors (None entries stay NULL), or the
    prebuilt array itself."""
    if isinstance(tensors, C.Array):
        return tensors
    return (C.c_void_p * len(tensors))(*[(t.data_ptr() if t is not None else None)
                                         for t in tensors])


def views_array(views):
    """Pack view dicts once into an sg_view array that the render calls
    accept as they are (for callers that render the same views more than
    once, or derive one set of views from another)."""
    return _views(views)


def pointer_array(tensors):
    """Pack the device addresses of output tensors once (see views_array)."""
    return _ptrs(tensors)


def sg_render_views(vol, views, params, out_rgba, out_depth=None, stream=None):
    """params: a dict (see make_params) or a prebuilt sg_render_params."""
    n = len(views)
    varr = _views(views)
    p = params if isinstance(params, sg_render_params) else make_params(params)
    rgba = _ptrs(out_rgba)
    dep = _ptrs(out_depth) if out_depth is not None else None
    _check(_lib.sg_render_views(vol, n, varr, C.byref(p), rgba, dep, _stream(stream)),
           "sg_render_views")


def sg_render_views_noalloc(vol, views, params, out_rgba, out_depth=None, stream=None):
    """sg_render_views with its per-render scratch in the library's static
    device array (no allocation; at most 4 views, committed volume)."""
    n = len(views)
    varr = _views(views)
    p = params if isinstance(params, sg_render_params) else make_params(params)
    rgba = _ptrs(out_rgba)
    dep = _ptrs(out_depth) if out_depth is not None else None
    _check(_lib.sg_render_views_noalloc(vol, n, varr, C.byref(p), rgba, dep, _stream(stream)),
           "sg_render_views_noalloc")

def sg_render_views_if(vol, views, params, out_rgba, enable, out_depth=None, stream=None):
    """sg_render_views carried out only if the device int32 `enable` (a
    one-element tensor) is nonzero when the render runs."""
    n = len(views)
    varr = _views(views)
    p = params if isinstance(params, sg_render_params) else make_params(params)
    rgba = _ptrs(out_rgba)
    dep = _ptrs(out_depth) if out_depth is not None else None
    if enable is None:
        raise ValueError("sg_render_views_if needs a device flag")
    _check(_lib.sg_render_views_if(vol, n, varr, C.byref(p), rgba, dep,
                                   C.c_void_p(enable.data_ptr()), _stream(stream)),
           "sg_render_views_if")


def sg_composite_over(view, parts, boxes, out_rgba, stream=None):
    """Front-over-back composite of the part images (device float4 tensors,
    one per box) of one view, in the order each pixel's ray enters the boxes
    (boxes: one (lo x, y, z, hi x, y, z) per part)."""
    n = len(parts)
    v = make_view(view)
    arr = (C.c_void_p * n)(*[p.data_ptr() for p in parts])
    b = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(n, 6))
    _check(_lib.sg_composite_over(C.byref(v), n, arr,
                                  b.ctypes.data_as(C.POINTER(C.c_double)),
                                  C.c_void_p(out_rgba.data_ptr()), _stream(stream)),
           "sg_composite_over")


def sg_render_views_stats(vol, views, params, out_rgba, out_depth=None, out_samples=None,
                          stream=None):
    n = len(views)
    varr = _views(views)
    p = make_params(params)
    rgba = _ptrs(out_rgba)
    dep = _ptrs(out_depth) if out_depth is not None else None
    st = sg_render_stats()
    if out_samples is not None:
        smp = (C.c_void_p * n)(*[(o.data_ptr() if o is not None else None) for o in out_samples])
        st.samples = C.cast(smp, C.POINTER(C.c_void_p))
    _check(_lib.sg_render_views_stats(vol, n, varr, C.byref(p), rgba, dep, C.byref(st),
                                      _stream(stream)), "sg_render_views_stats")
    return {"total_samples": int(st.total_samples), "microblocks": int(st.microblocks),
            "node_visits": int(st.node_visits), "slabs": int(st.slabs),
            "staged_bytes": int(st.staged_bytes), "node_lanes": int(st.node_lanes),
            "loop_iterations": int(st.loop_iterations), "pool_samples": int(st.pool_samples),
            "slab_retries": int(st.slab_retries), "alive_lanes": int(st.alive_lanes),
            "wide_slabs": int(st.wide_slabs)}


def sg_get_lod_cut(vol, view, params, capacity=1 << 20, stream=None):
    v = make_view(view)
    p = make_params(params)
    nodes = np.zeros(capacity, dtype=np.uint64)
    empty = np.zeros(capacity, dtype=np.uint8)
    n = C.c_int32(capacity)
    _check(_lib.sg_get_lod_cut(vol, C.byref(v), C.byref(p),
                               nodes.ctypes.data_as(C.POINTER(C.c_uint64)), C.byref(n),
                               empty.ctypes.data_as(C.POINTER(C.c_uint8)), _stream(stream)),
           "sg_get_lod_cut")
    return nodes[:n.value].copy(), empty[:n.value].astype(bool)


def sg_volume_memory(vol) -> int:
    b = C.c_uint64()
    _check(_lib.sg_volume_memory(vol, C.byref(b)), "sg_volume_memory")
    return int(b.value)


def sg_set_kernel_timing(vol, enable=True):
    _check(_lib.sg_set_kernel_timing(vol, int(bool(enable))), "sg_set_kernel_timing")


def sg_get_kernel_timing(vol):
    """(renders, cut-map ms, ray-cast ms) summed since the last query."""
    n, a, b = C.c_int32(), C.c_double(), C.c_double()
    _check(_lib.sg_get_kernel_timing(vol, C.byref(n), C.byref(a), C.byref(b)),
           "sg_get_kernel_timing")
    return int(n.value), float(a.value), float(b.value)


# ------------------------------------------------- launch configuration
LAUNCH_FIELDS = ("kernel", "tile", "block", "stage_bytes", "persistent")
DEFAULT_LAUNCH = {"kernel": 0, "tile": 16, "block": 64, "stage_bytes": 8192, "persistent": 0}


def _launch_struct(cfg) -> sg_launch_config:
    c = dict(DEFAULT_LAUNCH, **(cfg or {}))
    o = sg_launch_config()
    for k in LAUNCH_FIELDS:
        setattr(o, k, int(c[k]))
    return o


def launch_config_struct(cfg) -> sg_launch_config:
    """A launch configuration dict packed once (sg_set_launch_config takes it
    as it is)."""
    return _launch_struct(cfg)


def _launch_dict(o: sg_launch_config) -> dict:
    return {k: int(getattr(o, k)) for k in LAUNCH_FIELDS}


def sg_set_launch_config(vol, cfg=None):
    """cfg: dict with kernel / tile / block / stage_bytes / persistent, a
    prebuilt sg_launch_config, or None for the default."""
    c = cfg if isinstance(cfg, sg_launch_config) or cfg is None else _launch_struct(cfg)
    _check(_lib.sg_set_launch_config(vol, C.byref(c) if c is not None else None),
           "sg_set_launch_config")


def sg_get_launch_config(vol) -> dict:
    o = sg_launch_config()
    _check(_lib.sg_get_launch_config(vol, C.byref(o)), "sg_get_launch_config")
    return _launch_dict(o)


def sg_autotune(vol, views, params, out_rgba, repeats=3, stream=None):
    """Tune the volume's launch configuration on this render; returns
    (config dict, ms per render)."""
    n = len(views)
    varr = _views(views)
    p = make_params(params)
    rgba = (C.c_void_p * n)(*[o.data_ptr() for o in out_rgba])
    best = sg_launch_config()
    ms = C.c_double()
    _check(_lib.sg_autotune(vol, n, varr, C.byref(p), rgba, int(repeats), C.byref(best),
                            C.byref(ms), _stream(stream)), "sg_autotune")
    return _launch_dict(best), float(ms.value)


class RenderGraph:
    """A render prepared once as a HIP graph and replayed per frame."""

    def __init__(self, vol, views, params, out_rgba, out_depth=None):
        n = len(views)
        self.n = n
        varr = _views(views)
        p = make_params(params)
        rgba = (C.c_void_p * n)(*[o.data_ptr() for o in out_rgba])
        dep = None
        if out_depth is not None:
            dep = (C.c_void_p * n)(*[(o.data_ptr() if o is not None else None)
                                     for o in out_depth])
        h = C.c_void_p()
        _check(_lib.sg_render_graph_create(vol, n, varr, C.byref(p), rgba, dep, C.byref(h)),
               "sg_render_graph_create")
        self.handle = h

    def set_views(self, views, stream=None):
        assert len(views) == self.n
        _check(_lib.sg_render_graph_set_views(self.handle, _views(views), _stream(stream)),
               "sg_render_graph_set_views")

    def launch(self, stream=None):
        _check(_lib.sg_render_graph_launch(self.handle, _stream(stream)),
               "sg_render_graph_launch")

    def destroy(self):
        if self.handle is not None:
            _check(_lib.sg_render_graph_destroy(self.handle), "sg_render_graph_destroy")
            self.handle = None


# ------------------------------------------------------------ brick cache
def sg_cache_put(vol, channel, timepoint, level, coords, regions, stream=None):
    """Store whole bricks (regions [n, B+2, B+2, B+2], core plus apron, x
    fastest; numpy or a device tensor) of one (channel, timepoint, level)."""
    coords = np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 3)
    on_dev = not isinstance(regions, np.ndarray) and getattr(regions, "is_cuda", False)
    if isinstance(regions, np.ndarray):
        regions = np.ascontiguousarray(regions)
    else:
        regions = regions.contiguous()
    _check(_lib.sg_cache_put(vol, int(channel), int(timepoint), int(level), len(coords),
                             coords.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(regions),
                             int(bool(on_dev)), _stream(stream)), "sg_cache_put")


def sg_cache_put_scattered(vol, channel, timepoint, level, coords, addrs, stream=None):
    """Store whole bricks of one (channel, timepoint, level) whose regions
    ([B+2]^3 voxels each) sit at the addresses addrs[i] (integers: host or
    device pointers), one DMA per brick."""
    coords = np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 3)
    addrs = np.ascontiguousarray(addrs, dtype=np.uint64).reshape(-1)
    if len(addrs) != len(coords):
        raise ValueError("one address per brick")
    _check(_lib.sg_cache_put_scattered(vol, int(channel), int(timepoint), int(level),
                                       len(coords), coords.ctypes.data_as(C.POINTER(C.c_int32)),
                                       addrs.ctypes.data_as(C.POINTER(C.c_void_p)),
                                       _stream(stream)), "sg_cache_put_scattered")


def sg_cache_requests(vol, stream=None):
    """Requested nodes since the last call: (ids uint64, timepoints int32)."""
    n = C.c_int32(0)
    st = _lib.sg_cache_requests(vol, None, None, C.byref(n), _stream(stream))
    if st == SG_OK:
        return np.zeros(0, np.uint64), np.zeros(0, np.int32)
    if st != SG_ERR_INVALID_ARG:
        _check(st, "sg_cache_requests")
    ids = np.zeros(n.value, np.uint64)
    tps = np.zeros(n.value, np.int32)
    _check(_lib.sg_cache_requests(vol, ids.ctypes.data_as(C.POINTER(C.c_uint64)),
                                  tps.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n),
                                  _stream(stream)), "sg_cache_requests")
    return ids[:n.value], tps[:n.value]



# ------------------------------------------------------- out-of-core import
def _voxel_dtype(t) -> int:
    if t.element_size() == 1:
        return SG_U8
    if t.element_size() == 2:
        return SG_U16
    raise ValueError("voxel arrays are 8- or 16-bit")


def sg_pyramid_level(src, dst, stream=None):
    """One coarser pyramid level: src and dst are contiguous device tensors
    [z, y, x] of 8- or 16-bit voxels, dst of shape ceil(src.shape / 2)."""
    want = tuple(-(-int(n) // 2) for n in src.shape)
    if tuple(dst.shape) != want or dst.element_size() != src.element_size():
        raise ValueError("dst must have shape %s and src's voxel size" % (want,))
    if not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous")
    dims = (C.c_int32 * 3)(*[int(n) for n in src.shape[::-1]])
    _check(_lib.sg_pyramid_level(_voxel_dtype(src), dims, _ptr(src), _ptr(dst),
                                 _stream(stream)), "sg_pyramid_level")


def sg_brick_regions(level, brick, coords, out, stream=None):
    """Whole bricks (core plus one-voxel apron, clamped) of the device level
    tensor [z, y, x] at coords [n, 3] = (bx, by, bz) into the device tensor
    out [n, B+2, B+2, B+2]."""
    coords = np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 3)
    S = int(brick) + 2
    if tuple(out.shape) != (len(coords), S, S, S) or out.element_size() != level.element_size():
        raise ValueError("out must be [n, B+2, B+2, B+2] of the level's voxel size")
    if not (level.is_contiguous() and out.is_contiguous()):
        raise ValueError("level and out must be contiguous")
    dims = (C.c_int32 * 3)(*[int(n) for n in level.shape[::-1]])
    _check(_lib.sg_brick_regions(_voxel_dtype(level), dims, _ptr(level), int(brick), len(coords),
                                 coords.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(out),
                                 _stream(stream)), "sg_brick_regions")

def sg_cache_get_info(vol) -> dict:
    o = sg_cache_info()
    _check(_lib.sg_cache_get_info(vol, C.byref(o)), "sg_cache_get_info")
    return {k: int(getattr(o, k)) for k, _ in sg_cache_info._fields_}


def sg_cache_resident(vol, channel, timepoint, level, b) -> bool:
    bb = (C.c_int32 * 3)(*[int(x) for x in b])
    r = C.c_int32()
    _check(_lib.sg_cache_resident(vol, int(channel), int(timepoint), int(level), bb,
                                  C.byref(r)), "sg_cache_resident")
    return bool(r.value)
