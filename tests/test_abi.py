"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/sg.h, the ctypes structures match the C layout,
and argument errors are reported without touching a device."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sg.h")


@pytest.fixture(scope="module")
def sg():
    lib = os.path.join(ROOT, "paper_1804_08197_amd", "libsg.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    from paper_1804_08197_amd import sg as mod
    return mod


def declared_functions():
    """Every function declared in include/*.h."""
    import glob
    names = set()
    for h in sorted(glob.glob(os.path.join(os.path.dirname(HEADER), "*.h"))):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(sg_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sg_volume_create", "sg_upload_bricks", "sg_set_transfer_function",
              "sg_render_views", "sg_volume_destroy", "sg_build_lod", "sg_volume_commit",
              "sg_get_lod_cut", "sg_render_views_stats", "sg_status_string", "sg_last_error",
              "sg_abi_version", "sg_volume_memory", "sg_up_forward", "sg_up_train_step",
              "sg_cache_put", "sg_render_graph_launch", "sg_autotune"):
        assert n in names


def test_library_exports_every_declared_symbol(sg):
    lib = sg.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", sg.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (sg_\w+)", out))
    assert set(declared_functions()) <= exported


def test_struct_layout_matches_c(sg):
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "sg.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(sg_volume_desc), sizeof(sg_view),
         sizeof(sg_render_params), sizeof(sg_render_stats));
  printf("%zu %zu %zu %zu %zu\n", offsetof(sg_view, width), offsetof(sg_render_params, lod_bias),
         offsetof(sg_render_params, flags), offsetof(sg_render_params, depth_alpha),
         offsetof(sg_render_stats, microblocks));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(sg_view, lens), offsetof(sg_view, ray_limit),
         offsetof(sg_render_params, model), offsetof(sg_render_params, planes),
         offsetof(sg_render_params, roi), sizeof(sg_launch_config));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), c, "-o", exe],
                       check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(x) for x in lines[0].split()]
    offs = [int(x) for x in lines[1].split()]
    assert sizes == [C.sizeof(sg.sg_volume_desc), C.sizeof(sg.sg_view),
                     C.sizeof(sg.sg_render_params), C.sizeof(sg.sg_render_stats)]
    assert offs == [sg.sg_view.width.offset, sg.sg_render_params.lod_bias.offset,
                    sg.sg_render_params.flags.offset, sg.sg_render_params.depth_alpha.offset,
                    sg.sg_render_stats.microblocks.offset]
    more = [int(x) for x in lines[2].split()]
    assert more == [sg.sg_view.lens.offset, sg.sg_view.ray_limit.offset,
                    sg.sg_render_params.model.offset, sg.sg_render_params.planes.offset,
                    sg.sg_render_params.roi.offset, C.sizeof(sg.sg_launch_config)]


def test_version_and_status_strings(sg):
    assert sg.sg_abi_version() == sg.SG_ABI_VERSION == 5
    for code, name in [(0, "SG_OK"), (-1, "SG_ERR_INVALID_ARG"), (-2, "SG_ERR_OUT_OF_MEMORY"),
                       (-3, "SG_ERR_DEVICE"), (-4, "SG_ERR_STATE"), (-5, "SG_ERR_UNSUPPORTED")]:
        assert sg.sg_status_string(code) == name
    assert sg.sg_status_string(42) == "SG_ERR_UNKNOWN"


@pytest.mark.parametrize("kw", [
    dict(dims=(0, 8, 8)), dict(dims=(8, 8, 8), channels=5), dict(dims=(8, 8, 8), channels=0),
    dict(dims=(8, 8, 8), timepoints=0), dict(dims=(8, 8, 8), dtype=3),
    dict(dims=(8, 8, 8), brick=48), dict(dims=(8, 8, 8), brick=1), dict(dims=(8, 8, 8), brick=512),
    dict(dims=(8, 8, 8), levels=0), dict(dims=(8, 8, 8), levels=17),
    dict(dims=(8, 8, 8), device=-1), dict(dims=(8, 8, 8), layout=2),
    dict(dims=(8, 8, 8), layout=-1)])
def test_create_rejects_bad_descriptions_without_a_device(sg, kw):
    with pytest.raises(sg.SgError) as ex:
        sg.sg_volume_create(**kw)
    assert ex.value.status == sg.SG_ERR_INVALID_ARG
    assert sg.sg_last_error()


def test_null_arguments_are_invalid(sg):
    lib = sg.lib()
    assert lib.sg_volume_create(None, None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_volume_destroy(None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_volume_commit(None, None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_build_lod(None, 0, 0, None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_upload_bricks(None, 0, 0, 0, 0, None, None, 0, None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_set_transfer_function(None, 0, None, 256, 0.0, 1.0) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_render_views(None, 1, None, None, None, None, None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_render_views_stats(None, 1, None, None, None, None, None, None) == \
        sg.SG_ERR_INVALID_ARG
    assert lib.sg_get_lod_cut(None, None, None, None, None, None, None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_volume_memory(None, None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_render_views_if(None, 1, None, None, None, None, None, None) == \
        sg.SG_ERR_INVALID_ARG
    assert lib.sg_cache_put_scattered(None, 0, 0, 0, 1, None, None, None) == \
        sg.SG_ERR_INVALID_ARG
    assert lib.sg_composite_over(None, 1, None, None, None, None) == sg.SG_ERR_INVALID_ARG
    from paper_1804_08197_amd import upsampler as up
    assert up._lib.sg_up_forward_flag(None, 1, 1, 1, None, None, None, 1.0, None, None, 40.0,
                                      None, None) == sg.SG_ERR_INVALID_ARG
    assert up._lib.sg_up_forward(None, 1, 1, 1, None, None, None, 1.0, None, None, None,
                                 None) == sg.SG_ERR_INVALID_ARG
    assert up._lib.sg_up_set_fused(None, 1) == sg.SG_ERR_INVALID_ARG


def test_valid_description_without_gpu_reports_device_error(sg):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: covered by the GPU tests")
    with pytest.raises(sg.SgError) as ex:
        sg.sg_volume_create((64, 64, 64), brick=16, levels=3)
    assert ex.value.status == sg.SG_ERR_DEVICE


def test_pack_bricks_layout():
    from paper_1804_08197_amd import pack_bricks
    v = np.arange(5 * 6 * 7, dtype=np.uint16).reshape(5, 6, 7)
    coords, cores = pack_bricks(v, 4)
    assert coords.shape == (8, 3) and cores.shape == (8, 4, 4, 4)
    for (bx, by, bz), core in zip(coords, cores):
        for z in range(4):
            for y in range(4):
                for x in range(4):
                    gz, gy, gx = min(4 * bz + z, 4), min(4 * by + y, 5), min(4 * bx + x, 6)
                    assert core[z, y, x] == v[gz, gy, gx]


def test_composite_argument_checks_need_no_device(sg):
    """sg_composite_over rejects bad part counts, misaligned images and
    empty or non-finite boxes before it touches a device."""
    import ctypes as C

    import gen
    lib = sg.lib()
    v = sg.make_view(gen.view(gen.look_at((-100.0, 50.0, 40.0), (16, 16, 16)), 8, 6, 0.5))
    buf = np.zeros(8 * 6 * 4 + 8, np.float32)
    base = buf.ctypes.data + (-buf.ctypes.data) % 16
    parts = (C.c_void_p * 2)(base, base)
    out = C.c_void_p(base)

    def call(n, boxes, arr=parts, o=out):
        b = np.ascontiguousarray(np.asarray(boxes, np.float64))
        return lib.sg_composite_over(C.byref(v), n, arr, b.ctypes.data_as(C.POINTER(C.c_double)),
                                     o, None)
    good = [[0, 0, 0, 16, 32, 32], [16, 0, 0, 32, 32, 32]]
    assert call(0, good) == sg.SG_ERR_INVALID_ARG
    assert call(9, good * 5) == sg.SG_ERR_INVALID_ARG
    assert call(2, [[0, 0, 0, 16, 32, 32], [16, 0, 0, 16, 32, 32]]) == sg.SG_ERR_INVALID_ARG
    assert call(2, [[0, 0, 0, 16, 32, 32], [16, 0, np.nan, 32, 32, 32]]) == sg.SG_ERR_INVALID_ARG
    assert call(2, good, arr=(C.c_void_p * 2)(base, base + 4)) == sg.SG_ERR_INVALID_ARG
    assert call(2, good, o=C.c_void_p(base + 8)) == sg.SG_ERR_INVALID_ARG


def test_import_calls_check_arguments_without_a_device(sg):
    """sg_pyramid_level and sg_brick_regions reject bad dtypes, dims, bricks
    and coordinates before any device work; n = 0 is a no-op."""
    lib = sg.lib()
    dims = (C.c_int32 * 3)(11, 10, 9)
    p = C.c_void_p(4096)
    cz = (C.c_int32 * 3)(0, 0, 0)
    assert lib.sg_pyramid_level(3, dims, p, C.c_void_p(1 << 20), None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_pyramid_level(1, None, p, p, None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_pyramid_level(1, (C.c_int32 * 3)(0, 1, 1), p, p, None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_pyramid_level(2, dims, None, p, None) == sg.SG_ERR_INVALID_ARG
    # overlapping source and destination
    assert lib.sg_pyramid_level(1, dims, p, C.c_void_p(4096 + 100), None) == \
        sg.SG_ERR_INVALID_ARG
    assert lib.sg_brick_regions(1, dims, p, 3, 1, cz, p, None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_brick_regions(1, dims, p, 4, -1, cz, p, None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_brick_regions(1, dims, p, 4, 1, (C.c_int32 * 3)(3, 0, 0), p, None) == \
        sg.SG_ERR_INVALID_ARG
    assert lib.sg_brick_regions(1, dims, p, 4, 1, cz, None, None) == sg.SG_ERR_INVALID_ARG
    assert lib.sg_brick_regions(2, dims, p, 4, 0, None, None, None) == sg.SG_OK


def test_binding_shares_torch_hip_runtime_whatever_the_import_order():
    """Importing the binding before torch must not load a second HIP
    runtime: the library would then hold its own runtime and receive
    torch's pointers and streams from another one."""
    code = ("from paper_1804_08197_amd import sg\n"
            "import torch, re\n"
            "m = open('/proc/self/maps').read()\n"
            "print(len(set(re.findall(r'\\S*libamdhip64\\S*', m))))\n")
    out = subprocess.run(["python", "-c", code], capture_output=True, text=True, cwd=ROOT,
                         check=True).stdout.split()
    assert out[-1] == "1"


def test_view_packing_and_prebuilt_arrays(sg):
    """make_view packs every field of a view dict (checked field by field
    against the dict); the render calls' helpers pass prebuilt view,
    pointer and launch structures through untouched."""
    import math

    import gen
    rng = np.random.default_rng(5)
    v = gen.view(gen.look_at(rng.normal(size=3) * 300, (10.0, 20.0, 30.0)), 70, 46,
                 math.tan(math.radians(25)))
    v = dict(v, lens=(0.1, -0.2, 0.05, -0.03), ray_limit=123456, tile_any=654321)
    o = sg.make_view(v)
    assert list(o.cam_to_world) == [float(x) for x in np.asarray(v["cam_to_world"]).ravel()]
    assert (o.tan_left, o.tan_right, o.tan_bottom, o.tan_top) == (
        v["tan_left"], v["tan_right"], v["tan_bottom"], v["tan_top"])
    assert (o.width, o.height) == (70, 46)
    assert list(o.lens) == [0.1, -0.2, 0.05, -0.03]
    assert (o.ray_limit, o.tile_any) == (123456, 654321)
    plain = sg.make_view(dict(v, lens=None, ray_limit=None, tile_any=None))
    assert list(plain.lens) == [0.0] * 4 and not plain.ray_limit and not plain.tile_any
    arr = sg.views_array([v, v])
    assert sg._views(arr) is arr and bytes(arr[0]) == bytes(o)
    ptrs = sg.pointer_array([None])
    assert sg._ptrs(ptrs) is ptrs and ptrs[0] is None
    cfg = sg.launch_config_struct({"kernel": 1, "tile": 8})
    assert sg._launch_dict(cfg)["kernel"] == 1 and sg._launch_dict(cfg)["tile"] == 8
