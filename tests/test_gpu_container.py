"""The library's import step for out-of-core volumes (sg_pyramid_level,
sg_brick_regions; Sec 4.1 chunks at several resolutions, Sec 5.2 pyramid)
against the oracle, byte for byte, through the C-ABI: every level of the
pyramid, and bricks (core plus clamped one-voxel apron) at the corners,
edges and interior of ragged levels, 8- and 16-bit voxels."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _host(t):
    import torch
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


@pytest.mark.parametrize("shape,brick,levels", [((40, 48, 56), 8, 4), ((21, 24, 27), 4, 5),
                                                ((1, 1, 1), 2, 1), ((33, 7, 65), 16, 3),
                                                ((70, 66, 130), 64, 3)])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_pyramid_and_regions_equal_the_oracle(shape, brick, levels, dtype):
    from paper_1804_08197_amd.container import (brick_regions, build_levels, grid_coords,
                                                level_grids)
    print("container case", shape, brick, levels, dtype.__name__, flush=True)
    rng = np.random.default_rng(sum(shape) + brick)
    vol = rng.integers(0, np.iinfo(dtype).max + 1, size=shape, dtype=dtype)
    dims0 = shape[::-1]
    grids = level_grids(dims0, brick, levels)
    ref = oracle.pyramid(vol, levels)
    pyr = build_levels(vol, levels)
    for L in range(levels):
        got = _host(pyr[L])
        assert got.dtype == dtype and np.array_equal(got, ref[L]), L
        coords = grid_coords(grids[L])
        pick = coords[rng.permutation(len(coords))[:24]]
        regs = _host(brick_regions(pyr[L], brick, pick))
        for i, b in enumerate(pick):
            assert np.array_equal(regs[i], oracle.brick_region(ref[L], brick, b)), (L, b)


def test_import_calls_reject_bad_arguments():
    import torch

    from paper_1804_08197_amd import sg
    lvl = torch.zeros((9, 10, 11), dtype=torch.uint8, device="cuda")
    out = torch.empty((1, 6, 6, 6), dtype=torch.uint8, device="cuda")
    for coords in ([[3, 0, 0]], [[0, -1, 0]], [[0, 0, 3]]):  # grid is 3 x 3 x 3 at brick 4
        with pytest.raises(sg.SgError) as ex:
            sg.sg_brick_regions(lvl, 4, coords, out)
        assert ex.value.status == sg.SG_ERR_INVALID_ARG
    with pytest.raises(sg.SgError) as ex:
        sg.sg_brick_regions(lvl, 3, [[0, 0, 0]], torch.empty((1, 5, 5, 5), dtype=torch.uint8,
                                                             device="cuda"))
    assert ex.value.status == sg.SG_ERR_INVALID_ARG
    # a destination that overlaps its source
    big = torch.zeros(9 * 10 * 11 + 5 * 5 * 6, dtype=torch.uint8, device="cuda")
    with pytest.raises(sg.SgError) as ex:
        sg.sg_pyramid_level(big[:990].view(9, 10, 11), big[5:155].view(5, 5, 6))
    assert ex.value.status == sg.SG_ERR_INVALID_ARG
