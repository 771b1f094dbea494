"""Pack a linear volume into brick cores and upload it (input marshalling).

``sg_upload_bricks`` takes consecutive brick cores of brick^3 voxels,
x fastest. These helpers cut a linear [z, y, x] array (numpy on the host or
a torch tensor on the device) into that layout, padding partial bricks at
the far faces (their out-of-extent voxels are replaced on the device by the
clamped edge values at commit).
"""
from __future__ import annotations

import numpy as np

from . import sg


def pack_bricks(vol, brick: int, z_range=None):
    """Return (coords [n, 3] int32 as (bx, by, bz), cores [n, B, B, B]).

    ``vol`` is indexed [z, y, x]; works on numpy arrays and torch tensors.
    ``z_range`` = (bz0, bz1) restricts the output to brick layers bz0..bz1-1.
    """
    nz, ny, nx = vol.shape
    B = int(brick)
    gx, gy, gz = -(-nx // B), -(-ny // B), -(-nz // B)
    z0, z1 = (0, gz) if z_range is None else z_range
    sub = vol[z0 * B:min(z1 * B, nz)]
    pz = (z1 - z0) * B - sub.shape[0]
    py, px = gy * B - ny, gx * B - nx
    if isinstance(vol, np.ndarray):
        sub = np.pad(sub, ((0, pz), (0, py), (0, px)), mode="edge")
        cores = sub.reshape(z1 - z0, B, gy, B, gx, B).transpose(0, 2, 4, 1, 3, 5)
        cores = np.ascontiguousarray(cores).reshape(-1, B, B, B)
    else:
        import torch
        if pz or py or px:
            sub = torch.nn.functional.pad(sub[None, None].float(), (0, px, 0, py, 0, pz),
                                          mode="replicate")[0, 0].to(vol.dtype)
        cores = sub.reshape(z1 - z0, B, gy, B, gx, B).permute(0, 2, 4, 1, 3, 5)
        cores = cores.contiguous().reshape(-1, B, B, B)
    bz, by, bx = np.meshgrid(np.arange(z0, z1), np.arange(gy), np.arange(gx), indexing="ij")
    coords = np.stack([bx.ravel(), by.ravel(), bz.ravel()], axis=1).astype(np.int32)
    return coords, cores


def upload_volume(vol_handle, data, brick: int, channel=0, timepoint=0, stream=None,
                  build_lod=True, layers_per_call=None):
    """Upload a whole level-0 volume ([z, y, x]) and build its pyramid."""
    nz = data.shape[0]
    gz = -(-nz // brick)
    step = layers_per_call or gz
    for z0 in range(0, gz, step):
        coords, cores = pack_bricks(data, brick, (z0, min(gz, z0 + step)))
        sg.sg_upload_bricks(vol_handle, channel, timepoint, 0, coords, cores, stream=stream)
    if build_lod:
        sg.sg_build_lod(vol_handle, channel, timepoint, stream=stream)
