"""Drivers of the GPU/CPU generator (gen.hip) for the large workloads.

``TubeVolume`` is the 2048^3 uint16 bricked stereo workload: 400 branching
Gaussian tubes (radius 1-6, intensity 2000-60000) over Poisson(200).
``CellVolume`` is one timepoint of the 3-channel 1024x1024x512 uint16 time
series: 200 moving Gaussian cells per channel over 4 broad Gaussians.
Both evaluate any box region either on the GPU (torch tensor out) or on the
CPU (numpy out), from the same seeded primitive lists.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import (CELLS_BRICK, CELLS_DIMS, TUBES_BRICK, TUBES_DIMS, bin_primitives, cell_tracks,
               poisson_cdf, tube_geometry)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libsggen.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            from . import build
            build.build()
        import torch  # noqa: F401  -- torch's HIP runtime first: see paper_1804_08197_amd/sg.py
        L = C.CDLL(_LIB)
        vp = C.c_void_p
        L.sggen_tubes.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp, vp, vp, vp, C.c_int32,
                                  C.c_uint64, C.c_int32, vp]
        L.sggen_cells.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp, vp, C.c_float,
                                  C.c_int32, vp]
        _lib = L
    return _lib


def _addr(x):
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


class _Base:
    dims: tuple
    bin: int

    def _tables(self):
        raise NotImplementedError

    def to_device(self, device="cuda"):
        import torch
        self.dev = {k: torch.from_numpy(np.ascontiguousarray(v)).to(device)
                    for k, v in self._tables().items()}
        return self

    def region(self, org, size, device=False, out=None, stream=None):
        """Voxels of the box [org, org + size) as a [z, y, x] array (numpy on
        the CPU, or a torch tensor on the device when device=True)."""
        org_a = np.asarray(org, dtype=np.int64)
        size_a = np.asarray(size, dtype=np.int32)
        dims_a = np.asarray(self.dims, dtype=np.int32)
        shape = (int(size[2]), int(size[1]), int(size[0]))
        if device:
            import torch
            if out is None:
                out = torch.empty(shape, dtype=torch.uint16, device="cuda")
            st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
            rc = self._call(out, org_a, size_a, dims_a, self.dev, 1, st)
        else:
            out = np.empty(shape, dtype=np.uint16) if out is None else out
            rc = self._call(out, org_a, size_a, dims_a, self._tables(), 0, 0)
        if rc != 0:
            raise RuntimeError("generator failed (%d)" % rc)
        return out


class TubeVolume(_Base):
    def __init__(self, seed=1002, dims=TUBES_DIMS, bin_edge=TUBES_BRICK, **kw):
        self.dims, self.bin, self.seed = tuple(dims), int(bin_edge), int(seed)
        p0, p1, r, amp, bid = tube_geometry(seed=seed, dims=dims, **kw)
        pad = 3.0 * r[:, None]
        off, ids = bin_primitives(np.minimum(p0, p1) - pad, np.maximum(p0, p1) + pad, dims,
                                  self.bin)
        self.A = np.concatenate([p0, r[:, None]], axis=1).astype(np.float32)
        self.Bv = np.concatenate([p1, amp[:, None]], axis=1).astype(np.float32)
        self.br = bid.astype(np.int32)
        self.off = off.astype(np.int64)
        self.ids = ids.astype(np.int32)
        self.cdf = poisson_cdf(200.0, 400)
        self.n_segments = len(p0)

    def _tables(self):
        return {"A": self.A, "Bv": self.Bv, "br": self.br, "off": self.off, "ids": self.ids,
                "cdf": self.cdf}

    def _call(self, out, org, size, dims, t, on_dev, stream):
        return lib().sggen_tubes(_addr(out), org.ctypes.data, size.ctypes.data, dims.ctypes.data,
                                 self.bin, _addr(t["A"]), _addr(t["Bv"]), _addr(t["br"]),
                                 _addr(t["off"]), _addr(t["ids"]), _addr(t["cdf"]),
                                 len(self.cdf) - 1, self.seed, on_dev, stream)


class CellVolume(_Base):
    def __init__(self, channel, timepoint, dims=CELLS_DIMS, bin_edge=CELLS_BRICK, **kw):
        self.dims, self.bin = tuple(dims), int(bin_edge)
        pos, sig, amp, bg_c, bg_a = cell_tracks(channel, timepoint, dims=dims, **kw)
        pad = 3.0 * sig[:, None]
        off, ids = bin_primitives(pos - pad, pos + pad, dims, self.bin)
        cells = np.zeros((len(pos), 2, 4), dtype=np.float32)
        cells[:, 0, :3] = pos
        cells[:, 1, 0] = sig
        cells[:, 1, 1] = amp
        self.cells = cells.reshape(-1, 4)
        self.bg = np.concatenate([bg_c, bg_a[:, None]], axis=1).astype(np.float32)
        self.off = off.astype(np.int64)
        self.ids = ids.astype(np.int32)
        self.bg_sigma = 200.0

    def _tables(self):
        return {"cells": self.cells, "off": self.off, "ids": self.ids, "bg": self.bg}

    def _call(self, out, org, size, dims, t, on_dev, stream):
        return lib().sggen_cells(_addr(out), org.ctypes.data, size.ctypes.data, dims.ctypes.data,
                                 self.bin, _addr(t["cells"]), _addr(t["off"]), _addr(t["ids"]),
                                 _addr(t["bg"]), self.bg_sigma, on_dev, stream)


def upload_generated(sg_handle, genvol, brick, channel=0, timepoint=0, host_out=None,
                     slab_bricks=1, build_lod=True):
    """Generate a volume on the GPU slab by slab (slab_bricks brick layers at
    a time), upload each slab's bricks, optionally copy it into ``host_out``
    ([z, y, x] numpy), then build the pyramid on the device."""
    import torch

    from paper_1804_08197_amd import pack_bricks, sg
    nx, ny, nz = genvol.dims
    gz = -(-nz // brick)
    for bz in range(0, gz, slab_bricks):
        z0 = bz * brick
        z1 = min(nz, (bz + slab_bricks) * brick)
        slab = genvol.region((0, 0, z0), (nx, ny, z1 - z0), device=True)
        coords, cores = pack_bricks(slab, brick)
        coords[:, 2] += bz
        sg.sg_upload_bricks(sg_handle, channel, timepoint, 0, coords, cores)
        if host_out is not None:
            host_out[z0:z1] = slab.cpu().numpy()
        del cores, slab
    if build_lod:
        sg.sg_build_lod(sg_handle, channel, timepoint)
    torch.cuda.synchronize()
