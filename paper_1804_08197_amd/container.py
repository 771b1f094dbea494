"""Host-side brick container and loader for out-of-core volumes.

Sec 4.1 stores a volume as chunks at several resolutions, made once at
import; Sec 4.2 keeps recently used chunks in a GPU cache and Sec 5.2 loads
the blocks a render asks for. This module is that import step and loader
for a cache volume (``sg_volume_create(..., cache_slots=...)``); the voxel
work runs in the library, this module allocates, calls and copies:

* ``build_levels`` makes the resolution pyramid of a level-0 array on the
  device, one ``sg_pyramid_level`` call per level;
* ``brick_regions`` cuts whole bricks (core plus a one-voxel apron) out of a
  level with ``sg_brick_regions``;
* ``BrickSource`` holds the pyramids of every (timepoint, channel) and
  answers the cache's request list with ``sg_cache_put`` calls;
* ``HostBrickStore`` keeps every brick in page-locked host memory (the CPU
  tier) and answers requests with ``sg_cache_put_scattered``.

Arrays are torch tensors [z, y, x] of 8- or 16-bit voxels; numpy inputs are
moved to the current device first.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

from . import sg


def _on_device(a):
    """A contiguous device tensor holding a (numpy or torch) voxel array."""
    import torch
    if isinstance(a, np.ndarray):
        a = np.ascontiguousarray(a)
        if a.dtype == np.uint16:  # moved as int16 bits: the copy kernels take either
            return torch.from_numpy(a.view(np.int16)).cuda().view(torch.uint16)
        return torch.from_numpy(a).cuda()
    if not a.is_cuda:
        if a.dtype == torch.uint16:
            return a.view(torch.int16).contiguous().cuda().view(torch.uint16)
        return a.contiguous().cuda()
    return a.contiguous()


def build_levels(vol0, levels: int, stream=None):
    """[level-0, level-1, ...] device tensors of the pyramid of vol0."""
    import torch
    out = [_on_device(vol0)]
    for _ in range(1, levels):
        src = out[-1]
        dst = torch.empty([-(-int(n) // 2) for n in src.shape], dtype=src.dtype,
                          device=src.device)
        sg.sg_pyramid_level(src, dst, stream=stream)
        out.append(dst)
    return out


def brick_regions(level, brick: int, coords, stream=None):
    """Device tensor [n, B+2, B+2, B+2] of the bricks coords [n, 3] =
    (bx, by, bz) of a level (a device tensor [z, y, x])."""
    import torch
    coords = np.asarray(coords, dtype=np.int32).reshape(-1, 3)
    S = int(brick) + 2
    out = torch.empty((len(coords), S, S, S), dtype=level.dtype, device=level.device)
    sg.sg_brick_regions(level, brick, coords, out, stream=stream)
    return out


def decode_ids(ids):
    ids = np.asarray(ids, dtype=np.uint64)
    return ((ids >> np.uint64(60)).astype(np.int64),
            np.stack([((ids >> np.uint64(40)) & np.uint64(0xFFFFF)).astype(np.int64),
                      ((ids >> np.uint64(20)) & np.uint64(0xFFFFF)).astype(np.int64),
                      (ids & np.uint64(0xFFFFF)).astype(np.int64)], axis=1))


class BrickSource:
    """Pyramids of every (timepoint, channel) of a cache volume, and the
    loader that serves its requests."""

    def __init__(self, handle, brick: int, levels: int):
        self.h = handle
        self.B = int(brick)
        self.levels = int(levels)
        self.pyr = {}

    def add(self, timepoint: int, channel: int, vol0):
        self.pyr[(int(timepoint), int(channel))] = build_levels(vol0, self.levels)

    def channels(self, timepoint):
        return sorted(c for (t, c) in self.pyr if t == timepoint)

    def put(self, timepoint, level, coords, stream=None):
        """Store the bricks coords of one level of every channel of one
        timepoint."""
        coords = np.asarray(coords, dtype=np.int32).reshape(-1, 3)
        if not len(coords):
            return
        for c in self.channels(timepoint):
            reg = brick_regions(self.pyr[(timepoint, c)][level], self.B, coords)
            sg.sg_cache_put(self.h, c, timepoint, level, coords, reg, stream=stream)

    def put_top(self, timepoint, stream=None):
        """Every top-level brick (renders need them resident)."""
        L = self.levels - 1
        a = self.pyr[(timepoint, self.channels(timepoint)[0])][L]
        g = [-(-s // self.B) for s in a.shape[::-1]]
        bz, by, bx = np.meshgrid(np.arange(g[2]), np.arange(g[1]), np.arange(g[0]),
                                 indexing="ij")
        self.put(timepoint, L, np.stack([bx.ravel(), by.ravel(), bz.ravel()], 1), stream)

    def serve_requests(self, max_bricks=None, stream=None) -> int:
        """Load what the renders since the last call asked for (up to
        max_bricks nodes, coarsest first); returns the number of nodes."""
        ids, tps = sg.sg_cache_requests(self.h, stream=stream)
        if not len(ids):
            return 0
        L, b = decode_ids(ids)
        order = np.lexsort((ids, -L))
        if max_bricks is not None:
            order = order[:max_bricks]
        groups = defaultdict(list)
        for i in order:
            groups[(int(tps[i]), int(L[i]))].append(b[i])
        for (t, lev), cs in groups.items():
            self.put(t, lev, np.array(cs), stream)
        return len(order)


def level_grids(dims, brick: int, levels: int):
    """Brick grid (x, y, z) of every level: level dims halve with rounding
    up; a level is cut into ceil(n / brick) bricks per axis."""
    d = [int(x) for x in dims]
    out = []
    for _ in range(levels):
        out.append(tuple(-(-x // brick) for x in d))
        d = [-(-x // 2) for x in d]
    return out


def grid_coords(grid):
    """Every brick (bx, by, bz) of a grid, x fastest."""
    bz, by, bx = np.meshgrid(np.arange(grid[2]), np.arange(grid[1]), np.arange(grid[0]),
                             indexing="ij")
    return np.stack([bx.ravel(), by.ravel(), bz.ravel()], 1)


class HostBrickStore:
    """The CPU-memory tier beside the GPU cache (Sec 4.2): whole bricks (core
    plus apron) of every registered (timepoint, channel) pyramid, kept in
    page-locked host chunks (1 GiB by default), and the loader that answers a cache
    volume's requests from them with one DMA per brick
    (``sg_cache_put_scattered``), as a chunk cache hands chunks to the GPU.

    ``add`` takes a level-0 volume on the device (torch [z, y, x]) or the
    host (numpy), builds its pyramid, cuts every brick and copies it into
    the chunks; ``served_bytes`` counts what the loader has sent."""

    def __init__(self, handle, dims, brick: int, levels: int, itemsize: int = 2,
                 chunk_bytes: int = 1 << 30):
        self.h = handle
        self.chunk_bytes = int(chunk_bytes)
        self.B = int(brick)
        self.levels = int(levels)
        self.grids = level_grids(dims, self.B, self.levels)
        self.itemsize = int(itemsize)
        self.region_bytes = (self.B + 2) ** 3 * self.itemsize
        self.per_chunk = self.chunk_bytes // self.region_bytes
        if self.per_chunk < 1:
            raise ValueError("a brick region is larger than a host chunk")
        self.chunks = []
        self.next = self.per_chunk  # regions used in the newest chunk
        self.addr = {}  # (timepoint, channel, level) -> host addresses, brick order x fastest
        self.served_bytes = 0
        self.served_nodes = 0

    def host_bytes(self) -> int:
        return len(self.chunks) * self.chunk_bytes

    def _slots(self, k):
        """(chunk tensor, first region index, count <= k) of the next free run."""
        import torch
        if self.next == self.per_chunk:
            self.chunks.append(torch.empty(self.chunk_bytes, dtype=torch.uint8, pin_memory=True))
            self.next = 0
        m = min(k, self.per_chunk - self.next)
        first = self.next
        self.next += m
        return self.chunks[-1], first, m

    def channels(self, timepoint):
        return sorted({c for (t, c, _) in self.addr if t == timepoint})

    def add(self, timepoint: int, channel: int, vol0, batch: int = 256):
        import torch
        dt = {1: torch.uint8, 2: torch.uint16}[self.itemsize]
        S = self.B + 2
        for lev, arr in enumerate(build_levels(vol0, self.levels)):
            coords = grid_coords(self.grids[lev])
            addrs = np.zeros(len(coords), np.uint64)
            i = 0
            while i < len(coords):
                chunk, first, m = self._slots(min(batch, len(coords) - i))
                reg = brick_regions(arr, self.B, coords[i:i + m])
                off = first * self.region_bytes
                dst = chunk[off:off + m * self.region_bytes].view(dt).view(m, S, S, S)
                dst.copy_(reg)
                addrs[i:i + m] = chunk.data_ptr() + off + \
                    np.arange(m, dtype=np.uint64) * np.uint64(self.region_bytes)
                i += m
            self.addr[(int(timepoint), int(channel), lev)] = addrs

    def _put(self, timepoint, level, coords, stream=None):
        g = self.grids[level]
        lin = (coords[:, 2] * g[1] + coords[:, 1]) * g[0] + coords[:, 0]
        order = np.argsort(lin, kind="stable")  # storage order: neighbours travel together
        coords, lin = coords[order], lin[order]
        chans = self.channels(timepoint)
        for c in chans:
            sg.sg_cache_put_scattered(self.h, c, timepoint, level, coords,
                                      self.addr[(timepoint, c, level)][lin], stream=stream)
        self.served_bytes += len(coords) * len(chans) * self.region_bytes
        self.served_nodes += len(coords)

    def put_top(self, timepoint, stream=None):
        """Every top-level brick of every channel (renders need them)."""
        L = self.levels - 1
        self._put(int(timepoint), L, grid_coords(self.grids[L]), stream)

    def serve_requests(self, stream=None) -> int:
        """Load every node the renders since the last call asked for (all
        channels of its timepoint); returns the number of nodes."""
        ids, tps = sg.sg_cache_requests(self.h, stream=stream)
        if not len(ids):
            return 0
        L, b = decode_ids(ids)
        groups = defaultdict(list)
        for i in np.lexsort((ids, -L)):
            groups[(int(tps[i]), int(L[i]))].append(b[i])
        for (t, lev), cs in groups.items():
            self._put(t, lev, np.asarray(cs, dtype=np.int64), stream)
        return len(ids)
