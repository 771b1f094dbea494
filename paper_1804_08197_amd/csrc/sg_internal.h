// sg_internal.h -- shared definitions of the gfx950 library behind sg.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sg.h"

namespace sg {

constexpr int kMaxLevels = 16;
constexpr int kMaxChannels = 4;
constexpr int kMaxTfEntries = 1024;
// Pool rows (x runs of a brick slot) start on 4-byte boundaries, the unit
// in which the ray caster copies brick regions into LDS. (16-byte units move
// four times the bytes per load but widen every staged row to 8 u16 voxels,
// which costs more slabs than it saves loads on the tube workload.)
constexpr int kRowAlignBytes = 4;
// LDS staging bytes per wave of the ray caster (SG_STAGE_BYTES overrides).
constexpr int kStageBytesDefault = 8192;
// Optical models (values of sg_render_params.model).
constexpr int kModelAbsorption = SG_MODEL_EMISSION_ABSORPTION;
constexpr int kModelEmission = SG_MODEL_EMISSION_ONLY;
constexpr int kModelMip = SG_MODEL_MAX_INTENSITY;

// Error plumbing: every entry point funnels through these.
sg_status fail(sg_status s, const std::string& msg);
sg_status hip_fail(hipError_t e, const char* what);
#define SG_HIP(call)                                             \
  do {                                                           \
    hipError_t e_ = (call);                                      \
    if (e_ != hipSuccess) return ::sg::hip_fail(e_, #call);      \
  } while (0)

// A kernel launch held as data: run on a stream, or added to a graph.
struct Launch {
  const void* func = nullptr;
  dim3 grid{1, 1, 1}, block{1, 1, 1};
  size_t lds = 0;
  std::vector<std::vector<uint8_t>> arg;  // a copy of each kernel argument
  template <typename X>
  void push(const X& x) {
    arg.emplace_back(sizeof(X));
    std::memcpy(arg.back().data(), &x, sizeof(X));
  }
  std::vector<void*> ptrs() {
    std::vector<void*> p;
    for (auto& b : arg) p.push_back(b.data());
    return p;
  }
  sg_status run(hipStream_t s) {
    std::vector<void*> p = ptrs();
    SG_HIP(hipLaunchKernel(func, grid, block, p.data(), lds, s));
    return SG_OK;
  }
};

// How the ray caster is launched (sg_launch_config in internal units).
struct LaunchConfig {
  int32_t gather = 0;       // 1: stencils read the pool (no LDS staging)
  int32_t tile_log = 1;     // log2 edge of a workgroup tile in 8x8 wave tiles: 0..2
  int32_t bt_log = 3;       // log2 edge of a screen block in 8x8 wave tiles: 2..4
  int32_t stage_bytes = kStageBytesDefault;
  int32_t persistent = 0;   // 1: persistent grid with per-XCD tile queues
};

// Node record, one per pyramid node (level L, brick b): used by the ray
// caster to turn a cut-map entry into a box and a level.
struct NodeInfo {
  int32_t level;
  int32_t b[3];
};

// Front-to-back key of node (L, b) for eye e: the octree path from a virtual
// root of key_levels levels over the volume, each child index flipped so
// that the child on the eye's side of each splitting plane comes first.
// Nodes of a cut sorted by this key are in front-to-back order for every ray
// from e (the order in which Sec 5.2 renders its blocks).
__device__ __forceinline__ uint64_t visibility_key(int key_levels, int B, const double e[3],
                                                   int L, const int b[3]) {
  uint64_t key = 0;
  for (int l = key_levels - 1; l >= L; --l) {
    uint32_t code = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int cb = b[i] >> (l - L);
      const double split = (double)((int64_t)B << l) * (double)(2 * (cb >> 1) + 1);
      const uint32_t f = (uint32_t)(cb & 1) ^ (uint32_t)(e[i] >= split);
      code = (code << 1) | f;
    }
    key = (key << 3) | code;
  }
  return key << (3 * L);
}

// Per-view constants consumed by the LOD and ray-casting kernels.
struct ViewDev {
  double e[3];
  double R[9];  // row-major rotation, camera -> world
  double tl, tr, tb, tt;
  double K;     // (tau * theta)^2
  int32_t W, H;
  int32_t tiles_x, tiles_y;  // 16x16 pixel tiles
  int32_t blocks_x;          // 4x4-tile blocks per row
  int32_t block_begin;       // first block of this view
  int64_t cut_off;     // offset of this view's cut map
  float* rgba;
  float* depth;
  int32_t* nsamp;
  const float* limit;  // per-pixel ray limit or NULL
  double lens[4];      // k1, k2, cx, cy
  int32_t lens_on;
  uint8_t* tile_any;   // per 8x8-pixel block content flag or NULL
};

// Up to kInlineViews view records travel inside the cut-map kernel's
// arguments; its first workgroup writes them to the device view table that
// the ray-casting kernel reads (stream order), so small renders need no
// host-to-device copy.
constexpr int kInlineViews = 4;
struct InlineViews {
  ViewDev v[kInlineViews];
  int32_t n;  // 0: the device table is already in place
};

// Element offset of stored voxel (x, y, z) in a pool slot, 0 <= x < Sx and
// 0 <= y, z < S. Linear slots (M = 0): rows of Sx voxels, x fastest.
// Micro-block slots (M = ceil(S / 4) >= Sx / 4): M^3 blocks of 4^3 voxels,
// each contiguous with x fastest inside it, the blocks in x-fastest order.
__host__ __device__ __forceinline__ int64_t slot_index(int x, int y, int z, int S, int Sx,
                                                       int M) {
  if (M == 0) return ((int64_t)z * S + y) * Sx + x;
  return ((((int64_t)(z >> 2) * M + (y >> 2)) * M + (x >> 2)) << 6) + ((z & 3) << 4) +
         ((y & 3) << 2) + (x & 3);
}

struct Volume {
  sg_volume_desc d{};
  int bpv = 0;       // bytes per voxel
  int B = 0;         // brick core edge
  int logB = 0;
  int S = 0;         // stored edge B + 2
  int Sx = 0;        // row stride in voxels (S rounded up to kRowAlignBytes)
  int M = 0;         // SG_LAYOUT_MICROBLOCK: 4^3 blocks per slot edge; 0: linear
  int L = 0;         // levels
  int32_t ldims[kMaxLevels][3]{};
  int32_t grid[kMaxLevels][3]{};
  int64_t node_off[kMaxLevels + 1]{};
  int64_t nodes = 0;          // nodes per (channel, timepoint)
  int64_t entries = 0;        // T * C * nodes (page table entries)
  int64_t slot_bytes = 0;     // bytes per pool slot (padded)
  int64_t slots = 0;          // pool slots (= entries unless a cache)
  uint8_t* pool = nullptr;    // [slots][S^3] voxels
  int32_t* page = nullptr;    // [T][C][nodes] -> slot, -1 if not resident
  uint32_t* range = nullptr;  // [T][C][nodes][2] min, max of stored voxels
  uint8_t* empty = nullptr;   // [T][nodes] bit 0: every channel transparent,
                              // bit 1: every channel emits nothing
  NodeInfo* info = nullptr;   // [nodes]
  float* tf = nullptr;        // [C][tf_n + 1][4] (last entry repeated)
  int tf_n = 0;
  std::vector<float> tf_host[kMaxChannels];
  double tf_lo[kMaxChannels]{}, tf_hi[kMaxChannels]{};
  bool tf_set[kMaxChannels]{};
  bool tf_dirty = true;
  std::vector<uint8_t> pending;  // [T][C] needs apron + range refresh
  bool empty_dirty = true;
  // per-render scratch
  int32_t* cutmap = nullptr;  // [views][cells0] cut node of each level-0 cell
  int64_t cutmap_cap = 0;
  uint8_t* view_dev = nullptr;
  InlineViews inline_views{};  // the last prepare_views' table when it is small
  int64_t view_cap = 0;
  // pinned staging for small uploads (view tables): a ring, so the host can
  // enqueue several renders ahead of the device
  static constexpr int kStageRing = 4;
  uint8_t* stage_host[kStageRing] = {};
  int64_t stage_cap[kStageRing] = {};
  hipEvent_t stage_done[kStageRing] = {};
  bool stage_pending[kStageRing] = {};
  int stage_next = 0;
  uint32_t* mb_bits = nullptr;  // micro-block bitmap (stats only)
  int64_t mb_words = 0;
  uint64_t* counters = nullptr;  // device counters (stats only), 16 of them
  uint64_t bytes = 0;
  // out-of-core mode (cache_slots > 0)
  bool cache = false;
  std::vector<int32_t> page_host;   // mirror of page
  std::vector<int64_t> owner;       // slot -> entry, -1 if free
  std::vector<int32_t> free_slots;
  uint32_t* stamp = nullptr;        // [slots] frame of last use
  uint32_t* req_flags = nullptr;    // [T * nodes] bits: requested since last read
  uint32_t* req_list = nullptr;     // [kReqCap] requested t * nodes + node
  uint32_t* req_count = nullptr;
  uint32_t frame = 0;
  int64_t uploads = 0, evictions = 0;
  // launch configuration of the ray caster, and the persistent grid's queues
  LaunchConfig cfg;
  uint32_t* queue = nullptr;  // 8 counters
  // kernel timing (instrumentation)
  bool timing = false;
  std::vector<hipEvent_t> ev_free;
  std::vector<hipEvent_t> ev_rec;  // triples: before cut map, before / after ray cast
};

// Capacity of the request list of a cache volume.
constexpr int kReqCap = 1 << 20;

// Record an event from the volume's pool on `s` (timing mode only).
sg_status timing_mark(Volume* v, hipStream_t s);

// Device-side current-device guard.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
};

// Stage `bytes` of host data into device memory on `stream` through the
// volume's ring of pinned buffers (waits for the copy that last used the
// slot).
sg_status stage_to_device(Volume* v, const void* host, int64_t bytes,
                          void* dev, hipStream_t stream);

// Kernel launchers (one .hip file each).
sg_status launch_upload(Volume* v, int c, int t, int level, int n,
                        const int32_t* dcoords, const void* dsrc,
                        hipStream_t s);
sg_status launch_downsample(Volume* v, int c, int t, int level_dst,
                            hipStream_t s);
sg_status launch_apron(Volume* v, int c, int t, hipStream_t s);
sg_status launch_range(Volume* v, int c, int t, hipStream_t s);
sg_status launch_empty(Volume* v, hipStream_t s);
// Cache volumes: every top-level node resident at timepoint t?
bool top_level_resident(const Volume* v, int t);
sg_status commit(Volume* v, hipStream_t s);



// Uses (and writes to the device table) v->inline_views when its n is set.
sg_status launch_cutmap(Volume* v, const ViewDev* dviews, int n_views,
                        int bias, bool lod, int timepoint, hipStream_t s,
                        const int32_t* enable = nullptr);
// rgba may be NULL (cut queries); the render path checks it itself.
sg_status prepare_views(Volume* v, int n_views, const sg_view* views,
                        const sg_render_params* p, float* const* rgba,
                        float* const* depth, int32_t* const* nsamp,
                        hipStream_t s, int* total_blocks);
// Checked host copy of the per-view constants (screen blocks of 2^bt_log
// wave tiles per side) and the number of blocks over all views.
// Checks a view (finite matrix and tangents, sizes, lens, ray-limit
// alignment, non-singular rotation) and fills its eye, rotation, tangents,
// size and lens fields; the other fields are zero.
sg_status view_geometry(const sg_view& w, ViewDev* out);
sg_status build_views(const Volume* v, int n_views, const sg_view* views,
                      const sg_render_params* p, float* const* rgba, float* const* depth,
                      int32_t* const* nsamp, int bt_log, std::vector<ViewDev>* hv,
                      int64_t* total_blocks);
// The same into a caller-provided array of n_views records.
sg_status build_views_into(const Volume* v, int n_views, const sg_view* views,
                           const sg_render_params* p, float* const* rgba, float* const* depth,
                           int32_t* const* nsamp, int bt_log, ViewDev* hv,
                           int64_t* total_blocks);
// The cut-map kernel for views already on the device, writing `cutmap`.
// enable: NULL, or a device flag read by the kernel (0: it does nothing).
// iv: NULL or n == 0, or the views to use and to write to dviews.
sg_status cutmap_launch(const Volume* v, const ViewDev* dviews, int n_views, int bias,
                        bool lod, int timepoint, int32_t* cutmap, Launch* out,
                        const int32_t* enable = nullptr, const InlineViews* iv = nullptr);
// The same cut-map kernel enqueued on `s` at once, with its arguments on
// the stack (no host or device allocation).
sg_status cutmap_run(const Volume* v, const ViewDev* dviews, int n_views, int bias, bool lod,
                     int timepoint, int32_t* cutmap, const InlineViews& iv, hipStream_t s);

struct RenderArgs {
  const uint8_t* pool;
  int64_t slot_bytes;
  const int32_t* page;   // at timepoint: [C][nodes]
  const uint8_t* empty;  // at timepoint: [nodes] skip bits (see Volume::empty)
  const uint32_t* range; // at timepoint: [C][nodes][2] stored min, max
  const NodeInfo* info;
  const float* tf;
  const int32_t* cutmap;
  int32_t key_levels;   // levels of the virtual octree over the volume
  const ViewDev* views;
  uint32_t* mb_bits;
  uint64_t* counters;
  int64_t nodes;
  int64_t level_mb_off[kMaxChannels * kMaxLevels];  // bit offsets (stats)
  int32_t ldims[kMaxLevels][3];
  float tf_scale[kMaxChannels];
  float tf_bias[kMaxChannels];
  float bg[4];
  int32_t dims[3];
  int32_t grid0[3];
  int32_t n_views;
  int32_t total_blocks;  // screen blocks over all views
  // Dealing of blocks to the XCDs. Dealt block g runs on XCD g % 8. With
  // pair_views = 0, g is the block's index over all views (view by view).
  // With pair_views = P > 1 (every view has the same size, e.g. the two
  // eyes), g = 8 s + x holds the block at screen position
  // x + 8 (s / P) of view s % P: the blocks at one position in all views
  // share an XCD and its L2, and follow one another.
  int32_t pair_views;
  int32_t view_blocks;   // blocks per view (pair_views > 0)
  int32_t dealt_blocks;  // dealt block indices (a multiple of 8)
  int32_t grid;          // workgroups launched
  int32_t tf_n;
  int32_t tile_log;     // log2 edge of a workgroup tile in 8x8 wave tiles
  int32_t wg_log;       // log2 waves per workgroup (min(2, 2 tile_log))
  int32_t wave_tiles;   // wave tiles per wave in a direct grid
  int32_t bt_log;       // log2 edge of a screen block in 8x8 wave tiles
  int32_t persistent;   // 1: waves take tiles from the per-XCD queues
  uint32_t* queue;      // 8 counters, zero at launch (persistent grid)
  uint32_t* stamp;      // cache volumes: [slots] frame of last use, else NULL
  uint32_t frame;
  int32_t B, S, Sx;     // brick core edge, stored edge, row stride (voxels)
  int32_t M;            // micro-blocks per slot edge, 0 for linear slots
  float Bf;             // B as a float (stencil index clamps)
  int32_t skip_empty;
  int32_t gather;       // 1: stencils read the pool directly (no LDS staging)
  int32_t stage_bytes;  // LDS staging bytes per wave
  double step;
  float ert;
  float t_ert;          // the largest float T with fl(1 - T) >= ert: T <= t_ert terminates
  float depth_alpha;
  int32_t model;        // kModel*
  int32_t n_planes;     // cut planes in use (0..4)
  int32_t roi_on;
  double planes[4][4];  // plane j keeps (n . p) + w <= 0: (nx, ny, nz, w)
  double roi[6];        // region of interest lo xyz, hi xyz
  const int32_t* enable;  // NULL, or a device flag: 0 = every workgroup returns at once
};

// The ray-casting launch (kernel, grid, LDS) for arguments `a`; a.grid is
// set to the grid chosen.
struct RaycastPlan {
  const void* func = nullptr;
  dim3 grid{1, 1, 1}, block{1, 1, 1};
  size_t lds = 0;
};
sg_status raycast_plan(Volume* v, RenderArgs& a, bool stats, RaycastPlan* out);
sg_status raycast_launch(Volume* v, RenderArgs& a, bool stats, Launch* out);
// Kernel instances per optical model (one translation unit each); mb:
// micro-block pool slots.
const void* raycast_kernel_absorption(int bpv, int channels, bool stats, bool gather,
                                      bool loop, bool mb);
const void* raycast_kernel_emission(int bpv, int channels, bool stats, bool gather, bool loop,
                                    bool mb);
const void* raycast_kernel_mip(int bpv, int channels, bool stats, bool gather, bool loop,
                               bool mb);

}  // namespace sg

struct sg_volume {
  sg::Volume v;
};
