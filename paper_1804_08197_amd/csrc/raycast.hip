// raycast.hip -- host side of the ray caster: argument checks, per-view
// constants, the LOD cut-map launch, the launch configuration (direct or
// persistent grid, tile and block shapes, LDS staging size), the autotuner
// and the graph objects that replay a render without host work.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "sg_internal.h"

namespace sg {

namespace {

bool finite(double x) { return std::isfinite(x); }

// Do all views have one size (so one block grid)?
bool same_size(int n_views, const sg_view* views) {
  for (int i = 1; i < n_views; ++i)
    if (views[i].width != views[0].width || views[i].height != views[0].height) return false;
  return true;
}

// Zero the 8 per-XCD tile queues of the persistent grid (a kernel, not a
// memset, so that graphs replay it reliably).
__global__ void reset_queue_kernel(uint32_t* q) {
  if (threadIdx.x < 8) q[threadIdx.x] = 0u;
}

sg_status check_params(const Volume* v, const sg_render_params* p) {
  if (!(finite(p->step_voxels) && p->step_voxels >= 1.0 / 64 && p->step_voxels <= 64.0) ||
      !finite(p->ert_alpha) ||
      !(finite(p->lod_tau_px) && p->lod_tau_px > 0.0) || !finite(p->depth_alpha) ||
      p->lod_bias < 0 || p->lod_bias >= v->L || p->timepoint < 0 ||
      p->timepoint >= v->d.timepoints ||
      (p->flags & ~(uint32_t)(SG_LOD | SG_SKIP_EMPTY | SG_GATHER)) || p->model < 0 ||
      p->model > SG_MODEL_MAX_INTENSITY || p->n_planes < 0 || p->n_planes > 4 ||
      (p->roi_on != 0 && p->roi_on != 1))
    return fail(SG_ERR_INVALID_ARG, "render params out of range");
  for (int j = 0; j < p->n_planes; ++j) {
    const double* q = p->planes[j];
    if (!(finite(q[0]) && finite(q[1]) && finite(q[2]) && finite(q[3])) ||
        (q[0] == 0.0 && q[1] == 0.0 && q[2] == 0.0))
      return fail(SG_ERR_INVALID_ARG, "cut planes must be finite with a nonzero normal");
  }
  if (p->roi_on)
    for (int i = 0; i < 3; ++i)
      if (!(finite(p->roi[i]) && finite(p->roi[i + 3]) && p->roi[i] <= p->roi[i + 3]))
        return fail(SG_ERR_INVALID_ARG, "region of interest must be finite with lo <= hi");
  for (int i = 0; i < 4; ++i)
    if (!finite(p->background[i])) return fail(SG_ERR_INVALID_ARG, "background not finite");
  return SG_OK;
}

// The launch configuration a render uses: the volume's, with the SG_GATHER
// flag and the SG_STAGE_BYTES environment variable as overrides.
LaunchConfig effective_config(const Volume* v, const sg_render_params* p) {
  LaunchConfig c = v->cfg;
  if (p->flags & SG_GATHER) c.gather = 1;
  if (const char* e = std::getenv("SG_STAGE_BYTES")) {
    const int x = std::atoi(e);
    if (x >= 1024 && x <= 32768) c.stage_bytes = x & ~15;
  }
  return c;
}

// log2 waves per workgroup: one wave per wave tile, at most four
int wg_log_of(const LaunchConfig& c) { return std::min(2, 2 * c.tile_log); }

size_t lds_bytes(const Volume* v, const LaunchConfig& c) {
  size_t tf = (size_t)v->d.channels * v->tf_n * 32;  // value and difference per entry
  return c.gather ? tf : tf + ((size_t)1 << wg_log_of(c)) * (size_t)c.stage_bytes;
}

sg_status check_config(const Volume* v, const LaunchConfig& c) {
  if (!(c.gather == 0 || c.gather == 1) || !(c.persistent == 0 || c.persistent == 1) ||
      c.tile_log < 0 || c.tile_log > 2 || c.bt_log < 2 || c.bt_log > 4 ||
      c.bt_log < c.tile_log || c.stage_bytes < 1024 || c.stage_bytes > 32768 ||
      c.stage_bytes % 16 != 0)
    return fail(SG_ERR_INVALID_ARG, "launch configuration out of range");
  if (v && lds_bytes(v, c) > 160 * 1024)
    return fail(SG_ERR_UNSUPPORTED, "launch configuration exceeds the LDS budget");
  return SG_OK;
}

int log2i(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

// The early-termination test on the transmittance: the largest float t with
// fl(1 - t) >= ert. fl(1 - t) never rises as t rises, so for every float T
// the test T <= t decides exactly as 1 - T >= ert does, one subtraction
// fewer per sample. NaN stays NaN (no ray terminates, as before).
float ert_transmittance(float ert) {
  if (std::isnan(ert)) return ert;
  const float one = 1.0f;
  float t = (float)(1.0 - (double)ert);
  for (int i = 0; i < 64 && !(one - t >= ert); ++i) t = std::nextafter(t, -INFINITY);
  for (int i = 0; i < 64; ++i) {
    const float u = std::nextafter(t, INFINITY);
    if (!(one - u >= ert)) break;
    t = u;
  }
  return t;
}


// Arguments shared by the stream path and the graph path.
void fill_args(const Volume* v, const sg_render_params* params, int n_views,
               const ViewDev* dviews, const int32_t* cutmap, int64_t blocks,
               const LaunchConfig& cfg, bool same_size, RenderArgs* out) {
  RenderArgs& a = *out;
  std::memset(&a, 0, sizeof(a));
  const int C = v->d.channels;
  a.pool = v->pool;
  a.slot_bytes = v->slot_bytes;
  a.M = v->M;
  a.Bf = (float)v->B;
  a.page = v->page + (int64_t)params->timepoint * C * v->nodes;
  a.empty = v->empty + (int64_t)params->timepoint * v->nodes;
  a.range = v->range + (int64_t)params->timepoint * C * v->nodes * 2;
  a.info = v->info;
  a.tf = v->tf;
  a.cutmap = cutmap;
  a.views = dviews;
  a.nodes = v->nodes;
  for (int L = 0; L < v->L; ++L)
    for (int i = 0; i < 3; ++i) a.ldims[L][i] = v->ldims[L][i];
  for (int c = 0; c < C; ++c) {
    const double sc = (double)(v->tf_n - 1) / (v->tf_hi[c] - v->tf_lo[c]);
    a.tf_scale[c] = (float)sc;
    a.tf_bias[c] = (float)(-v->tf_lo[c] * sc);
  }
  for (int i = 0; i < 4; ++i) a.bg[i] = (float)params->background[i];
  int key_levels = 0;
  for (int i = 0; i < 3; ++i) {
    a.dims[i] = v->d.dims[i];
    a.grid0[i] = v->grid[0][i];
    while (((int64_t)v->B << key_levels) < v->d.dims[i]) ++key_levels;
  }
  a.key_levels = key_levels;
  a.n_views = n_views;
  a.total_blocks = (int32_t)blocks;
  if (same_size && n_views > 1) {
    // the views' blocks at one screen position go to one XCD in turn
    a.pair_views = n_views;
    a.view_blocks = (int32_t)(blocks / n_views);
    a.dealt_blocks = 8 * n_views * ((a.view_blocks + 7) / 8);
  } else {
    a.pair_views = 0;
    a.view_blocks = 0;
    a.dealt_blocks = (int32_t)(((blocks + 7) / 8) * 8);
  }
  a.tf_n = v->tf_n;
  a.tile_log = cfg.tile_log;
  a.wg_log = wg_log_of(cfg);
  a.wave_tiles = 1 << (2 * cfg.tile_log - a.wg_log);
  a.bt_log = cfg.bt_log;
  a.persistent = cfg.persistent;
  a.queue = v->queue;
  a.stamp = v->cache ? v->stamp : nullptr;
  a.frame = v->frame;
  a.B = v->B;
  a.S = v->S;
  a.Sx = v->Sx;
  a.skip_empty = (params->flags & SG_SKIP_EMPTY) ? 1 : 0;
  a.gather = cfg.gather;
  a.stage_bytes = cfg.stage_bytes;
  a.step = params->step_voxels;
  a.ert = (float)params->ert_alpha;
  a.t_ert = ert_transmittance(a.ert);
  a.depth_alpha = (float)params->depth_alpha;
  a.model = params->model;
  a.n_planes = params->n_planes;
  a.roi_on = params->roi_on;
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i) a.planes[j][i] = j < params->n_planes ? params->planes[j][i] : 0.0;
  for (int i = 0; i < 6; ++i) a.roi[i] = params->roi_on ? params->roi[i] : 0.0;
}

sg_status ensure_queue(Volume* v) {
  if (!v->queue && hipMalloc((void**)&v->queue, 8 * sizeof(uint32_t)) != hipSuccess)
    return fail(SG_ERR_OUT_OF_MEMORY, "tile queue allocation failed");
  return SG_OK;
}

Launch queue_reset_launch(uint32_t* q) {
  Launch l;
  l.func = reinterpret_cast<const void*>(reset_queue_kernel);
  l.block = dim3(64);
  l.push(q);
  return l;
}

}  // namespace

sg_status raycast_plan(Volume* v, RenderArgs& a, bool stats, RaycastPlan* out) {
  const bool gather = a.gather != 0;
  const bool loop = a.persistent || a.wave_tiles > 1;
  const int C = v->d.channels;
  const bool mb = v->M != 0;
  const void* f =
      a.model == kModelEmission ? raycast_kernel_emission(v->bpv, C, stats, gather, loop, mb)
      : a.model == kModelMip    ? raycast_kernel_mip(v->bpv, C, stats, gather, loop, mb)
                                : raycast_kernel_absorption(v->bpv, C, stats, gather, loop, mb);
  LaunchConfig c;
  c.gather = a.gather;
  c.tile_log = a.tile_log;
  c.stage_bytes = a.stage_bytes;
  const size_t lds = lds_bytes(v, c);
  if (lds > 65536)
    SG_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const int threads = 64 << a.wg_log;
  int grid;
  if (a.persistent) {
    // as many workgroups as fit on the device at once, a multiple of the
    // 8 XCDs so that every XCD's queue is served
    int dev = 0, cus = 0, per_cu = 0;
    SG_HIP(hipGetDevice(&dev));
    SG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    SG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, threads, lds));
    grid = std::max(8, ((cus * std::max(per_cu, 1)) / 8) * 8);
  } else {
    const int64_t g = (int64_t)a.dealt_blocks << (2 * (a.bt_log - a.tile_log));
    if (g > 0x7fffffff) return fail(SG_ERR_INVALID_ARG, "too many pixels in one call");
    grid = (int)g;
  }
  a.grid = grid;
  out->func = f;
  out->grid = dim3((unsigned)grid);
  out->block = dim3((unsigned)threads);
  out->lds = lds;
  return SG_OK;
}

sg_status raycast_launch(Volume* v, RenderArgs& a, bool stats, Launch* out) {
  RaycastPlan pl;
  sg_status st = raycast_plan(v, a, stats, &pl);
  if (st != SG_OK) return st;
  out->func = pl.func;
  out->grid = pl.grid;
  out->block = pl.block;
  out->lds = pl.lds;
  out->arg.clear();
  out->push(a);
  return SG_OK;
}

sg_status view_geometry(const sg_view& w, ViewDev* out) {
  for (int k = 0; k < 16; ++k)
    if (!finite(w.cam_to_world[k])) return fail(SG_ERR_INVALID_ARG, "camera matrix not finite");
  if (!(finite(w.tan_left) && finite(w.tan_right) && finite(w.tan_bottom) &&
        finite(w.tan_top) && w.tan_left < w.tan_right && w.tan_bottom < w.tan_top))
    return fail(SG_ERR_INVALID_ARG, "view tangents must be finite with left<right, bottom<top");
  if (w.width < 1 || w.height < 1 || w.width > 32768 || w.height > 32768)
    return fail(SG_ERR_INVALID_ARG, "view size must be in [1, 32768]");
  for (int k = 0; k < 4; ++k)
    if (!finite(w.lens[k])) return fail(SG_ERR_INVALID_ARG, "lens coefficients not finite");
  if (w.ray_limit && reinterpret_cast<uintptr_t>(w.ray_limit) % 4 != 0)
    return fail(SG_ERR_INVALID_ARG, "ray_limit must be 4-byte aligned");
  const double* m = w.cam_to_world;
  double det = m[0] * (m[5] * m[10] - m[6] * m[9]) - m[1] * (m[4] * m[10] - m[6] * m[8]) +
               m[2] * (m[4] * m[9] - m[5] * m[8]);
  if (!(std::fabs(det) > 1e-12)) return fail(SG_ERR_INVALID_ARG, "singular camera rotation");
  ViewDev& o = *out;
  std::memset(&o, 0, sizeof(o));
  o.e[0] = m[3];
  o.e[1] = m[7];
  o.e[2] = m[11];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) o.R[3 * r + c] = m[4 * r + c];
  o.tl = w.tan_left;
  o.tr = w.tan_right;
  o.tb = w.tan_bottom;
  o.tt = w.tan_top;
  o.W = w.width;
  o.H = w.height;
  o.lens_on = (w.lens[0] != 0.0 || w.lens[1] != 0.0) ? 1 : 0;
  for (int k = 0; k < 4; ++k) o.lens[k] = w.lens[k];
  return SG_OK;
}

sg_status build_views(const Volume* v, int n_views, const sg_view* views,
                      const sg_render_params* p, float* const* rgba, float* const* depth,
                      int32_t* const* nsamp, int bt_log, std::vector<ViewDev>* out,
                      int64_t* total_blocks) {
  if (n_views < 1 || n_views > 4096 || !views || !p)
    return fail(SG_ERR_INVALID_ARG, "views: n_views must be in [1, 4096]");
  out->assign(n_views, ViewDev{});
  return build_views_into(v, n_views, views, p, rgba, depth, nsamp, bt_log, out->data(),
                          total_blocks);
}

sg_status build_views_into(const Volume* v, int n_views, const sg_view* views,
                           const sg_render_params* p, float* const* rgba, float* const* depth,
                           int32_t* const* nsamp, int bt_log, ViewDev* hv,
                           int64_t* total_blocks) {
  if (n_views < 1 || n_views > 4096 || !views || !p)
    return fail(SG_ERR_INVALID_ARG, "views: n_views must be in [1, 4096]");
  sg_status st = check_params(v, p);
  if (st != SG_OK) return st;
  for (int i = 0; i < n_views; ++i) hv[i] = ViewDev{};
  int64_t blocks = 0;
  const int64_t cells = (int64_t)v->grid[0][0] * v->grid[0][1] * v->grid[0][2];
  const int bpx = 8 << bt_log;  // block edge in pixels
  for (int i = 0; i < n_views; ++i) {
    const sg_view& w = views[i];
    if ((st = view_geometry(w, &hv[i])) != SG_OK) return st;
    if (rgba && !rgba[i]) return fail(SG_ERR_INVALID_ARG, "out_rgba entry is NULL");
    if ((rgba && reinterpret_cast<uintptr_t>(rgba[i]) % 16 != 0) ||
        (depth && depth[i] && reinterpret_cast<uintptr_t>(depth[i]) % 4 != 0))
      return fail(SG_ERR_INVALID_ARG, "output buffers must be 16-byte (rgba) / 4-byte aligned");
    ViewDev& o = hv[i];
    const double theta = (w.tan_top - w.tan_bottom) / (double)w.height;
    o.K = (p->lod_tau_px * theta) * (p->lod_tau_px * theta);
    o.W = w.width;
    o.H = w.height;
    o.tiles_x = (w.width + 7) / 8;
    o.tiles_y = (w.height + 7) / 8;
    o.blocks_x = (w.width + bpx - 1) / bpx;
    o.block_begin = (int32_t)blocks;
    blocks += (int64_t)o.blocks_x * ((w.height + bpx - 1) / bpx);
    o.cut_off = (int64_t)i * cells;
    o.rgba = rgba ? rgba[i] : nullptr;
    o.depth = depth ? depth[i] : nullptr;
    o.nsamp = nsamp ? nsamp[i] : nullptr;
    o.limit = w.ray_limit;
    o.tile_any = w.tile_any;
    if (blocks > (1 << 24)) return fail(SG_ERR_INVALID_ARG, "too many pixels in one call");
  }
  *total_blocks = blocks;
  return SG_OK;
}

sg_status prepare_views(Volume* v, int n_views, const sg_view* views,
                        const sg_render_params* p, float* const* rgba,
                        float* const* depth, int32_t* const* nsamp, hipStream_t s,
                        int* total_blocks) {
  std::vector<ViewDev> hv;
  int64_t blocks = 0;
  sg_status st = build_views(v, n_views, views, p, rgba, depth, nsamp,
                             effective_config(v, p).bt_log, &hv, &blocks);
  if (st != SG_OK) return st;
  const int64_t cells = (int64_t)v->grid[0][0] * v->grid[0][1] * v->grid[0][2];
  const int64_t need_cut = (int64_t)n_views * cells;
  if (need_cut > v->cutmap_cap) {
    SG_HIP(hipStreamSynchronize(s));
    if (v->cutmap) SG_HIP(hipFree(v->cutmap));
    v->cutmap = nullptr;
    v->cutmap_cap = 0;
    if (hipMalloc((void**)&v->cutmap, (size_t)need_cut * sizeof(int32_t)) != hipSuccess)
      return fail(SG_ERR_OUT_OF_MEMORY, "cut map allocation failed");
    v->cutmap_cap = need_cut;
  }
  const int64_t vbytes = (int64_t)n_views * sizeof(ViewDev);
  if (vbytes > v->view_cap) {
    SG_HIP(hipStreamSynchronize(s));
    if (v->view_dev) SG_HIP(hipFree(v->view_dev));
    v->view_dev = nullptr;
    v->view_cap = 0;
    if (hipMalloc((void**)&v->view_dev, (size_t)vbytes) != hipSuccess)
      return fail(SG_ERR_OUT_OF_MEMORY, "view table allocation failed");
    v->view_cap = vbytes;
  }
  if (n_views <= kInlineViews) {
    // carried by the cut-map kernel's arguments (see InlineViews)
    v->inline_views.n = n_views;
    for (int i = 0; i < n_views; ++i) v->inline_views.v[i] = hv[(size_t)i];
  } else {
    v->inline_views.n = 0;
    st = stage_to_device(v, hv.data(), vbytes, v->view_dev, s);
    if (st != SG_OK) return st;
  }
  *total_blocks = (int)blocks;
  return SG_OK;
}

namespace {

sg_status check_volume_ready(Volume* v) {
  for (int c = 0; c < v->d.channels; ++c)
    if (!v->tf_set[c]) return fail(SG_ERR_STATE, "a channel has no transfer function");
  return SG_OK;
}

sg_status render(sg_volume* vol, int32_t n_views, const sg_view* views,
                 const sg_render_params* params, float* const* out_rgba,
                 float* const* out_depth, sg_render_stats* stats, void* hip_stream,
                 const int32_t* enable = nullptr) {
  if (!vol) return fail(SG_ERR_INVALID_ARG, "volume is NULL");
  Volume* v = &vol->v;
  if (!params || !out_rgba) return fail(SG_ERR_INVALID_ARG, "params / out_rgba is NULL");
  if (!views) return fail(SG_ERR_INVALID_ARG, "views is NULL");
  sg_status st = check_volume_ready(v);
  if (st != SG_OK) return st;
  const LaunchConfig cfg = effective_config(v, params);
  if ((st = check_config(v, cfg)) != SG_OK) return st;
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  hipStream_t s = (hipStream_t)hip_stream;
  if ((st = commit(v, s)) != SG_OK) return st;
  int blocks = 0;
  st = prepare_views(v, n_views, views, params, out_rgba, out_depth,
                     stats ? stats->samples : nullptr, s, &blocks);
  if (st != SG_OK) return st;
  if (cfg.persistent && (st = ensure_queue(v)) != SG_OK) return st;
  const ViewDev* dv = reinterpret_cast<const ViewDev*>(v->view_dev);
  const bool timed = v->timing && !stats;
  if (!top_level_resident(v, params->timepoint))
    return fail(SG_ERR_STATE, "a top-level node is not in the cache at this timepoint");
  ++v->frame;
  if (timed && (st = timing_mark(v, s)) != SG_OK) return st;
  st = launch_cutmap(v, dv, n_views, params->lod_bias, (params->flags & SG_LOD) != 0,
                     params->timepoint, s, enable);
  if (st != SG_OK) return st;
  if (cfg.persistent) {
    Launch q = queue_reset_launch(v->queue);
    if ((st = q.run(s)) != SG_OK) return st;
  }
  if (timed && (st = timing_mark(v, s)) != SG_OK) return st;

  RenderArgs a;
  fill_args(v, params, n_views, dv, v->cutmap, blocks, cfg, same_size(n_views, views), &a);
  a.enable = enable;
  const int C = v->d.channels;
  if (stats) {
    // micro-block bitmap: one bit per 4^3 block per (channel, level)
    int64_t bits = 0;
    int64_t offs[kMaxChannels * kMaxLevels] = {0};
    for (int c = 0; c < C; ++c)
      for (int L = 0; L < v->L; ++L) {
        offs[c * kMaxLevels + L] = bits;
        bits += (int64_t)((v->ldims[L][0] + 3) / 4) * ((v->ldims[L][1] + 3) / 4) *
                ((v->ldims[L][2] + 3) / 4);
      }
    const int64_t words = (bits + 31) / 32 + 1;
    if (words > v->mb_words) {
      SG_HIP(hipStreamSynchronize(s));
      if (v->mb_bits) SG_HIP(hipFree(v->mb_bits));
      v->mb_bits = nullptr;
      v->mb_words = 0;
      if (hipMalloc((void**)&v->mb_bits, (size_t)words * 4) != hipSuccess)
        return fail(SG_ERR_OUT_OF_MEMORY, "micro-block bitmap allocation failed");
      v->mb_words = words;
    }
    if (!v->counters && hipMalloc((void**)&v->counters, 128) != hipSuccess)
      return fail(SG_ERR_OUT_OF_MEMORY, "counter allocation failed");
    SG_HIP(hipMemsetAsync(v->mb_bits, 0, (size_t)words * 4, s));
    SG_HIP(hipMemsetAsync(v->counters, 0, 128, s));
    a.mb_bits = v->mb_bits;
    a.counters = v->counters;
    for (int i = 0; i < kMaxChannels * kMaxLevels; ++i) a.level_mb_off[i] = offs[i];
    Launch l;
    if ((st = raycast_launch(v, a, true, &l)) != SG_OK) return st;
    if ((st = l.run(s)) != SG_OK) return st;
    std::vector<uint32_t> hb((size_t)words);
    uint64_t cnt[16];
    SG_HIP(hipMemcpyAsync(hb.data(), v->mb_bits, (size_t)words * 4, hipMemcpyDeviceToHost, s));
    SG_HIP(hipMemcpyAsync(cnt, v->counters, 128, hipMemcpyDeviceToHost, s));
    SG_HIP(hipStreamSynchronize(s));
    uint64_t pop = 0;
    for (uint32_t x : hb) pop += (uint64_t)__builtin_popcount(x);
    stats->total_samples = cnt[0];
    stats->microblocks = pop;
    stats->node_visits = cnt[1];
    stats->slabs = cnt[2];
    stats->staged_bytes = cnt[3];
    stats->node_lanes = cnt[4];
    stats->loop_iterations = cnt[5];
    stats->pool_samples = cnt[6];
    stats->slab_retries = cnt[7];
    stats->alive_lanes = cnt[8];
    stats->wide_slabs = cnt[9];
    return SG_OK;
  }
  Launch l;
  if ((st = raycast_launch(v, a, false, &l)) != SG_OK) return st;
  if ((st = l.run(s)) != SG_OK) return st;
  if (timed) return timing_mark(v, s);
  return SG_OK;
}

// sg_launch_config <-> internal units
sg_status to_internal(const sg_launch_config* c, LaunchConfig* out) {
  if (!(c->tile == 8 || c->tile == 16 || c->tile == 32) ||
      !(c->block == 32 || c->block == 64 || c->block == 128) || c->block < c->tile)
    return fail(SG_ERR_INVALID_ARG, "launch configuration: tile 8/16/32, block 32/64/128 >= tile");
  LaunchConfig r;
  r.gather = c->kernel;
  r.tile_log = log2i(c->tile / 8);
  r.bt_log = log2i(c->block / 8);
  r.stage_bytes = c->stage_bytes;
  r.persistent = c->persistent;
  *out = r;
  return SG_OK;
}

void to_public(const LaunchConfig& c, sg_launch_config* out) {
  out->kernel = c.gather;
  out->tile = 8 << c.tile_log;
  out->block = 8 << c.bt_log;
  out->stage_bytes = c.stage_bytes;
  out->persistent = c.persistent;
}

}  // namespace

}  // namespace sg

using namespace sg;

extern "C" sg_status sg_render_views(sg_volume* vol, int32_t n_views, const sg_view* views,
                                     const sg_render_params* params, float* const* out_rgba,
                                     float* const* out_depth, void* hip_stream) {
  return render(vol, n_views, views, params, out_rgba, out_depth, nullptr, hip_stream);
}

extern "C" sg_status sg_render_views_if(sg_volume* vol, int32_t n_views, const sg_view* views,
                                        const sg_render_params* params, float* const* out_rgba,
                                        float* const* out_depth, const int32_t* enable,
                                        void* hip_stream) {
  if (!enable) return fail(SG_ERR_INVALID_ARG, "sg_render_views_if: NULL enable flag");
  return render(vol, n_views, views, params, out_rgba, out_depth, nullptr, hip_stream, enable);
}

extern "C" sg_status sg_render_views_stats(sg_volume* vol, int32_t n_views,
                                           const sg_view* views,
                                           const sg_render_params* params,
                                           float* const* out_rgba, float* const* out_depth,
                                           sg_render_stats* stats, void* hip_stream) {
  if (!stats) return fail(SG_ERR_INVALID_ARG, "stats is NULL");
  return render(vol, n_views, views, params, out_rgba, out_depth, stats, hip_stream);
}

extern "C" sg_status sg_set_launch_config(sg_volume* vol, const sg_launch_config* config) {
  if (!vol) return fail(SG_ERR_INVALID_ARG, "sg_set_launch_config: NULL volume");
  Volume* v = &vol->v;
  if (!config) {
    v->cfg = LaunchConfig{};
    return SG_OK;
  }
  LaunchConfig c;
  sg_status st = to_internal(config, &c);
  if (st != SG_OK) return st;
  if ((st = check_config(v->tf_n > 0 ? v : nullptr, c)) != SG_OK) return st;
  v->cfg = c;
  return SG_OK;
}

extern "C" sg_status sg_get_launch_config(const sg_volume* vol, sg_launch_config* config) {
  if (!vol || !config) return fail(SG_ERR_INVALID_ARG, "sg_get_launch_config: NULL argument");
  to_public(vol->v.cfg, config);
  return SG_OK;
}

// Autotuner: coordinate descent over the launch configuration. Every
// candidate renders the same image (only the work decomposition and the
// staging differ), so the choice is by time alone: each candidate is timed
// over `repeats` renders after one warm-up render, with events on the
// caller's stream; a dimension's best value is kept before the next
// dimension is tried, and the sweep runs twice.
extern "C" sg_status sg_autotune(sg_volume* vol, int32_t n_views, const sg_view* views,
                                 const sg_render_params* params, float* const* out_rgba,
                                 int32_t repeats, sg_launch_config* best, double* best_ms,
                                 void* hip_stream) {
  if (!vol || !views || !params || !out_rgba)
    return fail(SG_ERR_INVALID_ARG, "sg_autotune: NULL argument");
  if (repeats < 1 || repeats > 1000)
    return fail(SG_ERR_INVALID_ARG, "sg_autotune: repeats must be in [1, 1000]");
  if (params->flags & SG_GATHER)
    return fail(SG_ERR_INVALID_ARG, "sg_autotune: the kernel flavour is tuned; clear SG_GATHER");
  Volume* v = &vol->v;
  sg_status st = check_volume_ready(v);
  if (st != SG_OK) return st;
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  hipStream_t s = (hipStream_t)hip_stream;
  hipEvent_t e0, e1;
  SG_HIP(hipEventCreate(&e0));
  SG_HIP(hipEventCreate(&e1));
  const LaunchConfig saved = v->cfg;
  auto time_cfg = [&](const LaunchConfig& c, double* ms) -> sg_status {
    v->cfg = c;
    sg_status r = render(vol, n_views, views, params, out_rgba, nullptr, nullptr, s);
    if (r != SG_OK) return r;
    SG_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < repeats; ++i)
      if ((r = render(vol, n_views, views, params, out_rgba, nullptr, nullptr, s)) != SG_OK)
        return r;
    SG_HIP(hipEventRecord(e1, s));
    SG_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    SG_HIP(hipEventElapsedTime(&t, e0, e1));
    *ms = (double)t / repeats;
    return SG_OK;
  };
  LaunchConfig cur = LaunchConfig{};
  double cur_ms = 0.0;
  st = time_cfg(cur, &cur_ms);
  const int vals[5][3] = {{0, 1, -1}, {0, 1, 2}, {2, 3, 4}, {4096, 8192, 16384}, {0, 1, -1}};
  for (int sweep = 0; sweep < 2 && st == SG_OK; ++sweep) {
    for (int dim = 0; dim < 5 && st == SG_OK; ++dim) {
      std::vector<LaunchConfig> cand;
      for (int k = 0; k < 3; ++k) {
        if (vals[dim][k] < 0) continue;
        LaunchConfig c = cur;
        if (dim == 0) c.gather = vals[dim][k];
        if (dim == 1) c.tile_log = vals[dim][k];
        if (dim == 2) c.bt_log = vals[dim][k];
        if (dim == 3) c.stage_bytes = vals[dim][k];
        if (dim == 4) c.persistent = vals[dim][k];
        if (dim == 3 && c.gather) continue;  // the staging size is moot for gather
        if (c.bt_log < c.tile_log || lds_bytes(v, c) > 160 * 1024) continue;
        if (std::memcmp(&c, &cur, sizeof(c)) == 0) continue;
        cand.push_back(c);
      }
      for (const LaunchConfig& c : cand) {
        double ms = 0.0;
        if ((st = time_cfg(c, &ms)) != SG_OK) break;
        if (ms < cur_ms) {
          cur = c;
          cur_ms = ms;
        }
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != SG_OK) {
    v->cfg = saved;
    return st;
  }
  v->cfg = cur;
  if (best) to_public(cur, best);
  if (best_ms) *best_ms = cur_ms;
  return SG_OK;
}

// ---------------------------------------------------------------- graphs
struct sg_render_graph {
  Volume* v = nullptr;
  int n_views = 0;
  std::vector<int32_t> sizes;  // width, height per view
  sg_render_params params{};
  LaunchConfig cfg;
  std::vector<float*> rgba, depth;
  ViewDev* dviews = nullptr;
  int32_t* cutmap = nullptr;
  uint32_t* queue = nullptr;
  int tf_n = 0;
  double tf_lo[kMaxChannels]{}, tf_hi[kMaxChannels]{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void graph_free(sg_render_graph* g) {
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  if (g->dviews) hipFree(g->dviews);
  if (g->cutmap) hipFree(g->cutmap);
  if (g->queue) hipFree(g->queue);
  delete g;
}

sg_status add_node(hipGraph_t graph, Launch& l, hipGraphNode_t* dep, hipGraphNode_t* out) {
  std::vector<void*> p = l.ptrs();
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(l.func);
  kp.gridDim = l.grid;
  kp.blockDim = l.block;
  kp.sharedMemBytes = (unsigned)l.lds;
  kp.kernelParams = p.data();
  kp.extra = nullptr;
  SG_HIP(hipGraphAddKernelNode(out, graph, dep, dep ? 1 : 0, &kp));
  return SG_OK;
}

}  // namespace

extern "C" sg_status sg_render_graph_create(sg_volume* vol, int32_t n_views,
                                            const sg_view* views,
                                            const sg_render_params* params,
                                            float* const* out_rgba, float* const* out_depth,
                                            sg_render_graph** out) {
  if (!vol || !views || !params || !out_rgba || !out)
    return fail(SG_ERR_INVALID_ARG, "sg_render_graph_create: NULL argument");
  Volume* v = &vol->v;
  if (v->cache)
    return fail(SG_ERR_UNSUPPORTED, "sg_render_graph_create: not available for cache volumes");
  sg_status st = check_volume_ready(v);
  if (st != SG_OK) return st;
  const LaunchConfig cfg = effective_config(v, params);
  if ((st = check_config(v, cfg)) != SG_OK) return st;
  std::vector<ViewDev> hv;
  int64_t blocks = 0;
  st = build_views(v, n_views, views, params, out_rgba, out_depth, nullptr, cfg.bt_log, &hv,
                   &blocks);
  if (st != SG_OK) return st;
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  sg_render_graph* g = new sg_render_graph;
  g->v = v;
  g->n_views = n_views;
  g->params = *params;
  g->cfg = cfg;
  for (int i = 0; i < n_views; ++i) {
    g->sizes.push_back(views[i].width);
    g->sizes.push_back(views[i].height);
    g->rgba.push_back(out_rgba[i]);
    g->depth.push_back(out_depth ? out_depth[i] : nullptr);
  }
  g->tf_n = v->tf_n;
  for (int c = 0; c < v->d.channels; ++c) {
    g->tf_lo[c] = v->tf_lo[c];
    g->tf_hi[c] = v->tf_hi[c];
  }
  const int64_t cells = (int64_t)v->grid[0][0] * v->grid[0][1] * v->grid[0][2];
  auto bail = [&](sg_status s2) {
    graph_free(g);
    return s2;
  };
  if (hipMalloc((void**)&g->dviews, sizeof(ViewDev) * n_views) != hipSuccess ||
      hipMalloc((void**)&g->cutmap, sizeof(int32_t) * cells * n_views) != hipSuccess ||
      hipMalloc((void**)&g->queue, 8 * sizeof(uint32_t)) != hipSuccess)
    return bail(fail(SG_ERR_OUT_OF_MEMORY, "sg_render_graph_create: allocation failed"));
  if (hipMemcpy(g->dviews, hv.data(), sizeof(ViewDev) * n_views, hipMemcpyHostToDevice) !=
      hipSuccess)
    return bail(fail(SG_ERR_DEVICE, "sg_render_graph_create: view upload failed"));
  Launch cut, ray, reset = queue_reset_launch(g->queue);
  if ((st = cutmap_launch(v, g->dviews, n_views, params->lod_bias,
                          (params->flags & SG_LOD) != 0, params->timepoint, g->cutmap,
                          &cut)) != SG_OK)
    return bail(st);
  RenderArgs a;
  fill_args(v, params, n_views, g->dviews, g->cutmap, blocks, cfg, same_size(n_views, views),
            &a);
  a.queue = g->queue;
  if ((st = raycast_launch(v, a, false, &ray)) != SG_OK) return bail(st);
  if (hipGraphCreate(&g->graph, 0) != hipSuccess)
    return bail(fail(SG_ERR_DEVICE, "sg_render_graph_create: hipGraphCreate failed"));
  hipGraphNode_t n0 = nullptr, n1 = nullptr, n2 = nullptr;
  if ((st = add_node(g->graph, cut, nullptr, &n0)) != SG_OK) return bail(st);
  hipGraphNode_t last = n0;
  if (cfg.persistent) {
    if ((st = add_node(g->graph, reset, &last, &n1)) != SG_OK) return bail(st);
    last = n1;
  }
  if ((st = add_node(g->graph, ray, &last, &n2)) != SG_OK) return bail(st);
  if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
    return bail(fail(SG_ERR_DEVICE, "sg_render_graph_create: hipGraphInstantiate failed"));
  *out = g;
  return SG_OK;
}

extern "C" sg_status sg_render_graph_set_views(sg_render_graph* g, const sg_view* views,
                                               void* hip_stream) {
  if (!g || !views) return fail(SG_ERR_INVALID_ARG, "sg_render_graph_set_views: NULL argument");
  for (int i = 0; i < g->n_views; ++i)
    if (views[i].width != g->sizes[2 * i] || views[i].height != g->sizes[2 * i + 1])
      return fail(SG_ERR_INVALID_ARG, "sg_render_graph_set_views: view sizes must not change");
  std::vector<ViewDev> hv;
  int64_t blocks = 0;
  sg_status st = build_views(g->v, g->n_views, views, &g->params, g->rgba.data(),
                             g->depth.data(), nullptr, g->cfg.bt_log, &hv, &blocks);
  if (st != SG_OK) return st;
  DeviceGuard guard(g->v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  return stage_to_device(g->v, hv.data(), (int64_t)sizeof(ViewDev) * g->n_views, g->dviews,
                         (hipStream_t)hip_stream);
}

extern "C" sg_status sg_render_graph_launch(sg_render_graph* g, void* hip_stream) {
  if (!g) return fail(SG_ERR_INVALID_ARG, "sg_render_graph_launch: NULL graph");
  Volume* v = g->v;
  bool same = v->tf_n == g->tf_n;
  for (int c = 0; c < v->d.channels; ++c)
    same = same && v->tf_lo[c] == g->tf_lo[c] && v->tf_hi[c] == g->tf_hi[c];
  if (!same)
    return fail(SG_ERR_STATE, "sg_render_graph_launch: the transfer-function size or domain "
                              "changed since the graph was made");
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  hipStream_t s = (hipStream_t)hip_stream;
  sg_status st = commit(v, s);
  if (st != SG_OK) return st;
  SG_HIP(hipGraphLaunch(g->exec, s));
  return SG_OK;
}

extern "C" sg_status sg_render_graph_destroy(sg_render_graph* g) {
  if (!g) return fail(SG_ERR_INVALID_ARG, "sg_render_graph_destroy: NULL graph");
  DeviceGuard guard(g->v->d.device);
  hipDeviceSynchronize();
  graph_free(g);
  return SG_OK;
}

// ---------------------------------------------------- allocation-free render
// sg_render_views_noalloc keeps its per-render scratch -- the view table,
// the persistent grid's eight tile queues and the cut maps -- in one
// file-scope device array, of which every GPU the library runs on holds its
// own copy until the process ends. Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol): the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current.
namespace sg {
namespace {
constexpr size_t kScratchBytes = (size_t)4 << 20;
constexpr size_t kScratchQueue = 4096;  // view table [0, 4096), queues from here
constexpr size_t kScratchCut = 8192;    // cut maps [8192, kScratchBytes)
static_assert(kInlineViews * sizeof(ViewDev) <= kScratchQueue, "view table exceeds its room");
constexpr int kMaxDevices = 64;
}  // namespace
}  // namespace sg

static __device__ __align__(256) uint8_t scratch[sg::kScratchBytes];

namespace sg {
namespace {

std::mutex g_scratch_mu;
uint8_t* g_scratch[kMaxDevices] = {};

// The device address of this device's scratch (dev must be current).
sg_status scratch_base(int dev, uint8_t** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(SG_ERR_UNSUPPORTED, "sg_render_views_noalloc: device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SG_ERR_DEVICE, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch[dev] = static_cast<uint8_t*>(p);
  }
  *out = g_scratch[dev];
  return SG_OK;
}

}  // namespace
}  // namespace sg

extern "C" sg_status sg_render_views_noalloc(sg_volume* vol, int32_t n_views,
                                             const sg_view* views,
                                             const sg_render_params* params,
                                             float* const* out_rgba, float* const* out_depth,
                                             void* hip_stream) {
  if (!vol) return fail(SG_ERR_INVALID_ARG, "sg_render_views_noalloc: NULL volume");
  Volume* v = &vol->v;
  if (!views || !params || !out_rgba)
    return fail(SG_ERR_INVALID_ARG, "sg_render_views_noalloc: NULL views, params or out_rgba");
  if (n_views < 1 || n_views > kInlineViews)
    return fail(SG_ERR_INVALID_ARG, "sg_render_views_noalloc: n_views must be in [1, 4]");
  sg_status st = check_volume_ready(v);
  if (st != SG_OK) return st;
  // committing (aprons, ranges, table upload) may allocate: it must be done
  bool pending = v->empty_dirty || v->tf_dirty;
  for (uint8_t p : v->pending) pending = pending || p != 0;
  if (pending)
    return fail(SG_ERR_STATE, "sg_render_views_noalloc: uploads or transfer-function changes "
                              "are not committed (call sg_volume_commit first)");
  const LaunchConfig cfg = effective_config(v, params);
  if ((st = check_config(v, cfg)) != SG_OK) return st;
  const int64_t cells = (int64_t)v->grid[0][0] * v->grid[0][1] * v->grid[0][2];
  const int64_t cut_bytes = (int64_t)n_views * cells * (int64_t)sizeof(int32_t);
  if (cut_bytes > (int64_t)(kScratchBytes - kScratchCut))
    return fail(SG_ERR_INVALID_ARG,
                "sg_render_views_noalloc: the cut maps (views x level-0 bricks x 4 bytes = " +
                    std::to_string(cut_bytes) + ") exceed the " +
                    std::to_string(kScratchBytes - kScratchCut) + "-byte scratch");
  ViewDev hv[kInlineViews];
  int64_t blocks = 0;
  if ((st = build_views_into(v, n_views, views, params, out_rgba, out_depth, nullptr,
                             cfg.bt_log, hv, &blocks)) != SG_OK)
    return st;
  if (!top_level_resident(v, params->timepoint))
    return fail(SG_ERR_STATE, "a top-level node is not in the cache at this timepoint");
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  uint8_t* base = nullptr;
  if ((st = scratch_base(v->d.device, &base)) != SG_OK) return st;
  ViewDev* dviews = reinterpret_cast<ViewDev*>(base);
  uint32_t* queue = reinterpret_cast<uint32_t*>(base + kScratchQueue);
  int32_t* cutmap = reinterpret_cast<int32_t*>(base + kScratchCut);
  hipStream_t s = (hipStream_t)hip_stream;
  // the view records ride in the cut-map kernel's arguments; its first
  // workgroup writes them to the scratch view table (every call rewrites
  // the table, the cut maps and, for the persistent grid, the queues)
  InlineViews iv{};
  iv.n = n_views;
  for (int i = 0; i < n_views; ++i) iv.v[i] = hv[i];
  ++v->frame;
  if ((st = cutmap_run(v, dviews, n_views, params->lod_bias, (params->flags & SG_LOD) != 0,
                       params->timepoint, cutmap, iv, s)) != SG_OK)
    return st;
  if (cfg.persistent) {
    void* qa[] = {&queue};
    SG_HIP(hipLaunchKernel(reinterpret_cast<const void*>(reset_queue_kernel), dim3(1), dim3(64),
                           qa, 0, s));
  }
  RenderArgs a;
  fill_args(v, params, n_views, dviews, cutmap, blocks, cfg, same_size(n_views, views), &a);
  a.queue = queue;
  RaycastPlan pl;
  if ((st = raycast_plan(v, a, false, &pl)) != SG_OK) return st;
  void* args[1] = {&a};
  SG_HIP(hipLaunchKernel(pl.func, pl.grid, pl.block, args, pl.lds, s));
  return SG_OK;
}
