// raycast.hip -- host side of the ray caster: argument checks, per-view
// constants, the LOD cut-map launch and the dispatch to the ray-casting
// kernels (raycast_kernels.h, one translation unit per optical model).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "sg_internal.h"

namespace sg {

namespace {

bool finite(double x) { return std::isfinite(x); }

}  // namespace

sg_status launch_raycast(Volume* v, const RenderArgs& a, bool stats, hipStream_t s) {
  switch (a.model) {
    case kModelEmission:
      return launch_raycast_emission(v->bpv, v->d.channels, a, stats, s);
    case kModelMip:
      return launch_raycast_mip(v->bpv, v->d.channels, a, stats, s);
    default:
      return launch_raycast_absorption(v->bpv, v->d.channels, a, stats, s);
  }
}

sg_status prepare_views(Volume* v, int n_views, const sg_view* views,
                        const sg_render_params* p, float* const* rgba,
                        float* const* depth, int32_t* const* nsamp, hipStream_t s,
                        int* total_blocks) {
  if (n_views < 1 || n_views > 4096 || !views || !p)
    return fail(SG_ERR_INVALID_ARG, "views: n_views must be in [1, 4096]");
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
  std::vector<ViewDev> hv(n_views);
  int64_t blocks = 0;
  const int64_t cells = (int64_t)v->grid[0][0] * v->grid[0][1] * v->grid[0][2];
  for (int i = 0; i < n_views; ++i) {
    const sg_view& w = views[i];
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
    if (rgba && !rgba[i]) return fail(SG_ERR_INVALID_ARG, "out_rgba entry is NULL");
    if ((rgba && reinterpret_cast<uintptr_t>(rgba[i]) % 16 != 0) ||
        (depth && depth[i] && reinterpret_cast<uintptr_t>(depth[i]) % 4 != 0))
      return fail(SG_ERR_INVALID_ARG, "output buffers must be 16-byte (rgba) / 4-byte aligned");
    ViewDev& o = hv[i];
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
    const double theta = (w.tan_top - w.tan_bottom) / (double)w.height;
    o.K = (p->lod_tau_px * theta) * (p->lod_tau_px * theta);
    o.W = w.width;
    o.H = w.height;
    o.tiles_x = (w.width + 15) / 16;
    o.tiles_y = (w.height + 15) / 16;
    o.blocks_x = (o.tiles_x + 3) / 4;
    o.block_begin = (int32_t)blocks;
    blocks += (int64_t)o.blocks_x * ((o.tiles_y + 3) / 4);
    o.cut_off = (int64_t)i * cells;
    o.rgba = rgba ? rgba[i] : nullptr;
    o.depth = depth ? depth[i] : nullptr;
    o.nsamp = nsamp ? nsamp[i] : nullptr;
    o.limit = w.ray_limit;
    o.lens_on = (w.lens[0] != 0.0 || w.lens[1] != 0.0) ? 1 : 0;
    for (int k = 0; k < 4; ++k) o.lens[k] = w.lens[k];
  }
  if (blocks > (1 << 24)) return fail(SG_ERR_INVALID_ARG, "too many pixels in one call");
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
  sg_status st = stage_to_device(v, hv.data(), vbytes, v->view_dev, s);
  if (st != SG_OK) return st;
  *total_blocks = (int)blocks;
  return SG_OK;
}

static sg_status render(sg_volume* vol, int32_t n_views, const sg_view* views,
                        const sg_render_params* params, float* const* out_rgba,
                        float* const* out_depth, sg_render_stats* stats, void* hip_stream) {
  if (!vol) return fail(SG_ERR_INVALID_ARG, "volume is NULL");
  Volume* v = &vol->v;
  if (!params || !out_rgba) return fail(SG_ERR_INVALID_ARG, "params / out_rgba is NULL");
  if (!views) return fail(SG_ERR_INVALID_ARG, "views is NULL");
  for (int c = 0; c < v->d.channels; ++c)
    if (!v->tf_set[c]) return fail(SG_ERR_STATE, "a channel has no transfer function");
  int stage_bytes = kStageBytesDefault;
  if (const char* e = std::getenv("SG_STAGE_BYTES")) {
    const int x = std::atoi(e);
    if (x >= 1024 && x <= 32768) stage_bytes = x & ~15;
  }
  const size_t lds = (size_t)v->d.channels * (v->tf_n + 1) * 16 + 4 * (size_t)stage_bytes;
  if (lds > 160 * 1024) return fail(SG_ERR_UNSUPPORTED, "transfer tables exceed the LDS budget");
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  hipStream_t s = (hipStream_t)hip_stream;
  sg_status st = commit(v, s);
  if (st != SG_OK) return st;
  int blocks = 0;
  st = prepare_views(v, n_views, views, params, out_rgba, out_depth,
                     stats ? stats->samples : nullptr, s, &blocks);
  if (st != SG_OK) return st;
  const ViewDev* dv = reinterpret_cast<const ViewDev*>(v->view_dev);
  const bool timed = v->timing && !stats;
  if (timed && (st = timing_mark(v, s)) != SG_OK) return st;
  st = launch_cutmap(v, dv, n_views, params->lod_bias, (params->flags & SG_LOD) != 0, s);
  if (st != SG_OK) return st;
  if (timed && (st = timing_mark(v, s)) != SG_OK) return st;

  RenderArgs a;
  std::memset(&a, 0, sizeof(a));
  const int C = v->d.channels;
  a.pool = v->pool;
  a.slot_bytes = v->slot_bytes;
  a.page = v->page + (int64_t)params->timepoint * C * v->nodes;
  a.empty = v->empty + (int64_t)params->timepoint * v->nodes;
  a.range = v->range + (int64_t)params->timepoint * C * v->nodes * 2;
  a.info = v->info;
  a.tf = v->tf;
  a.cutmap = v->cutmap;
  a.views = dv;
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
  a.total_blocks = blocks;
  a.grid = ((blocks + 7) / 8) * 8 * 16;
  a.tf_n = v->tf_n;
  a.B = v->B;
  a.S = v->S;
  a.Sx = v->Sx;
  a.skip_empty = (params->flags & SG_SKIP_EMPTY) ? 1 : 0;
  a.gather = (params->flags & SG_GATHER) ? 1 : 0;
  a.stage_bytes = stage_bytes;
  a.step = params->step_voxels;
  a.ert = (float)params->ert_alpha;
  a.depth_alpha = (float)params->depth_alpha;
  a.model = params->model;
  a.n_planes = params->n_planes;
  a.roi_on = params->roi_on;
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i) a.planes[j][i] = j < params->n_planes ? params->planes[j][i] : 0.0;
  for (int i = 0; i < 6; ++i) a.roi[i] = params->roi_on ? params->roi[i] : 0.0;
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
    if (!v->counters && hipMalloc((void**)&v->counters, 64) != hipSuccess)
      return fail(SG_ERR_OUT_OF_MEMORY, "counter allocation failed");
    SG_HIP(hipMemsetAsync(v->mb_bits, 0, (size_t)words * 4, s));
    SG_HIP(hipMemsetAsync(v->counters, 0, 64, s));
    a.mb_bits = v->mb_bits;
    a.counters = v->counters;
    for (int i = 0; i < kMaxChannels * kMaxLevels; ++i) a.level_mb_off[i] = offs[i];
    st = launch_raycast(v, a, true, s);
    if (st != SG_OK) return st;
    std::vector<uint32_t> hb((size_t)words);
    uint64_t cnt[8];
    SG_HIP(hipMemcpyAsync(hb.data(), v->mb_bits, (size_t)words * 4, hipMemcpyDeviceToHost, s));
    SG_HIP(hipMemcpyAsync(cnt, v->counters, 64, hipMemcpyDeviceToHost, s));
    SG_HIP(hipStreamSynchronize(s));
    uint64_t pop = 0;
    for (uint32_t x : hb) pop += (uint64_t)__builtin_popcount(x);
    stats->total_samples = cnt[0];
    stats->microblocks = pop;
    stats->node_visits = cnt[1];
    stats->slabs = cnt[2];
    stats->staged_bytes = cnt[3];
    return SG_OK;
  }
  st = launch_raycast(v, a, false, s);
  if (st != SG_OK) return st;
  if (timed) return timing_mark(v, s);
  return SG_OK;
}

}  // namespace sg

extern "C" sg_status sg_render_views(sg_volume* vol, int32_t n_views, const sg_view* views,
                                     const sg_render_params* params, float* const* out_rgba,
                                     float* const* out_depth, void* hip_stream) {
  return sg::render(vol, n_views, views, params, out_rgba, out_depth, nullptr, hip_stream);
}

extern "C" sg_status sg_render_views_stats(sg_volume* vol, int32_t n_views,
                                           const sg_view* views,
                                           const sg_render_params* params,
                                           float* const* out_rgba, float* const* out_depth,
                                           sg_render_stats* stats, void* hip_stream) {
  if (!stats) return sg::fail(SG_ERR_INVALID_ARG, "stats is NULL");
  return sg::render(vol, n_views, views, params, out_rgba, out_depth, stats, hip_stream);
}
