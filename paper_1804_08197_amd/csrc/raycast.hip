// raycast.hip -- the hot loop: per-pixel rays through the LOD cut, front to
// back, with trilinear sampling, transfer-function lookup and
// emission-absorption compositing with early termination (Sec 5.1, 5.2).
//
// Launch: one 256-thread workgroup per 16x16 pixel tile, four wave64s of
// 8x8 pixels each; the tiles of all views form one grid (stereo pair or
// batch in one launch, Sec 5.3). Workgroup ids are remapped so that each of
// the 8 XCDs (each with its own L2) receives a contiguous band of tiles.
//
// Per ray:
//  * FP64 set-up: direction from the pixel tangents, entry/exit against the
//    volume box (Sec 5.1, x0 and x1).
//  * A 3D DDA over the level-0 brick grid finds the cut nodes the ray
//    crosses, in order (Sec 5.2: blocks rendered front to back, the ray
//    continued inside each block). The cut map gives the node of each cell;
//    consecutive cells of the same node are one segment. The node's
//    parameter interval [t_in, t_out] is computed from its box in FP64.
//    Empty nodes are skipped.
//  * Inside a segment of level L the ray is sampled every
//    D = step * 2^L level-0 units at the midpoints of the sub-intervals (the
//    last one partial). Sample positions are evaluated in FP32 in the node's
//    brick-local coordinates (small magnitudes), from an FP64 segment origin.
//  * Trilinear interpolation reads the 8 stencil voxels from the node's pool
//    slot; the apron makes clamping unnecessary. The transfer function lives
//    in LDS. a = 1 - exp(-rho s), C += (1 - A) a rgb, A += (1 - A) a; the ray
//    stops when A >= ert (early ray termination).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sg_internal.h"

namespace sg {

namespace {

// 1 - exp(-x) for x >= 0 with small absolute and relative error: a Taylor
// polynomial below 1/16 (avoids the cancellation of 1 - exp(-x)), the
// exponential above.
__device__ __forceinline__ float one_minus_exp_neg(float x) {
  float p = x * (1.0f - x * (0.5f - x * (0.16666667f - x * (0.041666668f - x * 0.0083333333f))));
  float q = 1.0f - __expf(-x);
  return x < 0.0625f ? p : q;
}

__device__ __forceinline__ float lerpf(float a, float b, float t) {
  return fmaf(t, b - a, a);
}

// Slab test of e + t d against [lo, hi]; same operations as the CPU
// reference so that segment ends agree to the bit.
__device__ __forceinline__ bool box_interval(const double e[3], const double d[3],
                                             const double lo[3], const double hi[3],
                                             double& t0, double& t1) {
  double a = -INFINITY, b = INFINITY;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (d[i] != 0.0) {
      double ta = (lo[i] - e[i]) / d[i];
      double tb = (hi[i] - e[i]) / d[i];
      double mn = ta < tb ? ta : tb;
      double mx = ta < tb ? tb : ta;
      if (mn > a) a = mn;
      if (mx < b) b = mx;
    } else if (!(lo[i] <= e[i] && e[i] <= hi[i])) {
      t0 = 0.0;
      t1 = 0.0;
      return false;
    }
  }
  t0 = a;
  t1 = b;
  return a < b;
}

template <typename T>
__device__ __forceinline__ float ld(const T* p) {
  return (float)(*p);
}

template <typename T, int CH, bool STATS>
__global__ __launch_bounds__(256) void raycast_kernel(RenderArgs a) {
  extern __shared__ float4 s_tf[];
  const int ntf = CH * (a.tf_n + 1);
  for (int i = threadIdx.x; i < ntf; i += 256)
    s_tf[i] = reinterpret_cast<const float4*>(a.tf)[i];
  __syncthreads();

  // XCD-aware tile order: hardware places workgroup i on XCD i % 8.
  const int G = a.total_tiles;
  const int q8 = G >> 3;
  const int bid = blockIdx.x;
  const int tile = bid < (q8 << 3) ? (bid & 7) * q8 + (bid >> 3) : bid;
  int v = 0;
  {
    int lo = 0, hi = a.n_views - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (a.views[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    v = lo;
  }
  const ViewDev& V = a.views[v];
  const int lt = tile - V.tile_begin;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int px = tx * 16 + (w & 1) * 8 + (lane & 7);
  const int py = ty * 16 + (w >> 1) * 8 + (lane >> 3);
  if (px >= V.W || py >= V.H) return;

  // --- ray set-up in FP64 (no contraction in this file)
  const double sx = V.tl + (((double)px + 0.5) / (double)V.W) * (V.tr - V.tl);
  const double sy = V.tt - (((double)py + 0.5) / (double)V.H) * (V.tt - V.tb);
  double e[3], d[3];
  {
    double w3[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      e[i] = V.e[i];
      w3[i] = (V.R[3 * i + 0] * sx + V.R[3 * i + 1] * sy) + V.R[3 * i + 2] * (-1.0);
    }
    double len = sqrt((w3[0] * w3[0] + w3[1] * w3[1]) + w3[2] * w3[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) d[i] = w3[i] / len;
  }

  float Cr = 0.f, Cg = 0.f, Cb = 0.f, A = 0.f;
  float depth = INFINITY;
  const bool want_depth = V.depth != nullptr;
  int nsamp = 0;
  double tn, tf;
  {
    const double lo[3] = {0.0, 0.0, 0.0};
    const double hi[3] = {(double)a.dims[0], (double)a.dims[1], (double)a.dims[2]};
    box_interval(e, d, lo, hi, tn, tf);
    if (tn < 0.0) tn = 0.0;
  }
  if (tn < tf) {
    // --- DDA over level-0 brick cells
    const double Bd = (double)a.B;
    int c[3], st[3];
    double tnext[3], inv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double p = e[i] + tn * d[i];
      int ci = (int)floor(p / Bd);
      c[i] = ci < 0 ? 0 : (ci > a.grid0[i] - 1 ? a.grid0[i] - 1 : ci);
      if (d[i] > 0.0) {
        st[i] = 1;
        inv[i] = 1.0 / d[i];
        tnext[i] = (Bd * (double)(c[i] + 1) - e[i]) * inv[i];
      } else if (d[i] < 0.0) {
        st[i] = -1;
        inv[i] = 1.0 / d[i];
        tnext[i] = (Bd * (double)c[i] - e[i]) * inv[i];
      } else {
        st[i] = 0;
        inv[i] = 0.0;
        tnext[i] = INFINITY;
      }
    }
    const int32_t* cutmap = a.cutmap + V.cut_off;
    bool alive = true;
    while (alive) {
      const int32_t node =
          cutmap[((int64_t)c[2] * a.grid0[1] + c[1]) * a.grid0[0] + c[0]];
      const NodeInfo ni = a.info[node];
      const int L = ni.level;
      // node box (level-0 units, clipped to the volume)
      double blo[3], bhi[3];
      int clo[3], chi[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        int64_t wdt = (int64_t)a.B << L;
        int64_t l0 = wdt * ni.b[i];
        int64_t h0 = wdt * (ni.b[i] + 1);
        if (h0 > a.dims[i]) h0 = a.dims[i];
        blo[i] = (double)l0;
        bhi[i] = (double)h0;
        clo[i] = ni.b[i] << L;
        chi[i] = min(((ni.b[i] + 1) << L) - 1, a.grid0[i] - 1);
      }
      double t0, t1;
      box_interval(e, d, blo, bhi, t0, t1);
      if (t0 < tn) t0 = tn;
      if (t1 > tf) t1 = tf;
      const bool skip = a.skip_empty && a.empty[node];
      if (t0 < t1 && !skip) {
        // --- segment integration at level L
        const double Dd = a.step * (double)((int64_t)1 << L);
        const double len = t1 - t0;
        const int n = (int)ceil(len / Dd);
        const float s_last = (float)(len - (double)(n - 1) * Dd);
        const float Df = (float)Dd;
        const double inv_s = 1.0 / (double)((int64_t)1 << L);
        float q0[3], dq[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          double o = (double)((int64_t)a.B * ((int64_t)ni.b[i] << L));
          q0[i] = (float)(((e[i] - o) + t0 * d[i]) * inv_s + 0.5);
          dq[i] = (float)(d[i] * inv_s);
        }
        const T* slot[CH];
#pragma unroll
        for (int ch = 0; ch < CH; ++ch)
          slot[ch] = reinterpret_cast<const T*>(
              a.pool + (int64_t)a.page[(int64_t)ch * a.nodes + node] * a.slot_bytes);
        const int S = a.S;
        const int S2 = S * S;
        for (int k = 0; k < n; ++k) {
          const float s = k == n - 1 ? s_last : Df;
          const float tau = fmaf((float)k, Df, 0.5f * s);
          const float qx = fmaf(tau, dq[0], q0[0]);
          const float qy = fmaf(tau, dq[1], q0[1]);
          const float qz = fmaf(tau, dq[2], q0[2]);
          // stencil origin, kept inside the slot (it always is for samples
          // inside the node box; the clamp only guards memory safety)
          const int ix = min(max((int)qx, 0), a.B);
          const int iy = min(max((int)qy, 0), a.B);
          const int iz = min(max((int)qz, 0), a.B);
          const float fx = qx - (float)ix, fy = qy - (float)iy, fz = qz - (float)iz;
          const int base = (iz * S + iy) * S + ix;
          float rho = 0.f, er = 0.f, eg = 0.f, eb = 0.f;
#pragma unroll
          for (int ch = 0; ch < CH; ++ch) {
            const T* p0 = slot[ch] + base;
            const T* p1 = p0 + S2;
            float c00 = lerpf(ld(p0), ld(p0 + 1), fx);
            float c10 = lerpf(ld(p0 + S), ld(p0 + S + 1), fx);
            float c01 = lerpf(ld(p1), ld(p1 + 1), fx);
            float c11 = lerpf(ld(p1 + S), ld(p1 + S + 1), fx);
            float c0 = lerpf(c00, c10, fy);
            float c1 = lerpf(c01, c11, fy);
            float val = lerpf(c0, c1, fz);
            float u = fmaf(val, a.tf_scale[ch], a.tf_bias[ch]);
            u = fminf(fmaxf(u, 0.0f), (float)(a.tf_n - 1));
            const int k0 = (int)u;
            const float wt = u - (float)k0;
            const float4 t0v = s_tf[ch * (a.tf_n + 1) + k0];
            const float4 t1v = s_tf[ch * (a.tf_n + 1) + k0 + 1];
            const float r = lerpf(t0v.x, t1v.x, wt);
            const float g = lerpf(t0v.y, t1v.y, wt);
            const float b = lerpf(t0v.z, t1v.z, wt);
            const float rh = lerpf(t0v.w, t1v.w, wt);
            if (CH == 1) {
              er = r;
              eg = g;
              eb = b;
              rho = rh;
            } else {
              rho += rh;
              er = fmaf(rh, r, er);
              eg = fmaf(rh, g, eg);
              eb = fmaf(rh, b, eb);
            }
            if (STATS) {
              // distinct 4^3 blocks of this level read by the stencil
              const int32_t* nL = a.ldims[L];
              int gl[3] = {a.B * ni.b[0] - 1 + ix, a.B * ni.b[1] - 1 + iy,
                           a.B * ni.b[2] - 1 + iz};
              int lo3[3], hi3[3], m3[3];
#pragma unroll
              for (int i = 0; i < 3; ++i) {
                int g0 = gl[i] < 0 ? 0 : (gl[i] > nL[i] - 1 ? nL[i] - 1 : gl[i]);
                int g1 = gl[i] + 1 > nL[i] - 1 ? nL[i] - 1 : gl[i] + 1;
                lo3[i] = g0 >> 2;
                hi3[i] = g1 >> 2;
                m3[i] = (nL[i] + 3) >> 2;
              }
              const int64_t off = a.level_mb_off[ch * kMaxLevels + L];
              for (int zz = lo3[2]; zz <= hi3[2]; ++zz)
                for (int yy = lo3[1]; yy <= hi3[1]; ++yy)
                  for (int xx = lo3[0]; xx <= hi3[0]; ++xx) {
                    int64_t bit = off + ((int64_t)zz * m3[1] + yy) * m3[0] + xx;
                    atomicOr(a.mb_bits + (bit >> 5), 1u << (bit & 31));
                  }
            }
          }
          if (CH > 1) {
            const float inv_r = rho > 0.f ? 1.0f / rho : 0.f;
            er *= inv_r;
            eg *= inv_r;
            eb *= inv_r;
          }
          const float al = one_minus_exp_neg(rho * s);
          const float wgt = (1.0f - A) * al;
          Cr = fmaf(wgt, er, Cr);
          Cg = fmaf(wgt, eg, Cg);
          Cb = fmaf(wgt, eb, Cb);
          A += wgt;
          if (STATS) ++nsamp;
          if (want_depth && depth == INFINITY && A >= a.depth_alpha)
            depth = (float)(t0 + (double)tau);
          if (A >= a.ert) {
            alive = false;
            break;
          }
        }
      }
      if (!alive) break;
      // --- advance the DDA out of this node
      bool inside = true;
      while (inside) {
        int ax = 0;
        if (tnext[1] < tnext[ax]) ax = 1;
        if (tnext[2] < tnext[ax]) ax = 2;
        if (!(tnext[ax] < tf)) {
          alive = false;
          break;
        }
        c[ax] += st[ax];
        if (c[ax] < 0 || c[ax] >= a.grid0[ax]) {
          alive = false;
          break;
        }
        tnext[ax] = (Bd * (double)(c[ax] + (st[ax] > 0 ? 1 : 0)) - e[ax]) * inv[ax];
        inside = c[0] >= clo[0] && c[0] <= chi[0] && c[1] >= clo[1] && c[1] <= chi[1] &&
                 c[2] >= clo[2] && c[2] <= chi[2];
      }
    }
  }
  const float omA = 1.0f - A;
  const int64_t pix = (int64_t)py * V.W + px;
  float4 out;
  out.x = fmaf(omA, a.bg[0], Cr);
  out.y = fmaf(omA, a.bg[1], Cg);
  out.z = fmaf(omA, a.bg[2], Cb);
  out.w = fmaf(omA, a.bg[3], A);
  reinterpret_cast<float4*>(V.rgba)[pix] = out;
  if (V.depth) V.depth[pix] = depth;
  if (STATS) {
    if (V.nsamp) V.nsamp[pix] = nsamp;
    atomicAdd((unsigned long long*)a.counters, (unsigned long long)nsamp);
  }
}

template <typename T, int CH>
sg_status launch_t(const RenderArgs& a, bool stats, hipStream_t s) {
  const size_t lds = (size_t)CH * (a.tf_n + 1) * sizeof(float4);
  if (stats)
    hipLaunchKernelGGL((raycast_kernel<T, CH, true>), dim3(a.total_tiles), dim3(256), lds, s,
                       a);
  else
    hipLaunchKernelGGL((raycast_kernel<T, CH, false>), dim3(a.total_tiles), dim3(256), lds,
                       s, a);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

template <typename T>
sg_status launch_ch(const RenderArgs& a, int C, bool stats, hipStream_t s) {
  switch (C) {
    case 1: return launch_t<T, 1>(a, stats, s);
    case 2: return launch_t<T, 2>(a, stats, s);
    case 3: return launch_t<T, 3>(a, stats, s);
    default: return launch_t<T, 4>(a, stats, s);
  }
}

bool finite(double x) { return std::isfinite(x); }

}  // namespace

sg_status launch_raycast(Volume* v, const RenderArgs& a, bool stats, hipStream_t s) {
  if (v->bpv == 1) return launch_ch<uint8_t>(a, v->d.channels, stats, s);
  return launch_ch<uint16_t>(a, v->d.channels, stats, s);
}

sg_status prepare_views(Volume* v, int n_views, const sg_view* views,
                        const sg_render_params* p, float* const* rgba,
                        float* const* depth, int32_t* const* nsamp, hipStream_t s,
                        int* total_tiles) {
  if (n_views < 1 || n_views > 4096 || !views || !p)
    return fail(SG_ERR_INVALID_ARG, "views: n_views must be in [1, 4096]");
  if (!(finite(p->step_voxels) && p->step_voxels >= 1.0 / 64 && p->step_voxels <= 64.0) || !finite(p->ert_alpha) ||
      !(finite(p->lod_tau_px) && p->lod_tau_px > 0.0) || !finite(p->depth_alpha) ||
      p->lod_bias < 0 || p->lod_bias >= v->L || p->timepoint < 0 ||
      p->timepoint >= v->d.timepoints || (p->flags & ~(uint32_t)(SG_LOD | SG_SKIP_EMPTY)) ||
      p->reserved != 0)
    return fail(SG_ERR_INVALID_ARG, "render params out of range");
  for (int i = 0; i < 4; ++i)
    if (!finite(p->background[i])) return fail(SG_ERR_INVALID_ARG, "background not finite");
  std::vector<ViewDev> hv(n_views);
  int64_t tiles = 0;
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
    o.tile_begin = (int32_t)tiles;
    tiles += (int64_t)o.tiles_x * ((w.height + 15) / 16);
    o.cut_off = (int64_t)i * cells;
    o.rgba = rgba ? rgba[i] : nullptr;
    o.depth = depth ? depth[i] : nullptr;
    o.nsamp = nsamp ? nsamp[i] : nullptr;
  }
  if (tiles > 0x7FFFFFFF) return fail(SG_ERR_INVALID_ARG, "too many pixels in one call");
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
  *total_tiles = (int)tiles;
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
  const size_t lds = (size_t)v->d.channels * (v->tf_n + 1) * 16;
  if (lds > 65536) return fail(SG_ERR_UNSUPPORTED, "transfer tables exceed 64 KiB of LDS");
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  hipStream_t s = (hipStream_t)hip_stream;
  sg_status st = commit(v, s);
  if (st != SG_OK) return st;
  int tiles = 0;
  st = prepare_views(v, n_views, views, params, out_rgba, out_depth,
                     stats ? stats->samples : nullptr, s, &tiles);
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
  for (int i = 0; i < 3; ++i) {
    a.dims[i] = v->d.dims[i];
    a.grid0[i] = v->grid[0][i];
  }
  a.n_views = n_views;
  a.total_tiles = tiles;
  a.tf_n = v->tf_n;
  a.B = v->B;
  a.S = v->S;
  a.skip_empty = (params->flags & SG_SKIP_EMPTY) ? 1 : 0;
  a.step = params->step_voxels;
  a.ert = (float)params->ert_alpha;
  a.depth_alpha = (float)params->depth_alpha;
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
