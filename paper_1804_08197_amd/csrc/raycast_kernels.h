// raycast_kernels.h -- the hot loop: per-pixel rays through the LOD cut, front to
// back, with trilinear sampling, transfer-function lookup and
// emission-absorption compositing with early termination (Sec 5.1, 5.2).
//
// Launch: one 256-thread workgroup per 16x16 pixel tile, four wave64s of
// 8x8 pixels each; the tiles of all views form one grid (stereo pair or
// batch in one launch, Sec 5.3). Workgroup ids are remapped so that blocks
// of 4x4 tiles are dealt to the 8 XCDs (each with its own L2) in turn.
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
//  * Trilinear interpolation of the node's brick (the apron makes clamping
//    unnecessary), transfer function from LDS, a = 1 - exp(-rho s),
//    C += (1 - A) a rgb, A += (1 - A) a; the ray stops when A >= ert.
//
// Optical models (Sec 5.1), a template parameter of both kernels:
//  * emission-absorption (above);
//  * emission-only: C += rgb s with rgb the summed emission of the channels,
//    alpha stays 0 (Sec 5.6), no early termination, dark nodes skipped;
//  * maximum intensity: the running maximum of each channel's trilinear
//    value; at the end C is the summed emission of the maxima, alpha 0. A
//    node whose stored maximum cannot raise any running maximum is passed
//    over (exact: a trilinear value never exceeds its largest voxel).
// Rays may be clipped (Sec 6 cut planes and region of interest; Sec 5.6 the
// distance of opaque geometry per pixel) and their pixels placed by a radial
// lens map (Sec 5.3, rays uniform over the wrapped image).
//
// Two kernels share all of the per-ray arithmetic, so they give bit-identical
// images:
//  * staged (default): the 64 rays of a wave walk their nodes in lockstep,
//    in the octree's front-to-back order for the view's eye (every ray meets
//    nodes in that order, so each lane still sees its own segments in
//    order). For the node at hand the wave stages, slab by slab along the
//    dominant ray axis, the part of the brick its rays cross into LDS with
//    coalesced dword loads, and the trilinear stencils read LDS.
//  * gather: every lane reads its stencils straight from the pool.
#pragma once

#include <cmath>

#include "sg_internal.h"

namespace sg {

namespace {

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

template <typename P>
__device__ __forceinline__ float ld(P p) {
  return (float)(*p);
}

// Trilinear value of the stencil whose (0,0,0) corner is at p0; sy / sz are
// the row and plane strides of the array p0 points into.
template <typename P>
__device__ __forceinline__ float trilinear(P p0, int sy, int sz, float fx, float fy, float fz) {
  const float c00 = lerpf(ld(p0), ld(p0 + 1), fx);
  const float c10 = lerpf(ld(p0 + sy), ld(p0 + sy + 1), fx);
  const float c01 = lerpf(ld(p0 + sz), ld(p0 + sz + 1), fx);
  const float c11 = lerpf(ld(p0 + sz + sy), ld(p0 + sz + sy + 1), fx);
  const float c0 = lerpf(c00, c10, fy);
  const float c1 = lerpf(c01, c11, fy);
  return lerpf(c0, c1, fz);
}

// Stencil corner index of a brick-local position along one axis, clamped to
// [0, B] (bf = B) for reads of the pool. Clamping the position first (one
// median) gives the same index as clamping the truncated one: a position
// in (-1, 0) truncates to 0 either way, and every finite position gives
// min(max(trunc(q), 0), B).
__device__ __forceinline__ int clamp_index(float q, float bf) {
  return (int)__builtin_amdgcn_fmed3f(q, 0.0f, bf);
}

// Offset of stored voxel (x, y, z) in a micro-block slot with M blocks per
// edge (slot_index for M > 0, in 32 bits: slots hold fewer than 2^31 voxels).
__device__ __forceinline__ int mb_index(int x, int y, int z, int M) {
  return ((__umul24(__umul24(z >> 2, M) + (y >> 2), M) + (x >> 2)) << 6) + ((z & 3) << 4) +
         ((y & 3) << 2) + (x & 3);
}
// The steps from a voxel to its +x, +y and +z neighbours in a micro-block
// slot: inside the voxel's block, or across into the next block.
struct MbSteps {
  int dx, dy, dz;
};
__device__ __forceinline__ MbSteps mb_steps(int x, int y, int z, int M) {
  // ((i & 3) + 1) >> 2 is 1 exactly on a block's last voxel; the products
  // take the scalar block strides as they are (a select between two
  // non-vector operands would first copy one into a vector register)
  const int cx = ((x & 3) + 1) >> 2, cy = ((y & 3) + 1) >> 2, cz = ((z & 3) + 1) >> 2;
  return MbSteps{1 + cx * (64 - 4), 4 + cy * (64 * M - 16), 16 + cz * (64 * M * M - 64)};
}
// trilinear's value, operations and order for the stencil at stored index
// (ix, iy, iz) of a micro-block slot. The voxels are global-memory reads at
// 32-bit byte offsets from the slot (a slot base held in scalar registers
// then costs one vector register per address, not two). LEAN: the four
// voxel pairs are read one after another (no instruction moves across the
// scheduling barriers), which keeps few registers live in a rarely taken
// path at the cost of latency.
template <typename T, bool LEAN = false>
__device__ __forceinline__ float trilinear_mb(const T* slot, int ix, int iy, int iz, int M,
                                              float fx, float fy, float fz) {
  typedef __attribute__((address_space(1))) const uint8_t* Global;
  const Global base = (Global)(reinterpret_cast<const uint8_t*>(slot));
  const uint32_t e0 = (uint32_t)mb_index(ix, iy, iz, M) * (uint32_t)sizeof(T);
  const MbSteps d = mb_steps(ix, iy, iz, M);
  const uint32_t bx = (uint32_t)d.dx * sizeof(T), by = (uint32_t)d.dy * sizeof(T),
                 bz = (uint32_t)d.dz * sizeof(T);
  auto at = [&](uint32_t e) {
    return (float)*(__attribute__((address_space(1))) const T*)(base + e);
  };
  const float c00 = lerpf(at(e0), at(e0 + bx), fx);
  if (LEAN) __builtin_amdgcn_sched_barrier(0);
  const float c10 = lerpf(at(e0 + by), at(e0 + by + bx), fx);
  if (LEAN) __builtin_amdgcn_sched_barrier(0);
  const float c01 = lerpf(at(e0 + bz), at(e0 + bz + bx), fx);
  if (LEAN) __builtin_amdgcn_sched_barrier(0);
  const float c11 = lerpf(at(e0 + bz + by), at(e0 + bz + by + bx), fx);
  const float c0 = lerpf(c00, c10, fy);
  const float c1 = lerpf(c01, c11, fy);
  return lerpf(c0, c1, fz);
}
// The pool stencil of either slot layout (MB: micro-block slots, see
// slot_index).
template <bool MB, typename T>
__device__ __forceinline__ float pool_trilinear(const RenderArgs& a, const T* slot, int ix, int iy,
                                                int iz, float fx, float fy, float fz) {
  if (MB) return trilinear_mb(slot, ix, iy, iz, a.M, fx, fy, fz);
  return trilinear(slot + (iz * a.S + iy) * a.Sx + ix, a.Sx, a.S * a.Sx, fx, fy, fz);
}

// A voxel of a staged region in LDS. The reads are volatile so that the
// compiler issues one aligned read per voxel: it would otherwise merge the
// two voxels of a stencil row into one 2- or 4-byte read, which is
// misaligned for every other stencil position, and misaligned LDS reads
// are many times slower than aligned ones on gfx950 (measured: the ray
// caster's frame took 8.4 ms with merged reads, 5.7 ms with aligned ones).
template <typename T>
__device__ __forceinline__ float lds_voxel(const char* p) {
  typedef __attribute__((address_space(3))) const volatile T* Lds;
  return (float)*(Lds)(__attribute__((address_space(3))) const char*)p;
}

// The same trilinear value from a byte address in LDS with row and plane
// steps in bytes (saves the index scaling in the sample loop).
template <typename T>
__device__ __forceinline__ float trilinear_bytes(const char* p0, int syb, int szb, float fx,
                                                 float fy, float fz) {
  auto at = [&](int off) { return lds_voxel<T>(p0 + off); };
  const float c00 = lerpf(at(0), at(sizeof(T)), fx);
  const float c10 = lerpf(at(syb), at(syb + sizeof(T)), fx);
  const float c01 = lerpf(at(szb), at(szb + sizeof(T)), fx);
  const float c11 = lerpf(at(szb + syb), at(szb + syb + sizeof(T)), fx);
  const float c0 = lerpf(c00, c10, fy);
  const float c1 = lerpf(c01, c11, fy);
  return lerpf(c0, c1, fz);
}

// ----------------------------------------------------------------- per ray
// The eye is not part of the per-ray state: every ray of a wave belongs to
// one view, so the kernels read it from the view record (scalar registers).
struct Ray {
  double d[3];
  double tn, tf;
  double tnext[3], inv[3];
  int c[3], st[3];
  bool alive;   // has entered the volume and is not terminated / exhausted
  // current segment (valid when alive)
  int node, L, b[3];
  double t0, t1;
  uint64_t key;
  // sampling state of the current segment (brick-local FP32 frame)
  float q0[3], dq[3], Df, s_last;
  float tau, tau_last;  // ray parameter of sample k and of the last sample
  int n, k;
  // accumulation: premultiplied colour and the transmittance T = 1 - alpha
  float Cr, Cg, Cb, T, depth;
  // depth: the smallest ray parameter in the current segment whose alpha
  // reached the depth threshold (+inf: none yet, or no depth wanted),
  // converted to the depth once, when the segment ends
  float dtau;
  float vmax[kMaxChannels];  // maximum intensity: running maxima
  bool sampled;              // maximum intensity: at least one sample taken
  int nsamp;
};

// The ray of pixel (px, py) of a view (Sec 5.1): eye e and unit direction d
// through the pixel centre, in FP64.
__device__ __forceinline__ void view_ray(const ViewDev& V, int px, int py, double e[3],
                                         double d[3]) {
  double sx = V.tl + (((double)px + 0.5) / (double)V.W) * (V.tr - V.tl);
  double sy = V.tt - (((double)py + 0.5) / (double)V.H) * (V.tt - V.tb);
  if (V.lens_on) {
    // wrapped space (Sec 5.3): the uniform pixel grid is moved radially
    // about the lens centre by 1 + k1 r^2 + k2 r^4
    const double dx = sx - V.lens[2], dy = sy - V.lens[3];
    const double r2 = dx * dx + dy * dy;
    const double f = 1.0 + r2 * (V.lens[0] + r2 * V.lens[1]);
    sx = V.lens[2] + dx * f;
    sy = V.lens[3] + dy * f;
  }
  double w3[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    e[i] = V.e[i];
    w3[i] = (V.R[3 * i + 0] * sx + V.R[3 * i + 1] * sy) + V.R[3 * i + 2] * (-1.0);
  }
  const double len = sqrt((w3[0] * w3[0] + w3[1] * w3[1]) + w3[2] * w3[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) d[i] = w3[i] / len;
}

__device__ __forceinline__ void ray_setup(Ray& r, const RenderArgs& a, const ViewDev& V, int px,
                                          int py) {
  double e_unused[3];
  view_ray(V, px, py, e_unused, r.d);
  const double* e = V.e;
  r.Cr = r.Cg = r.Cb = 0.f;
  r.T = 1.f;
#pragma unroll
  for (int c = 0; c < kMaxChannels; ++c) r.vmax[c] = -INFINITY;
  r.sampled = false;
  r.depth = INFINITY;
  r.dtau = INFINITY;
  r.nsamp = 0;
  r.n = r.k = 0;
  const double lo[3] = {0.0, 0.0, 0.0};
  const double hi[3] = {(double)a.dims[0], (double)a.dims[1], (double)a.dims[2]};
  box_interval(e, r.d, lo, hi, r.tn, r.tf);
  if (r.tn < 0.0) r.tn = 0.0;
  r.alive = r.tn < r.tf;
  if (!r.alive) return;
  // clipping: cut planes keep (n . p) + w <= 0 (Sec 6), the region of
  // interest keeps its box (Sec 6), opaque geometry ends the ray (Sec 5.6)
  for (int j = 0; j < a.n_planes; ++j) {
    const double* q = a.planes[j];
    const double pa = ((q[0] * e[0] + q[1] * e[1]) + q[2] * e[2]) + q[3];
    const double pb = (q[0] * r.d[0] + q[1] * r.d[1]) + q[2] * r.d[2];
    if (pb > 0.0) {
      const double t = -pa / pb;
      if (t < r.tf) r.tf = t;
    } else if (pb < 0.0) {
      const double t = -pa / pb;
      if (t > r.tn) r.tn = t;
    } else if (pa > 0.0) {
      r.tf = r.tn;
    }
  }
  if (a.roi_on) {
    double t0, t1;
    if (!box_interval(e, r.d, a.roi, a.roi + 3, t0, t1)) {
      r.tf = r.tn;
    } else {
      if (t0 > r.tn) r.tn = t0;
      if (t1 < r.tf) r.tf = t1;
    }
  }
  if (V.limit) {
    const double lim = (double)V.limit[(int64_t)py * V.W + px];
    if (lim < r.tf) r.tf = lim;
  }
  r.alive = r.tn < r.tf;
  if (!r.alive) return;
  const double Bd = (double)a.B;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double p = e[i] + r.tn * r.d[i];
    const int ci = (int)floor(p / Bd);
    r.c[i] = ci < 0 ? 0 : (ci > a.grid0[i] - 1 ? a.grid0[i] - 1 : ci);
    if (r.d[i] > 0.0) {
      r.st[i] = 1;
      r.inv[i] = 1.0 / r.d[i];
      r.tnext[i] = (Bd * (double)(r.c[i] + 1) - e[i]) * r.inv[i];
    } else if (r.d[i] < 0.0) {
      r.st[i] = -1;
      r.inv[i] = 1.0 / r.d[i];
      r.tnext[i] = (Bd * (double)r.c[i] - e[i]) * r.inv[i];
    } else {
      r.st[i] = 0;
      r.inv[i] = 0.0;
      r.tnext[i] = INFINITY;
    }
  }
}

// The depth of the first sample found in the current segment: t0 + tau in
// FP64, rounded once (the same operations as when formed at the sample);
// later segments cannot replace it.
__device__ __forceinline__ void finish_depth(Ray& r) {
  if (r.depth == INFINITY && r.dtau != INFINITY) r.depth = (float)(r.t0 + (double)r.dtau);
  r.dtau = INFINITY;
}

// Advance the ray to its next segment that needs samples: a cut node whose
// parameter interval is non-empty and that is not skipped as empty. With
// `first` the current DDA cell is examined before stepping.
template <int MODEL, int CH>
__device__ __forceinline__ void next_segment(Ray& r, const RenderArgs& a, const ViewDev& V,
                                             bool first) {
  finish_depth(r);  // before t0 moves on
  const int32_t* cutmap = a.cutmap + V.cut_off;
  const double* e = V.e;
  const double Bd = (double)a.B;
  bool step = !first;
  while (true) {
    if (step) {
      // leave the current node: step cells until one outside the node's box
      int clo[3], chi[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        clo[i] = r.b[i] << r.L;
        chi[i] = min(((r.b[i] + 1) << r.L) - 1, a.grid0[i] - 1);
      }
      bool inside = true;
      while (inside) {
        // next plane crossing; the axis is chosen with constant indices only
        // so that the ray state stays in registers
        const bool x_min = r.tnext[0] <= r.tnext[1] && r.tnext[0] <= r.tnext[2];
        const bool y_min = !x_min && r.tnext[1] <= r.tnext[2];
        const double tmin = x_min ? r.tnext[0] : (y_min ? r.tnext[1] : r.tnext[2]);
        if (!(tmin < r.tf)) {
          r.alive = false;
          return;
        }
        bool out;
        if (x_min) {
          r.c[0] += r.st[0];
          out = r.c[0] < 0 || r.c[0] >= a.grid0[0];
          r.tnext[0] = (Bd * (double)(r.c[0] + (r.st[0] > 0 ? 1 : 0)) - e[0]) * r.inv[0];
        } else if (y_min) {
          r.c[1] += r.st[1];
          out = r.c[1] < 0 || r.c[1] >= a.grid0[1];
          r.tnext[1] = (Bd * (double)(r.c[1] + (r.st[1] > 0 ? 1 : 0)) - e[1]) * r.inv[1];
        } else {
          r.c[2] += r.st[2];
          out = r.c[2] < 0 || r.c[2] >= a.grid0[2];
          r.tnext[2] = (Bd * (double)(r.c[2] + (r.st[2] > 0 ? 1 : 0)) - e[2]) * r.inv[2];
        }
        if (out) {
          r.alive = false;
          return;
        }
        inside = r.c[0] >= clo[0] && r.c[0] <= chi[0] && r.c[1] >= clo[1] &&
                 r.c[1] <= chi[1] && r.c[2] >= clo[2] && r.c[2] <= chi[2];
      }
    }
    step = true;
    r.node = cutmap[((int64_t)r.c[2] * a.grid0[1] + r.c[1]) * a.grid0[0] + r.c[0]];
    const NodeInfo ni = a.info[r.node];
    r.L = ni.level;
#pragma unroll
    for (int i = 0; i < 3; ++i) r.b[i] = ni.b[i];
    // skipped nodes are dropped before any box arithmetic
    if (MODEL != kModelMip) {
      if (a.skip_empty && (a.empty[r.node] & (MODEL == kModelEmission ? 2 : 1))) continue;
    } else if (a.skip_empty && r.sampled) {
      bool raise = false;
#pragma unroll
      for (int ch = 0; ch < CH; ++ch)
        raise |= (float)a.range[2 * ((int64_t)ch * a.nodes + r.node) + 1] > r.vmax[ch];
      if (!raise) continue;
    }
    double blo[3], bhi[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int64_t wdt = (int64_t)a.B << r.L;
      const int64_t l0 = wdt * ni.b[i];
      int64_t h0 = wdt * (ni.b[i] + 1);
      if (h0 > a.dims[i]) h0 = a.dims[i];
      blo[i] = (double)l0;
      bhi[i] = (double)h0;
    }
    double t0, t1;
    box_interval(e, r.d, blo, bhi, t0, t1);
    if (t0 < r.tn) t0 = r.tn;
    if (t1 > r.tf) t1 = r.tf;
    if (!(t0 < t1)) continue;
    r.key = visibility_key(a.key_levels, a.B, e, r.L, r.b);
    r.t0 = t0;
    r.t1 = t1;
    // sampling frame: stored index of the brick, FP32 from an FP64 origin
    const double Dd = a.step * (double)((int64_t)1 << r.L);
    const double len = t1 - t0;
    r.n = (int)ceil(len / Dd);
    r.k = 0;
    r.s_last = (float)(len - (double)(r.n - 1) * Dd);
    r.Df = (float)Dd;
    r.tau = 0.5f * r.Df;  // (k + 1/2) D is exact: D is a power of two
    r.tau_last = fmaf((float)(r.n - 1), r.Df, 0.5f * r.s_last);
    const double inv_s = 1.0 / (double)((int64_t)1 << r.L);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double o = (double)((int64_t)a.B * ((int64_t)r.b[i] << r.L));
      r.q0[i] = (float)(((e[i] - o) + t0 * r.d[i]) * inv_s + 0.5);
      r.dq[i] = (float)(r.d[i] * inv_s);
    }
    return;
  }
}

// Ray parameter (from the segment start, level-0 units) of sample k.
__device__ __forceinline__ float sample_tau(const Ray& r, int k) {
  const float s = k == r.n - 1 ? r.s_last : r.Df;
  return fmaf((float)k, r.Df, 0.5f * s);
}

// Shade and composite sample r.k; `fetch(ch, ix, iy, iz, fx, fy, fz)`
// returns the trilinear value of channel ch at stored index (ix, iy, iz)
// plus fraction. Returns false once the ray has terminated.
// Transfer function of channel ch at raw value val, from the table in LDS:
// linear interpolation between entries, clamped at both ends. The LDS table
// holds per entry k the value t[k] and the difference t[k+1] - t[k] (zero
// for the last entry), so each interpolation is one fused multiply-add,
// fma(w, t[k+1] - t[k], t[k]): the same operations, in the same FP32
// rounding, as lerpf(t[k], t[k+1], w).
__device__ __forceinline__ float4 tf_lookup(const RenderArgs& a, const float4* s_tf, int ch,
                                            float val, float scale, float bias) {
  float u = fmaf(val, scale, bias);
  u = __builtin_amdgcn_fmed3f(u, 0.0f, (float)(a.tf_n - 1));  // clamp (u is finite)
  const int k0 = (int)u;
  const float wt = __builtin_amdgcn_fractf(u);  // = u - k0 exactly, u >= 0
  const float4 t = s_tf[2 * (ch * a.tf_n + k0)];
  const float4 d = s_tf[2 * (ch * a.tf_n + k0) + 1];
  return make_float4(fmaf(wt, d.x, t.x), fmaf(wt, d.y, t.y), fmaf(wt, d.z, t.z),
                     fmaf(wt, d.w, t.w));
}

__device__ __forceinline__ float4 tf_lookup(const RenderArgs& a, const float4* s_tf, int ch,
                                            float val) {
  return tf_lookup(a, s_tf, ch, val, a.tf_scale[ch], a.tf_bias[ch]);
}

// The transfer-table windows of a run of samples, the offsets held in
// vector registers: the kernel arguments sit in scalar registers, and an FMA
// reads at most one of those, so an offset left there costs a move per
// sample.
template <int CH>
struct TfWin {
  float scale[CH], bias[CH];
};
template <int CH>
__device__ __forceinline__ TfWin<CH> tf_win(const RenderArgs& a) {
  TfWin<CH> w;
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) {
    float b = a.tf_bias[ch];
    asm volatile("" : "+v"(b));  // (a register move, no memory access)
    w.scale[ch] = a.tf_scale[ch];
    w.bias[ch] = b;
  }
  return w;
}

// Statistics: mark the distinct 4^3 blocks of the level read by the stencil
// at stored index (ix, iy, iz); consecutive samples mostly reuse the
// previous blocks, so marking happens only on change.
__device__ __forceinline__ void mark_microblocks(const Ray& r, const RenderArgs& a, int ch,
                                                 int ix, int iy, int iz, int* mk) {
  const int32_t* nL = a.ldims[r.L];
  const int gl[3] = {a.B * r.b[0] - 1 + ix, a.B * r.b[1] - 1 + iy, a.B * r.b[2] - 1 + iz};
  int lo3[3], hi3[3], m3[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int g0 = gl[i] < 0 ? 0 : (gl[i] > nL[i] - 1 ? nL[i] - 1 : gl[i]);
    const int g1 = gl[i] + 1 > nL[i] - 1 ? nL[i] - 1 : gl[i] + 1;
    lo3[i] = g0 >> 2;
    hi3[i] = g1 >> 2;
    m3[i] = (nL[i] + 3) >> 2;
  }
  const int key0 = (lo3[0] | (lo3[1] << 16)) ^ (r.L << 27);
  const int key1 = lo3[2] | (hi3[0] << 16);
  const int key2 = hi3[1] | (hi3[2] << 16);
  if (key0 == mk[0] && key1 == mk[1] && key2 == mk[2]) return;
  mk[0] = key0;
  mk[1] = key1;
  mk[2] = key2;
  const int64_t off = a.level_mb_off[ch * kMaxLevels + r.L];
  for (int zz = lo3[2]; zz <= hi3[2]; ++zz)
    for (int yy = lo3[1]; yy <= hi3[1]; ++yy)
      for (int xx = lo3[0]; xx <= hi3[0]; ++xx) {
        const int64_t bit = off + ((int64_t)zz * m3[1] + yy) * m3[0] + xx;
        atomicOr(a.mb_bits + (bit >> 5), 1u << (bit & 31));
      }
}

// Emission and extinction of the sample at ray parameter tau (from the
// segment start) of the emission-absorption model: the trilinear value of
// every channel, its table entry, channels added (extinction-weighted
// colour); `fetch(ch, ix, iy, iz, fx, fy, fz)` returns the trilinear value
// of channel ch at stored index (ix, iy, iz) plus fraction.
struct Shade {
  float rho, er, eg, eb;
};
template <int CH, bool STATS, bool CLAMP, typename F>
__device__ __forceinline__ Shade shade_ea(const Ray& r, const RenderArgs& a, const float4* s_tf,
                                          const TfWin<CH>& w, F&& fetch, float tau,
                                          int (*mb_key)[3]) {
  const float qx = fmaf(tau, r.dq[0], r.q0[0]);
  const float qy = fmaf(tau, r.dq[1], r.q0[1]);
  const float qz = fmaf(tau, r.dq[2], r.q0[2]);
  // stencil origin. Samples inside the node box always have it in
  // [0, B]; reads from the pool clamp it anyway to guard memory safety
  // (LDS reads need no guard: out-of-range LDS addresses cannot fault and
  // the staged region is proven to contain every staged stencil).
  const int ix = CLAMP ? clamp_index(qx, a.Bf) : (int)qx;
  const int iy = CLAMP ? clamp_index(qy, a.Bf) : (int)qy;
  const int iz = CLAMP ? clamp_index(qz, a.Bf) : (int)qz;
  // q >= 0, so fract(q) = q - floor(q) = q - ix (exact)
  const float fx = __builtin_amdgcn_fractf(qx), fy = __builtin_amdgcn_fractf(qy),
              fz = __builtin_amdgcn_fractf(qz);
  Shade z{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) {
    const float val = fetch(ch, ix, iy, iz, fx, fy, fz);
    if (STATS) mark_microblocks(r, a, ch, ix, iy, iz, mb_key[ch]);
    const float4 c = tf_lookup(a, s_tf, ch, val, w.scale[ch], w.bias[ch]);
    if (CH == 1) {
      z = Shade{c.w, c.x, c.y, c.z};
    } else {
      z.rho += c.w;
      z.er = fmaf(c.w, c.x, z.er);
      z.eg = fmaf(c.w, c.y, z.eg);
      z.eb = fmaf(c.w, c.z, z.eb);
    }
  }
  if (CH > 1) {
    const float inv_r = z.rho > 0.f ? 1.0f / z.rho : 0.f;
    z.er *= inv_r;
    z.eg *= inv_r;
    z.eb *= inv_r;
  }
  return z;
}

// -log2(e): exp(-x) = 2^(x * kNegLog2e)
constexpr float kNegLog2e = -1.44269504f;

// Over-compositing of one emission-absorption sample at ray parameter tau,
// in transmittance form: the sample's opacity is 1 - exp(-rho s) and its
// weight (1 - A) times that, i.e. T - T exp(-rho s) with T = 1 - A (the same
// recurrence). sc = s * kNegLog2e, so exp(-rho s) = 2^(rho sc). Returns
// whether the ray goes on: false once A >= ert, the early termination
// (the caller clears `alive`; 1 - T then reproduces A exactly). DEPTH false:
// the view asks for no depth, so the depth bookkeeping is left out.
template <bool DEPTH>
__device__ __forceinline__ bool composite_ea(Ray& r, const RenderArgs& a, const Shade& z,
                                             float sc, float tau) {
  const float tn = r.T * __builtin_amdgcn_exp2f(z.rho * sc);
  const float wgt = r.T - tn;
  r.Cr = fmaf(wgt, z.er, r.Cr);
  r.Cg = fmaf(wgt, z.eg, r.Cg);
  r.Cb = fmaf(wgt, z.eb, r.Cb);
  r.T = tn;
  // depth: tau rises along the segment, so the first sample whose alpha
  // reached the threshold has the smallest tau (the depth itself, t0 + tau in FP64,
  // is formed once per segment by finish_depth)
  if (DEPTH) r.dtau = (1.0f - tn >= a.depth_alpha && tau < r.dtau) ? tau : r.dtau;
  // A = 1 - T >= ert, decided on T itself (t_ert: the exact FP32 bound)
  return !(tn <= a.t_ert);
}

// Has the ray terminated early (emission-absorption)? The same test, on the
// same value, as composite_ea's.
__device__ __forceinline__ bool terminated(const Ray& r, const RenderArgs& a) {
  return r.T <= a.t_ert;
}

// Which step a sample_step takes: a full one, the segment's last (partial)
// one, or either, decided per sample.
enum StepKind { kFullStep = 0, kLastStep = 1, kAnyStep = 2 };

// Take sample r.k of the current segment under optical model MODEL (see
// shade_ea for `fetch`). Returns whether the ray goes on (false only when
// an emission-absorption ray terminates; the caller clears `alive`).
template <int MODEL, int CH, bool STATS, bool CLAMP, bool DEPTH, int KIND, typename F>
__device__ __forceinline__ bool sample_step(Ray& r, const RenderArgs& a, const float4* s_tf,
                                            const TfWin<CH>& w, F&& fetch, int (*mb_key)[3]) {
  const int k = r.k;
  const bool last = KIND == kLastStep || (KIND == kAnyStep && k == r.n - 1);
  const float s = last ? r.s_last : r.Df;
  const float tau = last ? r.tau_last : r.tau;  // = sample_tau(r, k)
  if (MODEL != kModelEmission && MODEL != kModelMip) {
    const Shade z = shade_ea<CH, STATS, CLAMP>(r, a, s_tf, w, fetch, tau, mb_key);
    r.k = k + 1;
    // (the loop tests the new index: comparing the old one instead keeps
    // both alive and costs a register copy per sample)
    asm("" : "+v"(r.k));
    r.tau += r.Df;
    if (STATS) ++r.nsamp;
    return composite_ea<DEPTH>(r, a, z, s * kNegLog2e, tau);
  }
  const float qx = fmaf(tau, r.dq[0], r.q0[0]);
  const float qy = fmaf(tau, r.dq[1], r.q0[1]);
  const float qz = fmaf(tau, r.dq[2], r.q0[2]);
  const int ix = CLAMP ? clamp_index(qx, a.Bf) : (int)qx;
  const int iy = CLAMP ? clamp_index(qy, a.Bf) : (int)qy;
  const int iz = CLAMP ? clamp_index(qz, a.Bf) : (int)qz;
  const float fx = __builtin_amdgcn_fractf(qx), fy = __builtin_amdgcn_fractf(qy),
              fz = __builtin_amdgcn_fractf(qz);
  float er = 0.f, eg = 0.f, eb = 0.f;
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) {
    const float val = fetch(ch, ix, iy, iz, fx, fy, fz);
    if (STATS) mark_microblocks(r, a, ch, ix, iy, iz, mb_key[ch]);
    if (MODEL == kModelMip) {
      r.vmax[ch] = fmaxf(r.vmax[ch], val);
      continue;
    }
    const float4 c = tf_lookup(a, s_tf, ch, val, w.scale[ch], w.bias[ch]);
    er += c.x;
    eg += c.y;
    eb += c.z;
  }
  r.k = k + 1;
  r.tau += r.Df;
  if (STATS) ++r.nsamp;
  if (MODEL == kModelMip) {
    r.sampled = true;
    return true;
  }
  // emission only
  r.Cr = fmaf(er, s, r.Cr);
  r.Cg = fmaf(eg, s, r.Cg);
  r.Cb = fmaf(eb, s, r.Cb);
  return true;
}

// Samples r.k .. kb (kb <= n - 1) of the current segment, stopping when the
// ray terminates: the full steps in a loop whose step length does not
// change, then the segment's partial last step if kb is the last sample.
template <int MODEL, int CH, bool STATS, bool CLAMP = true, bool DEPTH = true, typename F>
__device__ __forceinline__ void sample_run(Ray& r, const RenderArgs& a, const float4* s_tf,
                                           F&& fetch, int kb, int (*mb_key)[3]) {
  constexpr bool kEA = MODEL != kModelEmission && MODEL != kModelMip;
  const TfWin<CH> w = tf_win<CH>(a);
  if (CH > 1) {
    // several channels: one loop (a second copy of the larger body costs
    // more registers than the per-sample choice of step saves)
    bool go = r.k <= kb;
    while (go)
      go = sample_step<MODEL, CH, STATS, CLAMP, DEPTH, kAnyStep>(r, a, s_tf, w, fetch, mb_key) &&
           r.k <= kb;
  } else {
    const int kf = min(kb, r.n - 2);
    bool go = r.k <= kf;
    while (go)
      go = sample_step<MODEL, CH, STATS, CLAMP, DEPTH, kFullStep>(r, a, s_tf, w, fetch,
                                                                  mb_key) &&
           r.k <= kf;
    // here r.k <= kb only when r.k = n - 1 = kb
    const bool live = !(kEA && terminated(r, a));
    if (live && r.k <= kb)
      sample_step<MODEL, CH, STATS, CLAMP, DEPTH, kLastStep>(r, a, s_tf, w, fetch, mb_key);
  }
  if (kEA && terminated(r, a)) r.alive = false;
}

// Pool slot pointers of a node, one per channel. Cache volumes stamp the
// slots with the frame number (last use, for eviction) when `stamp_it`.
template <typename T, int CH>
__device__ __forceinline__ void slot_ptrs(const RenderArgs& a, int node, const T* slot[CH],
                                          bool stamp_it) {
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) {
    const int32_t sl = a.page[(int64_t)ch * a.nodes + node];
    slot[ch] = reinterpret_cast<const T*>(a.pool + (int64_t)sl * a.slot_bytes);
    if (stamp_it && a.stamp) a.stamp[sl] = a.frame;
  }
}

template <int MODEL, int CH>
// Returns whether the pixel has content (a nonzero RGBA or, when depth is
// written, a finite depth).
__device__ __forceinline__ bool write_pixel(Ray& r, const RenderArgs& a, const ViewDev& V,
                                            const float4* s_tf, int px, int py) {
  finish_depth(r);
  if (MODEL == kModelMip && r.sampled) {
    // the summed emission of the channel maxima
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
      const float4 c = tf_lookup(a, s_tf, ch, r.vmax[ch]);
      r.Cr += c.x;
      r.Cg += c.y;
      r.Cb += c.z;
    }
  }
  const float omA = r.T;
  const int64_t pix = (int64_t)py * V.W + px;
  float4 out;
  out.x = fmaf(omA, a.bg[0], r.Cr);
  out.y = fmaf(omA, a.bg[1], r.Cg);
  out.z = fmaf(omA, a.bg[2], r.Cb);
  out.w = fmaf(omA, a.bg[3], 1.0f - r.T);
  reinterpret_cast<float4*>(V.rgba)[pix] = out;
  if (V.depth) V.depth[pix] = r.depth;
  return out.x != 0.f || out.y != 0.f || out.z != 0.f || out.w != 0.f ||
         (V.depth != nullptr && r.depth < INFINITY);
}


// Work decomposition. A wave renders a tile of 8x8 pixels. A workgroup
// covers a square screen tile of 2^tile_log wave tiles per side with
// 2^wg_log waves (1 wave for 8x8 pixels, 4 for 16x16 and for 32x32, where
// each wave takes four wave tiles in turn). Workgroup tiles are grouped into
// square blocks of 2^bt_log wave tiles per side (64x64 pixels by default,
// about one brick's footprint at the selected level), and the blocks of all
// views are dealt to the 8 XCDs in turn (workgroup i runs on XCD i % 8,
// each XCD with its own L2): the tiles of a block share one L2 and every
// XCD gets an even share of the image.
//  * direct grid: workgroup i on XCD x = i % 8 takes workgroup tile
//    (i / 8) % (tiles per block) of that XCD's block (i / 8) / (tiles per
//    block);
//  * persistent grid: every wave takes wave tiles one at a time from its
//    XCD's queue (an atomic counter) in the same order, until the XCD's
//    blocks are exhausted.
struct TileLane {
  int view, px, py;
  bool in_image;
  bool tile_valid;
};

// The content byte of the wave's 8x8-pixel tile, when the view asks for the
// mask. Called by the whole wave (converged); nz: the lane's pixel has
// content.
__device__ __forceinline__ void mark_tile(const RenderArgs& a, const TileLane& tl, bool nz) {
  if (!tl.tile_valid) return;  // the same for every lane of the wave
  const ViewDev& V = a.views[tl.view];
  if (!V.tile_any) return;
  const uint64_t m = __ballot(nz);
  if ((threadIdx.x & 63) == 0)  // lane 0 holds the tile's first pixel
    V.tile_any[(int64_t)(tl.py >> 3) * ((V.W + 7) >> 3) + (tl.px >> 3)] = m != 0 ? 1 : 0;
}

// Lane's pixel of wave tile k (row-major) of workgroup tile t in global
// block `block`.
__device__ __forceinline__ TileLane tile_at(const RenderArgs& a, int block, int t, int k,
                                            int lane) {
  TileLane out;
  out.view = 0;
  out.px = out.py = 0;
  out.in_image = false;
  out.tile_valid = block < a.dealt_blocks;
  if (!out.tile_valid) return out;
  int lo = 0, lb;
  if (a.pair_views) {
    // views of one size: the block at one screen position in every view
    const int s = block >> 3;
    lo = s % a.pair_views;
    lb = (block & 7) + 8 * (s / a.pair_views);
    out.tile_valid = lb < a.view_blocks;
    if (!out.tile_valid) return out;
  } else {
    out.tile_valid = block < a.total_blocks;
    if (!out.tile_valid) return out;
    int hi = a.n_views - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.views[mid].block_begin <= block) lo = mid; else hi = mid - 1;
    }
    lb = block - a.views[lo].block_begin;
  }
  const ViewDev& V = a.views[lo];
  const int bx = lb % V.blocks_x, by = lb / V.blocks_x;
  const int per_row_log = a.bt_log - a.tile_log;  // workgroup tiles per block row (log2)
  const int gx = t & ((1 << per_row_log) - 1), gy = t >> per_row_log;
  const int tx = (bx << a.bt_log) + (gx << a.tile_log) + (k & ((1 << a.tile_log) - 1));
  const int ty = (by << a.bt_log) + (gy << a.tile_log) + (k >> a.tile_log);
  out.tile_valid = tx < V.tiles_x && ty < V.tiles_y;
  out.view = lo;
  out.px = tx * 8 + (lane & 7);
  out.py = ty * 8 + (lane >> 3);
  out.in_image = out.tile_valid && out.px < V.W && out.py < V.H;
  return out;
}

// Direct grid: the it-th tile of this wave (it < 4^tile_log / 2^wg_log).
__device__ __forceinline__ TileLane tile_lane(const RenderArgs& a, int it) {
  const int bid = blockIdx.x;
  const int x = bid & 7, j = bid >> 3;
  const int tiles_log = 2 * (a.bt_log - a.tile_log);  // workgroup tiles per block (log2)
  const int block = ((j >> tiles_log) << 3) + x;
  const int t = j & ((1 << tiles_log) - 1);
  const int k = (it << a.wg_log) + (int)(threadIdx.x >> 6);
  return tile_at(a, block, t, k, threadIdx.x & 63);
}

// Persistent grid: the wave's next tile from its XCD's queue; false once the
// XCD's blocks are exhausted (every wave reaches that point: the counter
// only grows). Called with the whole wave active.
__device__ __forceinline__ bool next_tile(const RenderArgs& a, TileLane& tl) {
  const int x = blockIdx.x & 7, lane = threadIdx.x & 63;
  uint32_t item = 0;
  if (lane == 0) item = atomicAdd(a.queue + x, 1u);
  item = (uint32_t)__builtin_amdgcn_readlane((int)item, 0);
  const int per_block_log = 2 * a.bt_log;          // wave tiles per block (log2)
  const int block = (int)((item >> per_block_log) << 3) + x;
  if (block >= a.dealt_blocks) return false;
  const int k = (int)(item & ((1u << per_block_log) - 1));
  const int wt_log = 2 * a.tile_log;               // wave tiles per workgroup tile (log2)
  tl = tile_at(a, block, k >> wt_log, k & ((1 << wt_log) - 1), lane);
  return true;
}

// The workgroup's LDS copy of the transfer tables: per channel and entry
// k < tf_n, t[k] and t[k+1] - t[k] (the device table repeats its last
// entry, so the last difference is zero).
template <int CH>
__device__ __forceinline__ void load_tf(const RenderArgs& a, float4* s_tf) {
  const int ntf = CH * a.tf_n;
  const float4* tf = reinterpret_cast<const float4*>(a.tf);
  for (int i = threadIdx.x; i < ntf; i += blockDim.x) {
    const int ch = i / a.tf_n, k = i - ch * a.tf_n;
    const float4 t0 = tf[ch * (a.tf_n + 1) + k], t1 = tf[ch * (a.tf_n + 1) + k + 1];
    s_tf[2 * i] = t0;
    s_tf[2 * i + 1] = make_float4(t1.x - t0.x, t1.y - t0.y, t1.z - t0.z, t1.w - t0.w);
  }
  __syncthreads();
}

// ------------------------------------------------------------ gather kernel
// The pool stencil of one sample: its eight voxels and fractions, loaded
// ahead of their use (the same index, clamp and fraction arithmetic as
// shade_ea's read of the pool; MB: micro-block slots).
struct Stencil {
  uint32_t v[8];
  float fx, fy, fz;
};
template <typename T, bool MB>
__device__ __forceinline__ Stencil stencil_at(const Ray& r, const RenderArgs& a, const T* slot,
                                              float tau) {
  const float qx = fmaf(tau, r.dq[0], r.q0[0]);
  const float qy = fmaf(tau, r.dq[1], r.q0[1]);
  const float qz = fmaf(tau, r.dq[2], r.q0[2]);
  const int ix = clamp_index(qx, a.Bf);
  const int iy = clamp_index(qy, a.Bf);
  const int iz = clamp_index(qz, a.Bf);
  Stencil st;
  st.fx = __builtin_amdgcn_fractf(qx);
  st.fy = __builtin_amdgcn_fractf(qy);
  st.fz = __builtin_amdgcn_fractf(qz);
  if (MB) {
    const T* p0 = slot + mb_index(ix, iy, iz, a.M);
    const MbSteps d = mb_steps(ix, iy, iz, a.M);
    st.v[0] = p0[0];
    st.v[1] = p0[d.dx];
    st.v[2] = p0[d.dy];
    st.v[3] = p0[d.dy + d.dx];
    st.v[4] = p0[d.dz];
    st.v[5] = p0[d.dz + d.dx];
    st.v[6] = p0[d.dz + d.dy];
    st.v[7] = p0[d.dz + d.dy + d.dx];
    return st;
  }
  // (an unsigned 32-bit element offset from 24-bit products: stored
  // indices and edges are below 2^9)
  const T* p0 = slot + (uint32_t)(__umul24(__umul24(iz, a.S) + iy, a.Sx) + ix);
  const int sy = a.Sx, sz = a.S * a.Sx;
  st.v[0] = p0[0];
  st.v[1] = p0[1];
  st.v[2] = p0[sy];
  st.v[3] = p0[sy + 1];
  st.v[4] = p0[sz];
  st.v[5] = p0[sz + 1];
  st.v[6] = p0[sz + sy];
  st.v[7] = p0[sz + sy + 1];
  return st;
}
// Its trilinear value: trilinear's operations in trilinear's order.
__device__ __forceinline__ float stencil_value(const Stencil& st) {
  const float c00 = lerpf((float)st.v[0], (float)st.v[1], st.fx);
  const float c10 = lerpf((float)st.v[2], (float)st.v[3], st.fx);
  const float c01 = lerpf((float)st.v[4], (float)st.v[5], st.fx);
  const float c11 = lerpf((float)st.v[6], (float)st.v[7], st.fx);
  const float c0 = lerpf(c00, c10, st.fy);
  const float c1 = lerpf(c01, c11, st.fy);
  return lerpf(c0, c1, st.fz);
}
// A full step of one channel (emission-absorption) from its table entry c:
// sample_step's full step after the lookup.
template <bool DEPTH>
__device__ __forceinline__ bool shade_step(Ray& r, const RenderArgs& a, const float4& c) {
  const float tau = r.tau;
  r.k += 1;
  r.tau += r.Df;
  return composite_ea<DEPTH>(r, a, Shade{c.w, c.x, c.y, c.z}, r.Df * kNegLog2e, tau);
}

// The gather kernel's samples of the current segment for one channel under
// emission-absorption: sample_run's samples, two full steps per iteration,
// with the stencils of the next two loaded while the current two are
// shaded, so that a ray waits for memory about once per two samples (the
// rays of a sparse frame are few, and a frame then lasts as long as its
// longest chain of dependent samples). The loads are issued at the top of
// the loop body and pinned there, and the loop-carried stencils copied at
// its end (no instruction moves across the scheduling barriers); a stencil
// past the last full step repeats the last full step's instead of reading
// the partial step's.
template <typename T, bool DEPTH, bool MB, typename F>
__device__ __forceinline__ void gather_run(Ray& r, const RenderArgs& a, const float4* s_tf,
                                           const T* slot, F&& fetch, int (*mb_key)[3]) {
  const TfWin<1> w = tf_win<1>(a);
  const int kb = r.n - 1, kf = r.n - 2;
  if (r.k <= kf) {
    Stencil c0 = stencil_at<T, MB>(r, a, slot, r.tau);
    Stencil c1 = stencil_at<T, MB>(r, a, slot, r.k < kf ? r.tau + r.Df : r.tau);
    bool go = true;
    while (go) {
      const float t1 = r.k < kf ? r.tau + r.Df : r.tau;
      const float t2 = r.k + 1 < kf ? t1 + r.Df : t1;
      const float t3 = r.k + 2 < kf ? t2 + r.Df : t2;
      const Stencil n0 = stencil_at<T, MB>(r, a, slot, t2);
      const Stencil n1 = stencil_at<T, MB>(r, a, slot, t3);
      __builtin_amdgcn_sched_barrier(0);
      const float4 e0 = tf_lookup(a, s_tf, 0, stencil_value(c0), w.scale[0], w.bias[0]);
      const float4 e1 = tf_lookup(a, s_tf, 0, stencil_value(c1), w.scale[0], w.bias[0]);
      go = shade_step<DEPTH>(r, a, e0) && r.k <= kf;
      if (go) go = shade_step<DEPTH>(r, a, e1) && r.k <= kf;
      __builtin_amdgcn_sched_barrier(0);
      c0 = n0;
      c1 = n1;
    }
  }
  if (!terminated(r, a) && r.k <= kb)
    sample_step<kModelAbsorption, 1, false, true, DEPTH, kLastStep>(r, a, s_tf, w, fetch, mb_key);
  if (terminated(r, a)) r.alive = false;
}

template <typename T, int CH, bool STATS, int MODEL, bool MB>
__device__ __forceinline__ bool gather_pixel(const RenderArgs& a, const float4* s_tf,
                                             const TileLane& tl) {
  // the view is the same for every lane of the wave (one 8x8 tile)
  const ViewDev& V = a.views[__builtin_amdgcn_readfirstlane(tl.view)];
  const bool depth_on = __builtin_amdgcn_readfirstlane(V.depth ? 1 : 0) != 0;
  int mb_key[CH][3];
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) mb_key[ch][0] = mb_key[ch][1] = mb_key[ch][2] = -1;
  Ray r;
  ray_setup(r, a, V, tl.px, tl.py);
  if (r.alive) next_segment<MODEL, CH>(r, a, V, true);
  while (r.alive) {
    const T* slot[CH];
    slot_ptrs<T, CH>(a, r.node, slot, true);
    if (STATS) atomicAdd((unsigned long long*)a.counters + 1, 1ull);
    auto fetch = [&](int ch, int ix, int iy, int iz, float fx, float fy, float fz) {
      return pool_trilinear<MB>(a, slot[ch], ix, iy, iz, fx, fy, fz);
    };
    if (CH == 1 && !STATS && MODEL == kModelAbsorption) {
      if (depth_on)
        gather_run<T, true, MB>(r, a, s_tf, slot[0], fetch, mb_key);
      else
        gather_run<T, false, MB>(r, a, s_tf, slot[0], fetch, mb_key);
    } else if (depth_on) {
      sample_run<MODEL, CH, STATS, true, true>(r, a, s_tf, fetch, r.n - 1, mb_key);
    } else {
      sample_run<MODEL, CH, STATS, true, false>(r, a, s_tf, fetch, r.n - 1, mb_key);
    }
    if (!r.alive) break;
    next_segment<MODEL, CH>(r, a, V, false);
  }
  const bool nz = write_pixel<MODEL, CH>(r, a, V, s_tf, tl.px, tl.py);
  if (STATS) {
    if (V.nsamp) V.nsamp[(int64_t)tl.py * V.W + tl.px] = r.nsamp;
    atomicAdd((unsigned long long*)a.counters, (unsigned long long)r.nsamp);
  }
  return nz;
}

// LOOP: the wave renders several tiles (persistent grid, or a direct grid
// with more wave tiles than waves per workgroup); without it exactly one.
// The two are separate instances because the loop costs registers.
template <typename T, int CH, bool STATS, int MODEL, bool LOOP, bool MB>
__global__ __launch_bounds__(256) void raycast_gather(RenderArgs a) {
  if (a.enable && *a.enable == 0) return;  // whole grid: before any barrier
  extern __shared__ float4 s_tf[];
  load_tf<CH>(a, s_tf);
  if (!LOOP) {
    const TileLane tl = tile_lane(a, 0);
    bool nz = false;
    if (tl.in_image) nz = gather_pixel<T, CH, STATS, MODEL, MB>(a, s_tf, tl);
    mark_tile(a, tl, nz);
  } else if (a.persistent) {
    TileLane tl;
    while (next_tile(a, tl)) {
      bool nz = false;
      if (tl.in_image) nz = gather_pixel<T, CH, STATS, MODEL, MB>(a, s_tf, tl);
      mark_tile(a, tl, nz);
    }
  } else {
    for (int it = 0; it < a.wave_tiles; ++it) {
      const TileLane tl = tile_lane(a, it);
      bool nz = false;
      if (tl.in_image) nz = gather_pixel<T, CH, STATS, MODEL, MB>(a, s_tf, tl);
      mark_tile(a, tl, nz);
    }
  }
}

// ------------------------------------------------------------ staged kernel
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave reductions without LDS traffic: within each 16-lane row, DPP lane
// swaps (quad_perm xor 1, quad_perm xor 2, half-row mirror, row mirror)
// leave the row's result in every lane; the four row results are then read
// as scalars. Every lane of the wave must be active at the call: each
// swap's source lane is then active, so the move has no fallback value to
// keep (and no register copy to make for one).
template <int C>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, C, 0xF, 0xF, false);
}
template <typename Op>
__device__ __forceinline__ int wave_reduce_i(int v, Op op) {
  v = op(v, dpp_i<0xB1>(v));
  v = op(v, dpp_i<0x4E>(v));
  v = op(v, dpp_i<0x141>(v));
  v = op(v, dpp_i<0x140>(v));
  const int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  const int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  return op(op(a, b), op(c, d));
}
__device__ __forceinline__ int wave_min_i(int v) {
  return wave_reduce_i(v, [](int x, int y) { return min(x, y); });
}
__device__ __forceinline__ int wave_max_i(int v) {
  return wave_reduce_i(v, [](int x, int y) { return max(x, y); });
}
template <int C>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const int lo = dpp_i<C>((int)(uint32_t)v), hi = dpp_i<C>((int)(uint32_t)(v >> 32));
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t rl_u64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  v = umin64(v, dpp_u64<0xB1>(v));
  v = umin64(v, dpp_u64<0x4E>(v));
  v = umin64(v, dpp_u64<0x141>(v));
  v = umin64(v, dpp_u64<0x140>(v));
  return umin64(umin64(rl_u64(v, 0), rl_u64(v, 16)), umin64(rl_u64(v, 32), rl_u64(v, 48)));
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float lane_f(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Component-wise minimum of the two 16-bit halves of a word, over the wave,
// for two words at once (the steps interleaved, so no move waits on the
// previous step's result); the four row results of each are combined in
// scalar registers.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t min_u16x2(uint32_t x, uint32_t y) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, x),
                                                                 __builtin_bit_cast(u16x2, y)));
}
__device__ __forceinline__ uint32_t rows_min_u16x2(uint32_t v) {
  const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
  const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
  const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
  const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
  uint32_t l0 = min(a & 0xFFFFu, b & 0xFFFFu), l1 = min(c & 0xFFFFu, d & 0xFFFFu);
  uint32_t h0 = min(a >> 16, b >> 16), h1 = min(c >> 16, d >> 16);
  // (kept in scalar registers: a three-way vector minimum would need moves)
  asm volatile("" : "+s"(l0), "+s"(l1), "+s"(h0), "+s"(h1));
  return min(l0, l1) | (min(h0, h1) << 16);
}
__device__ __forceinline__ void wave_min_u16x2_pair(uint32_t& v, uint32_t& w) {
  v = min_u16x2(v, (uint32_t)dpp_i<0xB1>((int)v));
  w = min_u16x2(w, (uint32_t)dpp_i<0xB1>((int)w));
  v = min_u16x2(v, (uint32_t)dpp_i<0x4E>((int)v));
  w = min_u16x2(w, (uint32_t)dpp_i<0x4E>((int)w));
  v = min_u16x2(v, (uint32_t)dpp_i<0x141>((int)v));
  w = min_u16x2(w, (uint32_t)dpp_i<0x141>((int)w));
  v = min_u16x2(v, (uint32_t)dpp_i<0x140>((int)v));
  w = min_u16x2(w, (uint32_t)dpp_i<0x140>((int)w));
  v = rows_min_u16x2(v);
  w = rows_min_u16x2(w);
}

// floor(x / d) for 0 <= x < 2^21, 1 <= d, from a reciprocal: within one of
// the exact quotient (used only where any nearby value serves).
__device__ __forceinline__ int quot(int x, int d) {
  return (int)(((float)x + 0.5f) * __builtin_amdgcn_rcpf((float)d));
}

// Main-axis stencil layer of sample k (same arithmetic as the sample),
// clamped to [0, B] (bf = B).
__device__ __forceinline__ int sample_layer(const Ray& r, int k, float dqm, float qm0, float bf) {
  return clamp_index(fmaf(sample_tau(r, k), dqm, qm0), bf);
}

// Stencil corner bounds (per axis; the stencil also reads corner + 1) of
// samples ka and kb of the lane's segment, hence of every sample between.
__device__ __forceinline__ void stencil_bounds(const Ray& r, int ka, int kb, float bf, int lo[3],
                                               int hi[3]) {
  const float ta = sample_tau(r, ka), tb = sample_tau(r, kb);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int ia = clamp_index(fmaf(ta, r.dq[i], r.q0[i]), bf);
    const int ib = clamp_index(fmaf(tb, r.dq[i], r.q0[i]), bf);
    lo[i] = min(ia, ib);
    hi[i] = max(ia, ib);
  }
}

__device__ __forceinline__ float pick(const float v[3], int m) {
  return m == 0 ? v[0] : (m == 1 ? v[1] : v[2]);
}
__device__ __forceinline__ int pick(const int v[3], int m) {
  return m == 0 ? v[0] : (m == 1 ? v[1] : v[2]);
}

// Statistics of one sample loop of the staged kernel (called by the whole
// wave; taken = the samples this lane took in it): wave iterations (the
// largest count) and, for loops that read the pool, the samples.
__device__ __forceinline__ void stat_loop(const RenderArgs& a, int taken, bool pool) {
  const int it = wave_max_i(taken);
  if ((threadIdx.x & 63) == 0 && it > 0)
    atomicAdd((unsigned long long*)a.counters + 5, (unsigned long long)it);
  if (pool && taken > 0) atomicAdd((unsigned long long*)a.counters + 6, (unsigned long long)taken);
}

// One wave tile of the staged kernel (the whole wave active).
template <typename T, int CH, bool STATS, int MODEL, bool MB>
__device__ __forceinline__ void staged_tile(const RenderArgs& a, const float4* s_tf, T* stage,
                                            const TileLane& tl) {
  const int lane = threadIdx.x & 63;
  // staging moves chunks of kRowAlignBytes (pool rows are aligned to
  // them); the capacity per channel is a whole number of chunks so every
  // channel's region starts chunk-aligned in LDS
  constexpr int align = kRowAlignBytes / (int)sizeof(T);  // voxels per chunk
  const int cap = (a.stage_bytes / (int)sizeof(T) / CH) & ~(align - 1);
  const ViewDev& V = a.views[uniform(tl.view)];  // one view per wave
  int mb_key[CH][3];
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) mb_key[ch][0] = mb_key[ch][1] = mb_key[ch][2] = -1;
  Ray r;
  r.alive = false;
  r.Cr = r.Cg = r.Cb = 0.f;
  r.T = 1.f;
  r.depth = INFINITY;
  r.dtau = INFINITY;
  r.nsamp = 0;
  r.n = r.k = 0;
  if (tl.in_image) {
    ray_setup(r, a, V, tl.px, tl.py);
    if (r.alive) next_segment<MODEL, CH>(r, a, V, true);
  }
  const int B = a.B, S = a.S, Sx = a.Sx;
  // the wave's rays belong to one view: its depth request is wave-uniform
  const bool depth_on = uniform(V.depth ? 1 : 0) != 0;

  while (true) {
    // --- the wave's next node: smallest front-to-back key among its rays
    const uint64_t K = wave_min_u64(r.alive ? r.key : ~0ull);
    if (K == ~0ull) break;
    const bool mine = r.alive && r.key == K;
    const uint64_t mask = __ballot(mine);
    const int first = __ffsll((unsigned long long)mask) - 1;
    const int node = uniform(__builtin_amdgcn_readlane(r.node, first));
    const T* slot[CH];
    slot_ptrs<T, CH>(a, node, slot, lane == 0);
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {  // the same for every lane: scalar registers
      const uint64_t p = reinterpret_cast<uint64_t>(slot[ch]);
      slot[ch] = reinterpret_cast<const T*>(
          (uint64_t)(uint32_t)uniform((int)(uint32_t)p) |
          ((uint64_t)(uint32_t)uniform((int)(uint32_t)(p >> 32)) << 32));
    }
    if (STATS) {
      const uint64_t alive = __ballot(r.alive);
      if (lane == 0) {
        atomicAdd((unsigned long long*)a.counters + 1, 1ull);
        atomicAdd((unsigned long long*)a.counters + 4, (unsigned long long)__popcll(mask));
        atomicAdd((unsigned long long*)a.counters + 8, (unsigned long long)__popcll(alive));
      }
    }

    // --- dominant axis of the node's first ray; every ray of the node must
    // advance along it with the same sign, else everything reads the pool
    const float d0[3] = {lane_f(r.dq[0], first), lane_f(r.dq[1], first),
                         lane_f(r.dq[2], first)};
    int m = 0;
    if (fabsf(d0[1]) > fabsf(d0[0])) m = 1;
    if (fabsf(d0[2]) > fabsf(pick(d0, m))) m = 2;
    m = uniform(m);
    const int sgn = uniform(pick(d0, m) > 0.f ? 1 : -1);
    const float my_dqm = pick(r.dq, m);
    const float my_qm0 = pick(r.q0, m);
    const float my_sum = fabsf(r.dq[0]) + fabsf(r.dq[1]) + fabsf(r.dq[2]);
    const bool bad = mine && !((float)sgn * my_dqm >= 0.25f * my_sum);
    const bool axis_ok = __ballot(bad) == 0;
    // samples r.k .. kb of this lane read from the pool (a sample loop per
    // slot layout: one loop choosing per sample would hold the registers of
    // both address forms)
    auto pool_run = [&](int kb) {
      if (MB) {
        auto fetch = [&](int ch, int ix, int iy, int iz, float fx, float fy, float fz) {
          return trilinear_mb<T, true>(slot[ch], ix, iy, iz, a.M, fx, fy, fz);
        };
        if (depth_on)
          sample_run<MODEL, CH, STATS, true, true>(r, a, s_tf, fetch, kb, mb_key);
        else
          sample_run<MODEL, CH, STATS, true, false>(r, a, s_tf, fetch, kb, mb_key);
      } else {
        auto fetch = [&](int ch, int ix, int iy, int iz, float fx, float fy, float fz) {
          return trilinear(slot[ch] + (iz * S + iy) * Sx + ix, Sx, S * Sx, fx, fy, fz);
        };
        if (depth_on)
          sample_run<MODEL, CH, STATS, true, true>(r, a, s_tf, fetch, kb, mb_key);
        else
          sample_run<MODEL, CH, STATS, true, false>(r, a, s_tf, fetch, kb, mb_key);
      }
    };

    // --- slabs along the main axis, in the rays' direction of travel. The
    // first slab starts at the first stencil layer any ray needs; each owns
    // D layers and stages them plus the one the stencils reach into. Every
    // lane takes exactly its samples whose layer lies in the slab, so the
    // next slab starts right after it.
    const int big = 0xFFFF;
    const bool more0 = mine && r.alive && r.k < r.n;
    int j;
    {
      const int my_im = more0 ? sample_layer(r, r.k, my_dqm, my_qm0, a.Bf) : (sgn > 0 ? big : -1);
      j = uniform(sgn > 0 ? wave_min_i(my_im) : wave_max_i(my_im));
    }
    int D = 8;
    while (true) {
      const bool more = mine && r.alive && r.k < r.n;
      if (__ballot(more) == 0) break;
      if (!axis_ok || (sgn > 0 ? j > B : j < 0)) {
        // no shared dominant direction (or, defensively, nothing left in
        // range): read the pool for all remaining samples
        const int k_before = r.k;
        if (more) pool_run(r.n - 1);
        if (STATS) stat_loop(a, r.k - k_before, true);
        continue;
      }
      int jl = j, jh = j, kb = r.k - 1;
      int o[3] = {0, 0, 0}, wd[3] = {0, 0, 0};
      bool fits = false;
      int ntries = 0;
      for (int tries = 0; tries < 8; ++tries) {
        ++ntries;
        jl = sgn > 0 ? j : max(j - D + 1, 0);
        jh = sgn > 0 ? min(j + D - 1, B) : j;
        // this lane's samples in the slab: k .. kb, found exactly
        kb = r.k - 1;
        uint32_t plo = 0xFFFFFFFFu, phi = 0xFFFFFFFFu;  // packed min(lo), min(~hi)
        if (more) {
          // a first guess of the last sample in the slab (reciprocals, not
          // divisions: the two searches below make it exact)
          const float edge = sgn > 0 ? (float)(jh + 1) : (float)jl;
          const float tlim = (edge - my_qm0) * __builtin_amdgcn_rcpf(my_dqm);
          kb = (int)ceilf(tlim * __builtin_amdgcn_rcpf(r.Df) - 0.5f) - 1;
          kb = min(max(kb, r.k - 1), r.n - 1);
          while (kb + 1 < r.n) {
            const int im = sample_layer(r, kb + 1, my_dqm, my_qm0, a.Bf);
            if (im < jl || im > jh) break;
            ++kb;
          }
          while (kb >= r.k) {
            const int im = sample_layer(r, kb, my_dqm, my_qm0, a.Bf);
            if (im >= jl && im <= jh) break;
            --kb;
          }
          if (kb >= r.k) {
            int lo3[3], hi3[3];
            stencil_bounds(r, r.k, kb, a.Bf, lo3, hi3);
            const int ua = m == 0 ? 1 : 0, ub = m == 2 ? 1 : 2;  // cross axes
            plo = (uint32_t)pick(lo3, ua) | ((uint32_t)pick(lo3, ub) << 16);
            phi = (uint32_t)(0xFFFF - pick(hi3, ua)) | ((uint32_t)(0xFFFF - pick(hi3, ub)) << 16);
          }
        }
        wave_min_u16x2_pair(plo, phi);
        const int la = (int)(plo & 0xFFFF), lb = (int)(plo >> 16);
        const int ha = 0xFFFF - (int)(phi & 0xFFFF), hb = 0xFFFF - (int)(phi >> 16);
        const int ua = m == 0 ? 1 : 0, ub = m == 2 ? 1 : 2;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          if (i == m) {
            o[i] = jl;
            wd[i] = jh - jl + 2;
          } else {
            const int l = i == ua ? la : lb, h = i == ua ? ha : hb;
            const int e = h - l;  // no lane has samples: l = 0xFFFF, h = 0, e < 0
            o[i] = e >= 0 ? l : 0;
            wd[i] = e >= 0 ? e + 2 : 0;
          }
        }
        // chunk-aligned rows: x origin rounded down, width rounded up
        const int ox = (o[0] / align) * align;
        wd[0] = ((o[0] + wd[0] - ox + align - 1) / align) * align;
        o[0] = ox;
        wd[0] = min(wd[0], Sx - o[0]);
        wd[1] = min(wd[1], S - o[1]);
        wd[2] = min(wd[2], S - o[2]);
        const int vox = wd[0] * wd[1] * wd[2];
        // (the depth only shapes the slabs, never which samples they hold,
        // so its quotients are taken with reciprocals)
        const int area = uniform(max(1, quot(vox, max(1, wd[m]))));
        if (vox <= cap) {
          fits = vox > 0;
          // next slab's depth from this slab's cross-section, with part of
          // it in reserve: cross-sections grow along the rays, and a slab
          // that does not fit costs a second search. One channel keeps 1/4
          // (with the staging copy at one vector instruction per load the
          // search weighs more than the extra slabs: 3/4 ran 1.2% faster
          // than 7/8, 15/16 1% slower, 2/3 and 5/8 no better); several
          // channels copy a region each per slab and keep 1/8 (3/4 ran 2%
          // slower there)
          const int keep = CH == 1 ? quot(cap * 3, area * 4) : quot(cap * 7, area * 8);
          D = uniform(min(max(keep - 1, 1), 64));
          break;
        }
        if (D == 1) break;
        // the cross-section of a thinner slab is no larger (its samples are
        // a subset), so this depth fits unless even one layer does not
        D = uniform(max(1, min(D - 1, quot(cap, area) - 1)));
      }
      if (STATS && lane == 0 && ntries > 1)
        atomicAdd((unsigned long long*)a.counters + 7, (unsigned long long)(ntries - 1));
      const int k_slab = r.k;
#pragma unroll
      for (int i = 0; i < 3; ++i) {  // the same for every lane: scalar registers
        o[i] = uniform(o[i]);
        wd[i] = uniform(wd[i]);
      }
      if (fits) {
        // --- stage the region of every channel straight from the pool into
        // LDS (global_load_lds: lane i of an instruction writes chunk i after
        // the instruction's LDS base). The region is wd[1] * wd[2] rows of
        // cpr chunks, row-major in LDS. The quotients below come from
        // (x + 1/2) * rcp(d) in FP32: rcp is within one ulp, so the product's
        // relative error is below 2^-22, and (x + 1/2) / d lies at least
        // 1/(2d) from an integer, so the floor is exact for every x < 2^21
        // (here x < 2^15: the region holds at most the staging capacity).
        const int cpr = wd[0] / align, P = Sx / align;
        const int wy = wd[1], rows = wd[1] * wd[2];
        const int total = cpr * rows;
        const float inv_cpr = __builtin_amdgcn_rcpf((float)cpr),
                    inv_wy = __builtin_amdgcn_rcpf((float)wy);
        constexpr int cb = kRowAlignBytes;
        if (cpr * wy <= 32) {
          // planes of at most 32 chunks: a pass moves k = 64 / Q whole
          // planes, lane pz * Q + i taking chunk i of plane pz of the pass
          // (row i / cpr, column i % cpr; lanes past k * Q rest). A lane's
          // offset in the slot is the part from its (x, y), kept, plus the
          // part from its plane, formed at each pass
          constexpr int vb = (int)sizeof(T), zin = 16 * vb;
          const int Q = cpr * wy;
          const float inv_q = __builtin_amdgcn_rcpf((float)Q);
          const int k = uniform((int)(64.5f * inv_q));
          const int zs = MB ? 64 * a.M * a.M * vb : S * Sx * vb, nz = wd[2];
          const int pz = (int)(((float)lane + 0.5f) * inv_q), i = lane - pz * Q;
          if (pz < k) {
            const int ry = (int)(((float)i + 0.5f) * inv_cpr);
            const int x = o[0] + (i - ry * cpr) * align, y = o[1] + ry;
            const uint32_t c =
                MB ? (uint32_t)((((x >> 2) + (y >> 2) * a.M) << 6) + ((y & 3) << 2) + (x & 3)) * vb
                   : (uint32_t)((y * Sx + x) * vb);
            for (int t = 0; t < nz; t += k) {
              if (t + pz < nz) {
                const int z = o[2] + t + pz;
                const uint32_t hz =
                    MB ? (uint32_t)(__umul24(z >> 2, zs) + (z & 3) * zin) : (uint32_t)__umul24(z, zs);
#pragma unroll
                for (int ch = 0; ch < CH; ++ch)
                  __builtin_amdgcn_global_load_lds(
                      reinterpret_cast<const uint8_t*>(slot[ch]) + hz + c,
                      reinterpret_cast<uint8_t*>(stage + ch * cap) + t * Q * cb, cb, 0, 0);
              }
            }
          }
        } else if (cpr <= 64) {
          // a lane keeps chunk i = s0 + lane of a region plane (row i / cpr,
          // column i % cpr) and a sub-pass walks the planes. A chunk's
          // offset in the slot is the sum of a part from its (x, y) and a
          // part from its plane z, the same for every lane and kept in
          // scalar registers: no per-lane work per load. In a micro-block
          // slot the chunk (two u16 or four u8 voxels from an even x) lies
          // in one block row, and the plane part steps by a block plane
          // every fourth plane.
          constexpr int vb = (int)sizeof(T), zin = 16 * vb;
          const int Q = cpr * wy;  // chunks per plane
          const int zs = MB ? 64 * a.M * a.M * vb : S * Sx * vb, zjump = zs - 3 * zin;
          const int nz = wd[2];
          const int h0 = MB ? (o[2] >> 2) * zs + (o[2] & 3) * zin : o[2] * zs;
          for (int s0 = 0; s0 < Q; s0 += 64) {
            const int i = s0 + lane;
            if (i < Q) {
              const int ry = (int)(((float)i + 0.5f) * inv_cpr);
              const int x = o[0] + (i - ry * cpr) * align, y = o[1] + ry;
              const uint32_t c =
                  MB ? (uint32_t)((((x >> 2) + (y >> 2) * a.M) << 6) + ((y & 3) << 2) + (x & 3)) * vb
                     : (uint32_t)((y * Sx + x) * vb);
              // the plane part's steps after planes o[2] + 4u + j: a block
              // plane after every fourth plane of a micro-block slot
              uint32_t st[4];
#pragma unroll
              for (int j = 0; j < 4; ++j)
                st[j] = (uint32_t)(MB ? (((o[2] + j) & 3) == 3 ? zjump : zin) : zs);
              uint32_t hz = (uint32_t)h0;
              auto load_plane = [&](int t) {
#pragma unroll
                for (int ch = 0; ch < CH; ++ch)
                  __builtin_amdgcn_global_load_lds(
                      reinterpret_cast<const uint8_t*>(slot[ch]) + hz + c,
                      reinterpret_cast<uint8_t*>(stage + ch * cap) + (t * Q + s0) * cb, cb, 0, 0);
              };
              int t = 0;
              for (; t + 4 <= nz; t += 4) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  load_plane(t + j);
                  hz += st[j];
                }
              }
              if (t < nz) {  // the last nz % 4 planes
                load_plane(t);
                hz += st[0];
                if (t + 1 < nz) {
                  load_plane(t + 1);
                  hz += st[1];
                  if (t + 2 < nz) load_plane(t + 2);
                }
              }
            }
          }
        } else {
          // rows wider than a pass (bricks of 128 or more): pass p moves
          // chunks p .. p+63 of the region; chunk i is row = i / cpr, plane
          // rz = row / wy, at base + i + row * skip_row + rz * skip_plane
          if (STATS && lane == 0) atomicAdd((unsigned long long*)a.counters + 9, 1ull);
          const int base = ((o[2] * S + o[1]) * Sx + o[0]) / align;
          const int skip_row = P - cpr, skip_plane = (S - wy) * P;
          for (int p0 = 0; p0 < total; p0 += 64) {
            const int i = p0 + lane;
            if (i < total) {
              const int row = (int)(((float)i + 0.5f) * inv_cpr);
              const int rz = (int)(((float)row + 0.5f) * inv_wy);
              // byte offset in the slot: chunk g of a linear slot, or the
              // chunk's first voxel in a micro-block slot
              const size_t off =
                  MB ? (size_t)mb_index(o[0] + (i - row * cpr) * align, o[1] + row - rz * wy,
                                         o[2] + rz, a.M) * sizeof(T)
                      : (size_t)(base + i + __mul24(row, skip_row) + __mul24(rz, skip_plane)) * cb;
#pragma unroll
              for (int ch = 0; ch < CH; ++ch)
                __builtin_amdgcn_global_load_lds(
                    reinterpret_cast<const uint8_t*>(slot[ch]) + off,
                    reinterpret_cast<uint8_t*>(stage + ch * cap) + p0 * cb, cb, 0, 0);
            }
          }
        }
        __builtin_amdgcn_s_waitcnt(0);  // the LDS writes of the loads have landed
        wave_sync();
        if (STATS && lane == 0) {
          atomicAdd((unsigned long long*)a.counters + 2, 1ull);
          atomicAdd((unsigned long long*)a.counters + 3,
                    (unsigned long long)(total * kRowAlignBytes * CH));
        }
        if (kb >= r.k) {
          const int sy_l = wd[0], wy = wd[1];
          const int base_off = (o[2] * wd[1] + o[1]) * wd[0] + o[0];  // region origin
          // byte addresses: the region's origin, and the row and plane steps
          const char* sb = reinterpret_cast<const char*>(stage - base_off);
          const int syb = sy_l * (int)sizeof(T), szb = sy_l * wy * (int)sizeof(T);
          auto fetch = [&](int ch, int ix, int iy, int iz, float fx, float fy, float fz) {
            // stencil corner: x step, then the row and plane steps as 24-bit
            // multiply-adds (every term below 2^23; written out, since the
            // compiler would form two products and a three-way add)
            typedef __attribute__((address_space(3))) const char* LdsP;
            uint32_t q = (uint32_t)(uintptr_t)(LdsP)(sb + ch * cap * (int)sizeof(T)) +
                         (uint32_t)(ix * (int)sizeof(T));
            asm("v_mad_u32_u24 %0, %1, %2, %0" : "+v"(q) : "v"(iy), "s"(syb));
            asm("v_mad_u32_u24 %0, %1, %2, %0" : "+v"(q) : "v"(iz), "s"(szb));
            return trilinear_bytes<T>((const char*)(LdsP)(uintptr_t)q, syb, szb, fx, fy, fz);
          };
          if (depth_on)
            sample_run<MODEL, CH, STATS, false, true>(r, a, s_tf, fetch, kb, mb_key);
          else
            sample_run<MODEL, CH, STATS, false, false>(r, a, s_tf, fetch, kb, mb_key);
        }
        if (STATS) stat_loop(a, r.k - k_slab, false);
        wave_sync();
      } else {
        if (kb >= r.k) {
          // the slab does not fit even one layer deep: read the pool for it
          pool_run(kb);
        }
        if (STATS) stat_loop(a, r.k - k_slab, true);
      }
      j = sgn > 0 ? jh + 1 : jl - 1;
    }
    // --- rays that finished this node move on to their next segment
    if (mine && r.alive) next_segment<MODEL, CH>(r, a, V, false);
  }
  bool nz = false;
  if (tl.in_image) {
    nz = write_pixel<MODEL, CH>(r, a, V, s_tf, tl.px, tl.py);
    if (STATS) {
      if (V.nsamp) V.nsamp[(int64_t)tl.py * V.W + tl.px] = r.nsamp;
      atomicAdd((unsigned long long*)a.counters, (unsigned long long)r.nsamp);
    }
  }
  mark_tile(a, tl, nz);
}

template <typename T, int CH, bool STATS, int MODEL, bool LOOP, bool MB>
__global__ __launch_bounds__(256) void raycast_staged(RenderArgs a) {
  if (a.enable && *a.enable == 0) return;  // whole grid: before any barrier
  extern __shared__ float4 smem[];
  float4* s_tf = smem;
  load_tf<CH>(a, s_tf);
  // the wave's staging space (the wave index is the same for all its lanes:
  // scalar registers)
  T* stage = reinterpret_cast<T*>(reinterpret_cast<uint8_t*>(smem + 2 * CH * a.tf_n) +
                                  uniform((int)(threadIdx.x >> 6)) * a.stage_bytes);
  // no workgroup barrier follows: the waves work independently from here
  if (!LOOP) {
    const TileLane tl = tile_lane(a, 0);
    if (tl.tile_valid) staged_tile<T, CH, STATS, MODEL, MB>(a, s_tf, stage, tl);
  } else if (a.persistent) {
    TileLane tl;
    while (next_tile(a, tl))
      if (tl.tile_valid) staged_tile<T, CH, STATS, MODEL, MB>(a, s_tf, stage, tl);
  } else {
    for (int it = 0; it < a.wave_tiles; ++it) {
      const TileLane tl = tile_lane(a, it);
      if (tl.tile_valid) staged_tile<T, CH, STATS, MODEL, MB>(a, s_tf, stage, tl);
    }
  }
}

template <typename T, int CH, int MODEL, bool LOOP, bool MB>
const void* kernel_for(bool stats, bool gather) {
  if (gather)
    return stats ? reinterpret_cast<const void*>(raycast_gather<T, CH, true, MODEL, LOOP, MB>)
                 : reinterpret_cast<const void*>(raycast_gather<T, CH, false, MODEL, LOOP, MB>);
  return stats ? reinterpret_cast<const void*>(raycast_staged<T, CH, true, MODEL, LOOP, MB>)
               : reinterpret_cast<const void*>(raycast_staged<T, CH, false, MODEL, LOOP, MB>);
}
template <typename T, int CH, int MODEL, bool LOOP>
const void* kernel_for(bool stats, bool gather, bool mb) {
  return mb ? kernel_for<T, CH, MODEL, LOOP, true>(stats, gather)
            : kernel_for<T, CH, MODEL, LOOP, false>(stats, gather);
}

template <typename T, int MODEL>
const void* kernel_ch(int C, bool stats, bool gather, bool loop, bool mb) {
  switch (C) {
    case 1: return loop ? kernel_for<T, 1, MODEL, true>(stats, gather, mb)
                        : kernel_for<T, 1, MODEL, false>(stats, gather, mb);
    case 2: return loop ? kernel_for<T, 2, MODEL, true>(stats, gather, mb)
                        : kernel_for<T, 2, MODEL, false>(stats, gather, mb);
    case 3: return loop ? kernel_for<T, 3, MODEL, true>(stats, gather, mb)
                        : kernel_for<T, 3, MODEL, false>(stats, gather, mb);
    default: return loop ? kernel_for<T, 4, MODEL, true>(stats, gather, mb)
                         : kernel_for<T, 4, MODEL, false>(stats, gather, mb);
  }
}

}  // namespace

// The ray-casting kernel of one optical model for a voxel type and channel
// count (instrumented or not, staged or gather, one tile per wave or a loop,
// linear or micro-block slots).
template <int MODEL>
const void* model_kernel(int bpv, int channels, bool stats, bool gather, bool loop, bool mb) {
  if (bpv == 1) return kernel_ch<uint8_t, MODEL>(channels, stats, gather, loop, mb);
  return kernel_ch<uint16_t, MODEL>(channels, stats, gather, loop, mb);
}

}  // namespace sg
