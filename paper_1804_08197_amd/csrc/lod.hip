// lod.hip -- per-view LOD cut and cut map (Sec 5.2).
//
// The cut is the set of nodes that suit the view while every ancestor does
// not (the top-down traversal of Sec 5.2). A node (L, b) suits when its
// voxel edge s = 2^L, seen from the eye at the distance d of the node's
// nearest point, subtends no more than tau pixels of angular size theta:
//   s*s <= K * d*d,  K = (tau * theta)^2,  theta = (tan_top - tan_bottom) / H,
// and every node at the finest allowed level (lod_bias) suits. Instead of a
// recursive traversal, one thread per level-0 brick cell walks its ancestor
// chain from the top level down and records the first node that suits: that
// node is in the cut (its ancestors were all rejected) and the map
// cell -> node covers the volume exactly once. The comparison is done in
// IEEE double with no contraction (this file is built with
// -ffp-contract=off), so it reproduces the CPU reference bit for bit.
//
// Cache volumes (Sec 5.2, 4.2): a node that does not suit is refined only
// when every existing child is resident for every channel at the render's
// timepoint; otherwise the walk stops there (the block is rendered one level
// coarser) and the missing children are requested (a bit per (timepoint,
// node) keeps each request once in the list until the host reads it). This
// is a property of the node, so all cells below it stop alike and the map
// stays a partition.
#include <algorithm>
#include <vector>

#include "sg_internal.h"

namespace sg {

namespace {

struct CutGeom {
  int32_t dims[3];
  int32_t grid[kMaxLevels][3];
  int64_t node_off[kMaxLevels];
  int32_t B;
  int32_t top;
  int32_t bias;
  int32_t lod;
  int64_t cells;  // level-0 bricks
  // cache volumes
  int32_t cache;
  int32_t channels;
  int64_t nodes;
  int64_t req_base;          // timepoint * nodes
  const int32_t* page;       // at timepoint: [C][nodes]
  uint32_t* req_flags;       // [T * nodes] bits
  uint32_t* req_list;
  uint32_t* req_count;
  const int32_t* enable;     // NULL, or a device flag: 0 = do nothing
};

__device__ __forceinline__ bool node_resident(const CutGeom& g, int64_t node) {
  for (int c = 0; c < g.channels; ++c)
    if (g.page[(int64_t)c * g.nodes + node] < 0) return false;
  return true;
}

__device__ __forceinline__ int64_t node_index(const CutGeom& g, int L, int bx, int by, int bz) {
  return g.node_off[L] + ((int64_t)bz * g.grid[L][1] + by) * g.grid[L][0] + bx;
}

// Does node (L, b)'s box lie outside every ray of view V (Sec 5.2: blocks
// no ray can see are left out)? The rays leave the eye inside the pyramid
// of the image's edge tangents, so a box whose eight corners all lie beyond
// one of its four side planes meets none of them; in the camera frame a
// corner lies beyond the right plane when x > tan_right z, z the distance
// along the view axis. Views with a lens map are never culled (their rays
// leave the pyramid). FP64, the box [B 2^L b, B 2^L (b+1)] clipped to the
// volume.
__device__ bool node_outside_view(const CutGeom& g, const ViewDev& V, int L, int bx, int by,
                                  int bz) {
  if (V.lens_on) return false;
  const int b[3] = {bx, by, bz};
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    const int64_t w = (int64_t)g.B << L;
    const int64_t h = w * (b[a] + 1);
    lo[a] = (double)(w * b[a]);
    hi[a] = (double)(h > g.dims[a] ? (int64_t)g.dims[a] : h);
  }
  int nr = 0, nl = 0, nt = 0, nb = 0;
  for (int k = 0; k < 8; ++k) {
    const double q0 = ((k & 1) ? hi[0] : lo[0]) - V.e[0];
    const double q1 = ((k & 2) ? hi[1] : lo[1]) - V.e[1];
    const double q2 = ((k & 4) ? hi[2] : lo[2]) - V.e[2];
    const double x = (q0 * V.R[0] + q1 * V.R[3]) + q2 * V.R[6];
    const double y = (q0 * V.R[1] + q1 * V.R[4]) + q2 * V.R[7];
    const double z = -((q0 * V.R[2] + q1 * V.R[5]) + q2 * V.R[8]);
    nr += x > V.tr * z;
    nl += x < V.tl * z;
    nt += y > V.tt * z;
    nb += y < V.tb * z;
  }
  return nr == 8 || nl == 8 || nt == 8 || nb == 8;
}

// Cache volumes: are all existing children of (L, b) resident? Requests the
// missing ones that a ray of view V can see.
__device__ bool children_resident(const CutGeom& g, const ViewDev& V, int L, int bx, int by,
                                  int bz) {
  bool all = true;
  for (int k = 0; k < 8; ++k) {
    const int cx = 2 * bx + (k & 1), cy = 2 * by + ((k >> 1) & 1), cz = 2 * bz + (k >> 2);
    if (cx >= g.grid[L - 1][0] || cy >= g.grid[L - 1][1] || cz >= g.grid[L - 1][2]) continue;
    const int64_t child = node_index(g, L - 1, cx, cy, cz);
    if (node_resident(g, child)) continue;
    all = false;
    if (node_outside_view(g, V, L - 1, cx, cy, cz)) continue;
    const int64_t e = g.req_base + child;
    const uint32_t bit = 1u << (e & 31);
    if ((atomicOr(g.req_flags + (e >> 5), bit) & bit) == 0u) {
      const uint32_t i = atomicAdd(g.req_count, 1u);
      if (i < (uint32_t)kReqCap) g.req_list[i] = (uint32_t)e;
    }
  }
  return all;
}

__device__ __forceinline__ bool node_suits(const CutGeom& g, const double e[3],
                                           double K, int L, int bx, int by,
                                           int bz) {
  int32_t b[3] = {bx, by, bz};
  double dl[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int64_t w = (int64_t)g.B << L;
    int64_t lo = w * b[a];
    int64_t hi = w * (b[a] + 1);
    if (hi > g.dims[a]) hi = g.dims[a];
    double u = (double)lo - e[a];
    double v = e[a] - (double)hi;
    double m = u > v ? u : v;
    dl[a] = m > 0.0 ? m : 0.0;
  }
  double d2 = (dl[0] * dl[0] + dl[1] * dl[1]) + dl[2] * dl[2];
  double s = (double)((int64_t)1 << L);
  return (s * s) <= (K * d2);
}

// Grid: x strides over the level-0 cells, y is the view (so the view's
// record is read once per workgroup, from the arguments when inline).
__global__ void cutmap_kernel(CutGeom g, ViewDev* views, int32_t* cutmap, InlineViews iv) {
  if (g.enable && *g.enable == 0) return;
  const int v = (int)blockIdx.y;
  if (iv.n && blockIdx.x == 0 && v == 0) {
    // the small view table, from the arguments into the device table
    const uint32_t* src = reinterpret_cast<const uint32_t*>(iv.v);
    uint32_t* dst = reinterpret_cast<uint32_t*>(views);
    const int words = iv.n * (int)(sizeof(ViewDev) / 4);
    for (int k = threadIdx.x; k < words; k += blockDim.x) dst[k] = src[k];
  }
  const ViewDev& V = iv.n ? iv.v[v] : views[v];
  const double e[3] = {V.e[0], V.e[1], V.e[2]};
  const double K = V.K;
  int32_t* out = cutmap + V.cut_off;
  for (int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; cell < g.cells;
       cell += (int64_t)gridDim.x * blockDim.x) {
    int32_t cx = (int32_t)(cell % g.grid[0][0]);
    int32_t cy = (int32_t)((cell / g.grid[0][0]) % g.grid[0][1]);
    int32_t cz = (int32_t)(cell / ((int64_t)g.grid[0][0] * g.grid[0][1]));
    int L = (g.lod || g.cache) ? g.top : g.bias;
    for (; L > g.bias; --L) {
      if (g.lod && node_suits(g, e, K, L, cx >> L, cy >> L, cz >> L)) break;
      if (g.cache && !children_resident(g, V, L, cx >> L, cy >> L, cz >> L)) break;
    }
    const int64_t node = node_index(g, L, cx >> L, cy >> L, cz >> L);
    out[cell] = (int32_t)node;
  }
}

__global__ void mark_kernel(const int32_t* cutmap, int64_t cells, uint8_t* flags) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cells;
       i += (int64_t)gridDim.x * blockDim.x)
    flags[cutmap[i]] = 1;
}

CutGeom cut_geom(const Volume* v, int bias, bool lod, int timepoint) {
  CutGeom g{};
  if (v->cache) {
    g.cache = 1;
    g.channels = v->d.channels;
    g.nodes = v->nodes;
    g.req_base = (int64_t)timepoint * v->nodes;
    g.page = v->page + (int64_t)timepoint * v->d.channels * v->nodes;
    g.req_flags = v->req_flags;
    g.req_list = v->req_list;
    g.req_count = v->req_count;
  }
  for (int a = 0; a < 3; ++a) g.dims[a] = v->d.dims[a];
  for (int L = 0; L < v->L; ++L) {
    for (int a = 0; a < 3; ++a) g.grid[L][a] = v->grid[L][a];
    g.node_off[L] = v->node_off[L];
  }
  g.B = v->B;
  g.top = v->L - 1;
  g.bias = bias;
  g.lod = lod ? 1 : 0;
  g.cells = (int64_t)v->grid[0][0] * v->grid[0][1] * v->grid[0][2];
  return g;
}

}  // namespace

sg_status cutmap_launch(const Volume* v, const ViewDev* dviews, int n_views, int bias,
                        bool lod, int timepoint, int32_t* cutmap, Launch* out,
                        const int32_t* enable, const InlineViews* iv) {
  CutGeom g = cut_geom(v, bias, lod, timepoint);
  g.enable = enable;
  const int64_t blocks = std::min<int64_t>((g.cells + 255) / 256, 4096);
  out->func = reinterpret_cast<const void*>(cutmap_kernel);
  out->grid = dim3((unsigned)std::max<int64_t>(blocks, 1), (unsigned)std::max(n_views, 1));
  out->block = dim3(256);
  out->lds = 0;
  out->arg.clear();
  InlineViews inl{};
  if (iv && iv->n) inl = *iv;
  out->push(g);
  out->push(const_cast<ViewDev*>(dviews));
  out->push(cutmap);
  out->push(inl);
  return SG_OK;
}

sg_status cutmap_run(const Volume* v, const ViewDev* dviews, int n_views, int bias, bool lod,
                     int timepoint, int32_t* cutmap, const InlineViews& iv, hipStream_t s) {
  CutGeom g = cut_geom(v, bias, lod, timepoint);
  const int64_t blocks = std::min<int64_t>((g.cells + 255) / 256, 4096);
  ViewDev* dv = const_cast<ViewDev*>(dviews);
  InlineViews ivc = iv;
  void* pa[] = {&g, &dv, &cutmap, &ivc};
  SG_HIP(hipLaunchKernel(reinterpret_cast<const void*>(cutmap_kernel),
                         dim3((unsigned)std::max<int64_t>(blocks, 1),
                              (unsigned)std::max(n_views, 1)),
                         dim3(256), pa, 0, s));
  return SG_OK;
}

sg_status launch_cutmap(Volume* v, const ViewDev* dviews, int n_views, int bias,
                        bool lod, int timepoint, hipStream_t s, const int32_t* enable) {
  Launch l;
  sg_status st = cutmap_launch(v, dviews, n_views, bias, lod, timepoint, v->cutmap, &l, enable,
                               &v->inline_views);
  if (st != SG_OK) return st;
  return l.run(s);
}

}  // namespace sg

extern "C" sg_status sg_get_lod_cut(sg_volume* vol, const sg_view* view,
                                    const sg_render_params* params, uint64_t* nodes,
                                    int32_t* n_nodes, uint8_t* empty, void* hip_stream) {
  using namespace sg;
  if (!vol || !view || !params || !n_nodes || (*n_nodes > 0 && !nodes) || *n_nodes < 0)
    return fail(SG_ERR_INVALID_ARG, "sg_get_lod_cut: NULL argument or negative capacity");
  Volume* v = &vol->v;
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "sg_get_lod_cut: cannot select device");
  hipStream_t s = (hipStream_t)hip_stream;
  int view_blocks = 0;
  sg_status st = commit(v, s);
  if (st != SG_OK) return st;
  st = prepare_views(v, 1, view, params, nullptr, nullptr, nullptr, s, &view_blocks);
  if (st != SG_OK) return st;
  const bool lod = (params->flags & SG_LOD) != 0;
  if (!top_level_resident(v, params->timepoint))
    return fail(SG_ERR_STATE, "sg_get_lod_cut: a top-level node is not in the cache");
  ++v->frame;
  st = launch_cutmap(v, reinterpret_cast<const ViewDev*>(v->view_dev), 1, params->lod_bias,
                     lod, params->timepoint, s);
  if (st != SG_OK) return st;
  const int64_t cells = (int64_t)v->grid[0][0] * v->grid[0][1] * v->grid[0][2];
  uint8_t* dflags = nullptr;
  SG_HIP(hipMallocAsync((void**)&dflags, (size_t)v->nodes, s));
  SG_HIP(hipMemsetAsync(dflags, 0, (size_t)v->nodes, s));
  int64_t blocks = std::min<int64_t>((cells + 255) / 256, 65536);
  hipLaunchKernelGGL(mark_kernel, dim3((unsigned)blocks), dim3(256), 0, s, v->cutmap, cells,
                     dflags);
  SG_HIP(hipGetLastError());
  std::vector<uint8_t> flags(v->nodes), emp(v->nodes, 0);
  SG_HIP(hipMemcpyAsync(flags.data(), dflags, (size_t)v->nodes, hipMemcpyDeviceToHost, s));
  const bool have_empty = !v->empty_dirty && !v->tf_dirty;
  if (empty && have_empty)
    SG_HIP(hipMemcpyAsync(emp.data(), v->empty + (int64_t)params->timepoint * v->nodes,
                          (size_t)v->nodes, hipMemcpyDeviceToHost, s));
  SG_HIP(hipStreamSynchronize(s));
  SG_HIP(hipFreeAsync(dflags, s));
  if (empty && !have_empty)
    return fail(SG_ERR_STATE, "sg_get_lod_cut: empty flags need a transfer function for "
                              "every channel");
  std::vector<std::pair<uint64_t, uint8_t>> out;
  for (int L = 0; L < v->L; ++L)
    for (int64_t z = 0; z < v->grid[L][2]; ++z)
      for (int64_t y = 0; y < v->grid[L][1]; ++y)
        for (int64_t x = 0; x < v->grid[L][0]; ++x) {
          int64_t n = v->node_off[L] + (z * v->grid[L][1] + y) * v->grid[L][0] + x;
          if (!flags[n]) continue;
          uint64_t id = ((uint64_t)L << 60) | ((uint64_t)x << 40) | ((uint64_t)y << 20) |
                        (uint64_t)z;
          out.emplace_back(id, emp[n]);
        }
  std::sort(out.begin(), out.end());
  if ((int64_t)out.size() > *n_nodes) {
    *n_nodes = (int32_t)out.size();
    return fail(SG_ERR_INVALID_ARG, "sg_get_lod_cut: capacity too small");
  }
  *n_nodes = (int32_t)out.size();
  // the skip bit of the requested optical model (none for maximum intensity)
  const uint8_t mask = params->model == SG_MODEL_EMISSION_ABSORPTION ? 1
                       : params->model == SG_MODEL_EMISSION_ONLY   ? 2
                                                                     : 0;
  for (size_t i = 0; i < out.size(); ++i) {
    nodes[i] = out[i].first;
    if (empty) empty[i] = (out[i].second & mask) ? 1 : 0;
  }
  return SG_OK;
}
