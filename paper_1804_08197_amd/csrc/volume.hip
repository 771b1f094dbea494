// volume.hip -- brick pool, page table, uploads, pyramid, aprons, value
// ranges and empty-node flags (the one-time per-volume work, and the
// per-transfer-function refresh).
//
// Pool layout: one slot per (timepoint, channel, node); a slot stores the
// node's brick as (B+2)^3 voxels, the core at offset (1, 1, 1) and a
// one-voxel apron around it holding the clamped neighbour values, in the
// volume's slot layout (slot_index): linear rows, x fastest, padded to a
// multiple of 4 bytes (row stride Sx), or 4^3-voxel micro-blocks
// (Sec 5.2: blocks of a multi-resolution pyramid; Sec 4.2: chunks resident
// in a GPU cache). With the apron, any trilinear sample inside a node reads
// only that node's slot.
#include <algorithm>
#include <cstring>

#include "sg_internal.h"

namespace sg {

namespace {

__device__ __forceinline__ int32_t clampi(int32_t v, int32_t lo, int32_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

template <typename T>
__device__ __forceinline__ T* slot_ptr(uint8_t* pool, int64_t slot_bytes,
                                       int32_t slot) {
  return reinterpret_cast<T*>(pool + (int64_t)slot * slot_bytes);
}

struct LevelGeom {
  int32_t n[3];      // level dims
  int32_t g[3];      // brick grid
  int64_t node_off;  // first node index of the level
};

// Upload: scatter n brick cores (x fastest) into their slots.
template <typename T>
__global__ void upload_kernel(uint8_t* pool, int64_t slot_bytes,
                              const int32_t* page, LevelGeom lg,
                              const int32_t* coords, const T* src, int n,
                              int logB, int S, int Sx, int M) {
  const int64_t per = (int64_t)1 << (3 * logB);
  const int64_t total = (int64_t)n * per;
  const int32_t B = 1 << logB, mask = B - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = i >> (3 * logB);
    int32_t v = (int32_t)(i & (per - 1));
    int32_t lx = v & mask, ly = (v >> logB) & mask, lz = v >> (2 * logB);
    const int32_t* c = coords + 3 * j;
    int64_t node = lg.node_off + ((int64_t)c[2] * lg.g[1] + c[1]) * lg.g[0] + c[0];
    T* dst = slot_ptr<T>(pool, slot_bytes, page[node]);
    dst[slot_index(lx + 1, ly + 1, lz + 1, S, Sx, M)] = src[i];
  }
}

// Pyramid: core voxel g of level L+1 = (sum of children 2g + delta, clamped
// to level L, + 4) >> 3. Children are read from level-L cores.
template <typename T>
__global__ void downsample_kernel(uint8_t* pool, int64_t slot_bytes,
                                  const int32_t* page, LevelGeom src,
                                  LevelGeom dst, int logB, int S, int Sx, int M) {
  const int32_t B = 1 << logB, mask = B - 1;
  const int64_t per = (int64_t)1 << (3 * logB);
  const int64_t nb = (int64_t)dst.g[0] * dst.g[1] * dst.g[2];
  const int64_t total = nb * per;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = i >> (3 * logB);
    int32_t v = (int32_t)(i & (per - 1));
    int32_t l[3] = {v & mask, (v >> logB) & mask, v >> (2 * logB)};
    int32_t b[3] = {(int32_t)(j % dst.g[0]), (int32_t)((j / dst.g[0]) % dst.g[1]),
                    (int32_t)(j / ((int64_t)dst.g[0] * dst.g[1]))};
    int32_t gc[3];
    for (int a = 0; a < 3; ++a) gc[a] = min(b[a] * B + l[a], dst.n[a] - 1);
    uint32_t sum = 0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          int32_t h[3] = {min(2 * gc[0] + dx, src.n[0] - 1),
                          min(2 * gc[1] + dy, src.n[1] - 1),
                          min(2 * gc[2] + dz, src.n[2] - 1)};
          int64_t node = src.node_off +
                         ((int64_t)(h[2] >> logB) * src.g[1] + (h[1] >> logB)) *
                             src.g[0] +
                         (h[0] >> logB);
          const T* p = slot_ptr<T>(pool, slot_bytes, page[node]);
          sum += p[slot_index((h[0] & mask) + 1, (h[1] & mask) + 1, (h[2] & mask) + 1, S, Sx,
                              M)];
        }
    T* q = slot_ptr<T>(pool, slot_bytes, page[dst.node_off + j]);
    q[slot_index(l[0] + 1, l[1] + 1, l[2] + 1, S, Sx, M)] = (T)((sum + 4u) >> 3);
  }
}

// Apron: every stored voxel that is not an in-extent core voxel receives the
// value of the clamped level index, read from the owning brick's core.
// One thread per stored row (y, z) of a slot.
template <typename T>
__global__ void apron_kernel(uint8_t* pool, int64_t slot_bytes,
                             const int32_t* page, LevelGeom lg, int logB,
                             int S, int Sx, int M) {
  const int32_t B = 1 << logB, mask = B - 1;
  const int64_t rows = (int64_t)S * S;
  const int64_t nb = (int64_t)lg.g[0] * lg.g[1] * lg.g[2];
  const int64_t total = nb * rows;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = i / rows;
    int32_t r = (int32_t)(i - j * rows);
    int32_t y = r % S, z = r / S;
    int32_t b[3] = {(int32_t)(j % lg.g[0]), (int32_t)((j / lg.g[0]) % lg.g[1]),
                    (int32_t)(j / ((int64_t)lg.g[0] * lg.g[1]))};
    int32_t gy = b[1] * B - 1 + y, gz = b[2] * B - 1 + z;
    bool row_core = y >= 1 && y <= B && z >= 1 && z <= B && gy < lg.n[1] &&
                    gz < lg.n[2];
    int32_t cy = clampi(gy, 0, lg.n[1] - 1), cz = clampi(gz, 0, lg.n[2] - 1);
    T* dst = slot_ptr<T>(pool, slot_bytes, page[lg.node_off + j]);
    for (int32_t x = 0; x < S; ++x) {
      int32_t gx = b[0] * B - 1 + x;
      bool core = row_core && x >= 1 && x <= B && gx < lg.n[0];
      if (core) continue;
      int32_t cx = clampi(gx, 0, lg.n[0] - 1);
      int64_t node = lg.node_off +
                     ((int64_t)(cz >> logB) * lg.g[1] + (cy >> logB)) * lg.g[0] +
                     (cx >> logB);
      const T* p = slot_ptr<T>(pool, slot_bytes, page[node]);
      dst[slot_index(x, y, z, S, Sx, M)] =
          p[slot_index((cx & mask) + 1, (cy & mask) + 1, (cz & mask) + 1, S, Sx, M)];
    }
  }
}

// Value range of every stored voxel of a slot (core and apron).
template <typename T>
__global__ __launch_bounds__(256) void range_kernel(const uint8_t* pool,
                                                    int64_t slot_bytes,
                                                    const int32_t* page,
                                                    uint32_t* range,
                                                    int64_t nodes, int S, int Sx, int M) {
  const int64_t node = blockIdx.x;
  const T* p = reinterpret_cast<const T*>(pool + (int64_t)page[node] * slot_bytes);
  const int32_t n = S * S * S;
  uint32_t lo = 0xFFFFFFFFu, hi = 0;
  for (int32_t i = threadIdx.x; i < n; i += 256) {
    const int32_t row = i / S, x = i - row * S;  // (not the row padding)
    const int32_t y = row % S, z = row / S;
    uint32_t v = p[slot_index(x, y, z, S, Sx, M)];
    lo = min(lo, v);
    hi = max(hi, v);
  }
  __shared__ uint32_t slo[256], shi[256];
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      slo[threadIdx.x] = min(slo[threadIdx.x], slo[threadIdx.x + s]);
      shi[threadIdx.x] = max(shi[threadIdx.x], shi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    range[2 * node] = slo[0];
    range[2 * node + 1] = shi[0];
  }
}

// Skip flags (one thread per (timepoint, node)). Bit 0 (transparent): for
// every channel the extinction of every table entry from floor(u_min) - 1
// to floor(u_max) + 2 is zero, u being the continuous table index of the
// node's min / max value. Bit 1 (dark): the same entries emit no colour.
// The one-entry guard band on each side keeps the flags exact for samples
// whose index is rounded in single precision.
__global__ void empty_kernel(const uint32_t* range, const float* tf, int tf_n,
                             const double* lo, const double* hi, int C,
                             int64_t nodes, int64_t total, uint8_t* empty) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = i / nodes, node = i - t * nodes;
    bool clear = true, dark = true;
    for (int c = 0; c < C && (clear || dark); ++c) {
      const uint32_t* r = range + 2 * ((t * C + c) * nodes + node);
      double umin = (((double)r[0] - lo[c]) / (hi[c] - lo[c])) * (double)(tf_n - 1);
      double umax = (((double)r[1] - lo[c]) / (hi[c] - lo[c])) * (double)(tf_n - 1);
      int64_t klo = (int64_t)floor(umin) - 1;
      int64_t khi = (int64_t)floor(umax) + 2;
      klo = klo < 0 ? 0 : (klo > tf_n - 1 ? tf_n - 1 : klo);
      khi = khi < 0 ? 0 : (khi > tf_n - 1 ? tf_n - 1 : khi);
      const float* tc = tf + (int64_t)c * (tf_n + 1) * 4;
      for (int64_t k = klo; k <= khi; ++k) {
        if (tc[4 * k + 3] != 0.0f) clear = false;
        if (tc[4 * k] != 0.0f || tc[4 * k + 1] != 0.0f || tc[4 * k + 2] != 0.0f) dark = false;
      }
    }
    empty[i] = (uint8_t)((clear ? 1 : 0) | (dark ? 2 : 0));
  }
}

LevelGeom geom(const Volume* v, int L) {
  LevelGeom g;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = v->ldims[L][a];
    g.g[a] = v->grid[L][a];
  }
  g.node_off = v->node_off[L];
  return g;
}

int blocks_for(int64_t work, int per_block = 256) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 262144) b = 262144;
  return (int)b;
}

const int32_t* page_at(const Volume* v, int c, int t) {
  return v->page + ((int64_t)t * v->d.channels + c) * v->nodes;
}

}  // namespace

sg_status launch_upload(Volume* v, int c, int t, int level, int n,
                        const int32_t* dcoords, const void* dsrc,
                        hipStream_t s) {
  LevelGeom lg = geom(v, level);
  int64_t work = (int64_t)n << (3 * v->logB);
  if (v->bpv == 1)
    hipLaunchKernelGGL(upload_kernel<uint8_t>, dim3(blocks_for(work)), dim3(256), 0, s,
                       v->pool, v->slot_bytes, page_at(v, c, t), lg, dcoords,
                       (const uint8_t*)dsrc, n, v->logB, v->S, v->Sx, v->M);
  else
    hipLaunchKernelGGL(upload_kernel<uint16_t>, dim3(blocks_for(work)), dim3(256), 0, s,
                       v->pool, v->slot_bytes, page_at(v, c, t), lg, dcoords,
                       (const uint16_t*)dsrc, n, v->logB, v->S, v->Sx, v->M);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

sg_status launch_downsample(Volume* v, int c, int t, int level_dst,
                            hipStream_t s) {
  LevelGeom src = geom(v, level_dst - 1), dst = geom(v, level_dst);
  int64_t work = ((int64_t)dst.g[0] * dst.g[1] * dst.g[2]) << (3 * v->logB);
  if (v->bpv == 1)
    hipLaunchKernelGGL(downsample_kernel<uint8_t>, dim3(blocks_for(work)), dim3(256), 0, s,
                       v->pool, v->slot_bytes, page_at(v, c, t), src, dst, v->logB, v->S, v->Sx,
                       v->M);
  else
    hipLaunchKernelGGL(downsample_kernel<uint16_t>, dim3(blocks_for(work)), dim3(256), 0,
                       s, v->pool, v->slot_bytes, page_at(v, c, t), src, dst, v->logB,
                       v->S, v->Sx, v->M);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

sg_status launch_apron(Volume* v, int c, int t, hipStream_t s) {
  for (int L = 0; L < v->L; ++L) {
    LevelGeom lg = geom(v, L);
    int64_t work = (int64_t)lg.g[0] * lg.g[1] * lg.g[2] * v->S * v->S;
    if (v->bpv == 1)
      hipLaunchKernelGGL(apron_kernel<uint8_t>, dim3(blocks_for(work)), dim3(256), 0, s,
                         v->pool, v->slot_bytes, page_at(v, c, t), lg, v->logB, v->S, v->Sx,
                         v->M);
    else
      hipLaunchKernelGGL(apron_kernel<uint16_t>, dim3(blocks_for(work)), dim3(256), 0, s,
                         v->pool, v->slot_bytes, page_at(v, c, t), lg, v->logB, v->S, v->Sx,
                         v->M);
    SG_HIP(hipGetLastError());
  }
  return SG_OK;
}

sg_status launch_range(Volume* v, int c, int t, hipStream_t s) {
  uint32_t* r = v->range + 2 * ((int64_t)t * v->d.channels + c) * v->nodes;
  if (v->bpv == 1)
    hipLaunchKernelGGL(range_kernel<uint8_t>, dim3((unsigned)v->nodes), dim3(256), 0, s,
                       v->pool, v->slot_bytes, page_at(v, c, t), r, v->nodes, v->S, v->Sx,
                       v->M);
  else
    hipLaunchKernelGGL(range_kernel<uint16_t>, dim3((unsigned)v->nodes), dim3(256), 0, s,
                       v->pool, v->slot_bytes, page_at(v, c, t), r, v->nodes, v->S, v->Sx,
                       v->M);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

sg_status launch_empty(Volume* v, hipStream_t s) {
  const int C = v->d.channels;
  // tables: TF [C][tf_n+1][4] floats, then lo[C], hi[C] doubles
  std::vector<uint8_t> blob;
  int64_t tf_bytes = (int64_t)C * (v->tf_n + 1) * 4 * sizeof(float);
  blob.resize(tf_bytes + 2 * C * sizeof(double));
  float* f = reinterpret_cast<float*>(blob.data());
  for (int c = 0; c < C; ++c) {
    const std::vector<float>& h = v->tf_host[c];
    float* o = f + (int64_t)c * (v->tf_n + 1) * 4;
    std::memcpy(o, h.data(), h.size() * sizeof(float));
    std::memcpy(o + 4 * v->tf_n, h.data() + 4 * (v->tf_n - 1), 4 * sizeof(float));
  }
  double* lohi = reinterpret_cast<double*>(blob.data() + tf_bytes);
  for (int c = 0; c < C; ++c) {
    lohi[c] = v->tf_lo[c];
    lohi[C + c] = v->tf_hi[c];
  }
  sg_status st = stage_to_device(v, blob.data(), (int64_t)blob.size(), v->tf, s);
  if (st != SG_OK) return st;
  const double* dlo = reinterpret_cast<const double*>(reinterpret_cast<uint8_t*>(v->tf) + tf_bytes);
  int64_t total = (int64_t)v->d.timepoints * v->nodes;
  hipLaunchKernelGGL(empty_kernel, dim3(blocks_for(total)), dim3(256), 0, s, v->range,
                     v->tf, v->tf_n, dlo, dlo + C, C, v->nodes, total, v->empty);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

sg_status commit(Volume* v, hipStream_t s) {
  bool any = false;
  for (int t = 0; t < v->d.timepoints; ++t)
    for (int c = 0; c < v->d.channels; ++c) {
      uint8_t& p = v->pending[(int64_t)t * v->d.channels + c];
      if (!p) continue;
      sg_status st = launch_apron(v, c, t, s);
      if (st != SG_OK) return st;
      st = launch_range(v, c, t, s);
      if (st != SG_OK) return st;
      p = 0;
      any = true;
    }
  if (any) v->empty_dirty = true;
  bool all_tf = true;
  for (int c = 0; c < v->d.channels; ++c) all_tf = all_tf && v->tf_set[c];
  if (all_tf && (v->empty_dirty || v->tf_dirty)) {
    sg_status st = launch_empty(v, s);
    if (st != SG_OK) return st;
    v->empty_dirty = false;
    v->tf_dirty = false;
  }
  return SG_OK;
}

}  // namespace sg
