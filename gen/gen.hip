// gen.hip -- seeded synthetic volume generators for the large workloads.
//
// Input generation only: nothing here is part of the ray caster, and the ray
// caster shares no code with it. Each voxel value is a pure function of the
// voxel index and the seeded primitive lists built in gen/__init__.py, so a
// region can be generated on the GPU (fast, for the 2048^3 volume) or on the
// CPU (small regions, for checking the generator itself).
//
//  * tubes: Poisson(200) background (inverse-CDF sampling with SplitMix64
//    counter-based uniforms, Steele, Lea & Flood 2014) plus, per branch of a
//    filament, amp * exp(-d^2 / (2 r^2)) with d the distance from the voxel
//    centre to the branch polyline, cut at d > 3r; sum clipped to 65535.
//  * cells: 4 broad background Gaussians plus Gaussian cells cut at 3 sigma.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#define HD __host__ __device__

namespace {

HD inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

HD inline int poisson_sample(uint64_t seed, uint64_t idx, const double* cdf, int kmax) {
  uint64_t h = splitmix64(idx ^ (seed * 0xD1B54A32D192ED03ull));
  double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);
  int lo = 0, hi = kmax;  // smallest k with cdf[k] > u
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (cdf[mid] > u) hi = mid; else lo = mid + 1;
  }
  return lo;
}

struct Region {
  int64_t x0, y0, z0;
  int32_t nx, ny, nz;
  int32_t dims[3];
  int32_t bin;  // bin (brick) edge of the primitive lists
  int32_t gx, gy;
};

HD inline int64_t bin_of(const Region& r, int32_t x, int32_t y, int32_t z) {
  return ((int64_t)(z / r.bin) * r.gy + (y / r.bin)) * r.gx + (x / r.bin);
}

HD inline float tube_sum(float px, float py, float pz, const float4* A, const float4* Bv,
                         const int32_t* br, const int64_t* off, const int32_t* ids, int64_t bin) {
  float sum = 0.f, best = INFINITY, rr = 0.f, amp = 0.f;
  int32_t cur = -1;
  for (int64_t k = off[bin]; k < off[bin + 1]; ++k) {
    int32_t i = ids[k];
    if (br[i] != cur) {
      if (cur >= 0 && best <= 9.f * rr * rr) sum += amp * expf(-best / (2.f * rr * rr));
      cur = br[i];
      best = INFINITY;
      rr = A[i].w;
      amp = Bv[i].w;
    }
    float ax = px - A[i].x, ay = py - A[i].y, az = pz - A[i].z;
    float dx = Bv[i].x - A[i].x, dy = Bv[i].y - A[i].y, dz = Bv[i].z - A[i].z;
    float l2 = dx * dx + dy * dy + dz * dz;
    float t = l2 > 0.f ? (ax * dx + ay * dy + az * dz) / l2 : 0.f;
    t = t < 0.f ? 0.f : (t > 1.f ? 1.f : t);
    float qx = ax - t * dx, qy = ay - t * dy, qz = az - t * dz;
    float d2 = qx * qx + qy * qy + qz * qz;
    best = d2 < best ? d2 : best;
  }
  if (cur >= 0 && best <= 9.f * rr * rr) sum += amp * expf(-best / (2.f * rr * rr));
  return sum;
}

HD inline uint16_t tube_voxel(const Region& r, int64_t li, const float4* A, const float4* Bv,
                              const int32_t* br, const int64_t* off, const int32_t* ids,
                              const double* cdf, int kmax, uint64_t seed) {
  int32_t lx = (int32_t)(li % r.nx);
  int32_t ly = (int32_t)((li / r.nx) % r.ny);
  int32_t lz = (int32_t)(li / ((int64_t)r.nx * r.ny));
  int32_t x = (int32_t)(r.x0 + lx), y = (int32_t)(r.y0 + ly), z = (int32_t)(r.z0 + lz);
  uint64_t gidx = ((uint64_t)z * r.dims[1] + y) * r.dims[0] + x;
  float v = (float)poisson_sample(seed, gidx, cdf, kmax);
  v += tube_sum(x + 0.5f, y + 0.5f, z + 0.5f, A, Bv, br, off, ids, bin_of(r, x, y, z));
  v = rintf(v);
  return (uint16_t)(v > 65535.f ? 65535.f : v);
}

HD inline uint16_t cell_voxel(const Region& r, int64_t li, const float4* C, const int64_t* off,
                              const int32_t* ids, const float4* bg, float bg_sigma) {
  int32_t lx = (int32_t)(li % r.nx);
  int32_t ly = (int32_t)((li / r.nx) % r.ny);
  int32_t lz = (int32_t)(li / ((int64_t)r.nx * r.ny));
  int32_t x = (int32_t)(r.x0 + lx), y = (int32_t)(r.y0 + ly), z = (int32_t)(r.z0 + lz);
  float px = x + 0.5f, py = y + 0.5f, pz = z + 0.5f;
  float v = 0.f;
  for (int k = 0; k < 4; ++k) {
    float dx = px - bg[k].x, dy = py - bg[k].y, dz = pz - bg[k].z;
    v += bg[k].w * expf(-(dx * dx + dy * dy + dz * dz) / (2.f * bg_sigma * bg_sigma));
  }
  int64_t bin = bin_of(r, x, y, z);
  for (int64_t k = off[bin]; k < off[bin + 1]; ++k) {
    const float4 c = C[2 * ids[k]];
    const float4 s = C[2 * ids[k] + 1];  // sigma, amp
    float dx = px - c.x, dy = py - c.y, dz = pz - c.z;
    float d2 = dx * dx + dy * dy + dz * dz;
    if (d2 <= 9.f * s.x * s.x) v += s.y * expf(-d2 / (2.f * s.x * s.x));
  }
  v = rintf(v);
  return (uint16_t)(v > 65535.f ? 65535.f : v);
}

__global__ void tubes_kernel(uint16_t* out, Region r, const float4* A, const float4* Bv,
                             const int32_t* br, const int64_t* off, const int32_t* ids,
                             const double* cdf, int kmax, uint64_t seed) {
  int64_t n = (int64_t)r.nx * r.ny * r.nz;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = tube_voxel(r, i, A, Bv, br, off, ids, cdf, kmax, seed);
}

__global__ void cells_kernel(uint16_t* out, Region r, const float4* C, const int64_t* off,
                             const int32_t* ids, const float4* bg, float bg_sigma) {
  int64_t n = (int64_t)r.nx * r.ny * r.nz;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = cell_voxel(r, i, C, off, ids, bg, bg_sigma);
}

Region make_region(const int64_t* org, const int32_t* size, const int32_t* dims, int32_t bin) {
  Region r;
  r.x0 = org[0];
  r.y0 = org[1];
  r.z0 = org[2];
  r.nx = size[0];
  r.ny = size[1];
  r.nz = size[2];
  for (int a = 0; a < 3; ++a) r.dims[a] = dims[a];
  r.bin = bin;
  r.gx = (dims[0] + bin - 1) / bin;
  r.gy = (dims[1] + bin - 1) / bin;
  return r;
}

}  // namespace

extern "C" {

// Generate the tube volume over a box region into out (x fastest).
// on_device: all pointers are device pointers and the work is enqueued on
// stream; otherwise they are host pointers and the CPU fills out.
int sggen_tubes(uint16_t* out, const int64_t* org, const int32_t* size, const int32_t* dims,
                int32_t bin, const float4* A, const float4* Bv, const int32_t* br,
                const int64_t* off, const int32_t* ids, const double* cdf, int32_t kmax,
                uint64_t seed, int32_t on_device, void* stream) {
  Region r = make_region(org, size, dims, bin);
  int64_t n = (int64_t)r.nx * r.ny * r.nz;
  if (on_device) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1 << 20) blocks = 1 << 20;
    hipLaunchKernelGGL(tubes_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       out, r, A, Bv, br, off, ids, cdf, kmax, seed);
    return hipGetLastError() == hipSuccess ? 0 : -3;
  }
  for (int64_t i = 0; i < n; ++i) out[i] = tube_voxel(r, i, A, Bv, br, off, ids, cdf, kmax, seed);
  return 0;
}

// Generate one channel of the cell volume over a box region.
// C holds per cell two float4: (x, y, z, -) and (sigma, amp, -, -).
int sggen_cells(uint16_t* out, const int64_t* org, const int32_t* size, const int32_t* dims,
                int32_t bin, const float4* C, const int64_t* off, const int32_t* ids,
                const float4* bg, float bg_sigma, int32_t on_device, void* stream) {
  Region r = make_region(org, size, dims, bin);
  int64_t n = (int64_t)r.nx * r.ny * r.nz;
  if (on_device) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1 << 20) blocks = 1 << 20;
    hipLaunchKernelGGL(cells_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       out, r, C, off, ids, bg, bg_sigma);
    return hipGetLastError() == hipSuccess ? 0 : -3;
  }
  for (int64_t i = 0; i < n; ++i) out[i] = cell_voxel(r, i, C, off, ids, bg, bg_sigma);
  return 0;
}

}  // extern "C"
