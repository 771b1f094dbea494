// bricks.hip -- the import step of an out-of-core volume on the device:
// the resolution pyramid of a linear level array and whole bricks (core plus
// a one-voxel apron) cut out of a level, in the form sg_cache_put stores
// (Sec 4.1: the volume is stored as chunks at several resolutions, made once
// at import; Sec 4.2: chunks move whole between the CPU and GPU caches).
//
// Both calls work on plain device arrays of the volume's voxel type, x
// fastest, indexed [z][y][x]; they need no volume handle and run on the
// current device.
#include <algorithm>
#include <vector>

#include "sg_internal.h"

namespace sg {

namespace {

struct Dims {
  int64_t n[3];
};

// One coarser level: voxel g = (sum of the 2x2x2 children 2g + delta, each
// child index clamped to the finer level, + 4) >> 3 (the pyramid rule of
// the resident volume's builder, on a linear array).
template <typename T>
__global__ void pyramid_level_kernel(const T* src, Dims s, T* dst, Dims d, int64_t total) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = i % d.n[0];
    const int64_t y = (i / d.n[0]) % d.n[1];
    const int64_t z = i / (d.n[0] * d.n[1]);
    const int64_t x0 = 2 * x, x1 = min(2 * x + 1, s.n[0] - 1);
    const int64_t y0 = 2 * y, y1 = min(2 * y + 1, s.n[1] - 1);
    const int64_t z0 = 2 * z, z1 = min(2 * z + 1, s.n[2] - 1);
    const int64_t sy = s.n[0], sz = s.n[0] * s.n[1];
    uint32_t sum = (uint32_t)src[z0 * sz + y0 * sy + x0] + (uint32_t)src[z0 * sz + y0 * sy + x1] +
                   (uint32_t)src[z0 * sz + y1 * sy + x0] + (uint32_t)src[z0 * sz + y1 * sy + x1] +
                   (uint32_t)src[z1 * sz + y0 * sy + x0] + (uint32_t)src[z1 * sz + y0 * sy + x1] +
                   (uint32_t)src[z1 * sz + y1 * sy + x0] + (uint32_t)src[z1 * sz + y1 * sy + x1];
    dst[i] = (T)((sum + 4u) >> 3);
  }
}

// Brick regions: region j holds level voxels B b_j - 1 .. B b_j + B per
// axis, indices clamped to the level, as an S^3 block (S = B + 2), x
// fastest. One thread per region voxel.
template <typename T>
__global__ void region_kernel(const T* level, Dims d, const int32_t* coords, int32_t B,
                              T* out, int64_t total) {
  const int64_t S = B + 2, S3 = S * S * S;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = i / S3;
    const int64_t r = i - j * S3;
    const int64_t lx = r % S, ly = (r / S) % S, lz = r / (S * S);
    const int32_t* c = coords + 3 * j;
    const int64_t gx = min(max((int64_t)B * c[0] - 1 + lx, (int64_t)0), d.n[0] - 1);
    const int64_t gy = min(max((int64_t)B * c[1] - 1 + ly, (int64_t)0), d.n[1] - 1);
    const int64_t gz = min(max((int64_t)B * c[2] - 1 + lz, (int64_t)0), d.n[2] - 1);
    out[i] = level[(gz * d.n[1] + gy) * d.n[0] + gx];
  }
}

int grid_for(int64_t work) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 65536));
}

// Select the caller's current device explicitly for this thread, as every
// other entry point does for its volume's device, before any launch.
sg_status current_device(int* dev) {
  SG_HIP(hipGetDevice(dev));
  SG_HIP(hipSetDevice(*dev));
  return SG_OK;
}

sg_status check_dims(const int32_t* dims, const char* where) {
  if (!dims) return fail(SG_ERR_INVALID_ARG, std::string(where) + ": NULL dims");
  for (int a = 0; a < 3; ++a)
    if (dims[a] < 1 || dims[a] > (1 << 20))
      return fail(SG_ERR_INVALID_ARG, std::string(where) + ": dims must be in [1, 2^20]");
  return SG_OK;
}

}  // namespace

}  // namespace sg

using namespace sg;

extern "C" sg_status sg_pyramid_level(int32_t dtype, const int32_t src_dims[3], const void* src,
                                      void* dst, void* hip_stream) {
  sg_status st = check_dims(src_dims, "sg_pyramid_level");
  if (st != SG_OK) return st;
  if (dtype != SG_U8 && dtype != SG_U16)
    return fail(SG_ERR_INVALID_ARG, "sg_pyramid_level: dtype must be SG_U8 or SG_U16");
  if (!src || !dst) return fail(SG_ERR_INVALID_ARG, "sg_pyramid_level: NULL src or dst");
  Dims s, d;
  for (int a = 0; a < 3; ++a) {
    s.n[a] = src_dims[a];
    d.n[a] = (src_dims[a] + 1) / 2;
  }
  const int64_t total = d.n[0] * d.n[1] * d.n[2];
  const int64_t bpv = dtype == SG_U8 ? 1 : 2;
  const uint8_t* sb = static_cast<const uint8_t*>(src);
  const uint8_t* db = static_cast<const uint8_t*>(dst);
  if (db < sb + s.n[0] * s.n[1] * s.n[2] * bpv && sb < db + total * bpv)
    return fail(SG_ERR_INVALID_ARG, "sg_pyramid_level: dst overlaps src");
  int dev = 0;
  if ((st = current_device(&dev)) != SG_OK) return st;
  // the launch's own status (not the thread's last-error state, which may
  // hold an earlier call's error)
  const void* sp = src;
  void* dp = dst;
  int64_t tot = total;
  void* pa[] = {&sp, &s, &dp, &d, &tot};
  const void* k = dtype == SG_U8 ? reinterpret_cast<const void*>(pyramid_level_kernel<uint8_t>)
                                 : reinterpret_cast<const void*>(pyramid_level_kernel<uint16_t>);
  SG_HIP(hipLaunchKernel(k, dim3(grid_for(total)), dim3(256), pa, 0, (hipStream_t)hip_stream));
  return SG_OK;
}

extern "C" sg_status sg_brick_regions(int32_t dtype, const int32_t dims[3], const void* level,
                                      int32_t brick, int32_t n, const int32_t* coords, void* out,
                                      void* hip_stream) {
  sg_status st = check_dims(dims, "sg_brick_regions");
  if (st != SG_OK) return st;
  if (dtype != SG_U8 && dtype != SG_U16)
    return fail(SG_ERR_INVALID_ARG, "sg_brick_regions: dtype must be SG_U8 or SG_U16");
  if (brick < 2 || brick > 256 || (brick & (brick - 1)) != 0)
    return fail(SG_ERR_INVALID_ARG, "sg_brick_regions: brick must be a power of two in [2, 256]");
  if (n < 0) return fail(SG_ERR_INVALID_ARG, "sg_brick_regions: n must be >= 0");
  if (n == 0) return SG_OK;
  if (!level || !coords || !out)
    return fail(SG_ERR_INVALID_ARG, "sg_brick_regions: NULL level, coords or out");
  for (int32_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      const int32_t g = (dims[a] + brick - 1) / brick;
      if (coords[3 * i + a] < 0 || coords[3 * i + a] >= g)
        return fail(SG_ERR_INVALID_ARG, "sg_brick_regions: brick coordinate outside the grid");
    }
  Dims d;
  for (int a = 0; a < 3; ++a) d.n[a] = dims[a];
  const int64_t S = brick + 2;
  const int64_t total = (int64_t)n * S * S * S;
  int dev = 0;
  if ((st = current_device(&dev)) != SG_OK) return st;
  hipStream_t str = (hipStream_t)hip_stream;
  int32_t* dc = nullptr;
  const size_t cbytes = (size_t)n * 3 * sizeof(int32_t);
  SG_HIP(hipMallocAsync((void**)&dc, cbytes, str));
  SG_HIP(hipMemcpyAsync(dc, coords, cbytes, hipMemcpyHostToDevice, str));
  // the host coordinates are consumed before the call returns
  SG_HIP(hipStreamSynchronize(str));
  const void* lvl = level;
  int64_t tot = total;
  void* pa[] = {&lvl, &d, &dc, &brick, &out, &tot};
  const void* k = dtype == SG_U8 ? reinterpret_cast<const void*>(region_kernel<uint8_t>)
                                 : reinterpret_cast<const void*>(region_kernel<uint16_t>);
  const hipError_t le = hipLaunchKernel(k, dim3(grid_for(total)), dim3(256), pa, 0, str);
  SG_HIP(hipFreeAsync(dc, str));
  if (le != hipSuccess) return hip_fail(le, "region_kernel launch");
  return SG_OK;
}
