// composite.hip -- sort-last compositing of the part images of one view.
//
// Each part is the render of one box of the volume (the region of interest
// clips every ray to it), premultiplied on a zero background. The over
// operator of emission-absorption compositing (Sec 5.1) is associative, so
// per pixel the parts combine front over back in the order the pixel's ray
// enters their boxes (disjoint boxes: a ray crosses them one after another):
//   C = sum_k (prod_{j<k} (1 - A_j)) C_k, and A likewise.
// With one box per GPU this is the exchange-free half of a sort-last split;
// here all parts are on one device.
#include <algorithm>
#include <cmath>

#include "raycast_kernels.h"

namespace sg {
namespace {

constexpr int kMaxParts = 8;

struct Parts {
  const float4* img[kMaxParts];
  double box[kMaxParts][6];  // lo xyz, hi xyz
  int n;
};

__global__ __launch_bounds__(256) void composite_kernel(ViewDev V, Parts P, float4* out) {
  const int64_t npix = (int64_t)V.W * V.H;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npix;
       i += (int64_t)gridDim.x * blockDim.x) {
    double e[3], d[3];
    view_ray(V, (int)(i % V.W), (int)(i / V.W), e, d);
    // the boxes the ray crosses, sorted by entry parameter (insertion)
    double t[kMaxParts];
    int idx[kMaxParts];
    int m = 0;
    for (int k = 0; k < P.n; ++k) {
      double t0, t1;
      if (!box_interval(e, d, P.box[k], P.box[k] + 3, t0, t1)) continue;
      int j = m++;
      while (j > 0 && t[j - 1] > t0) {
        t[j] = t[j - 1];
        idx[j] = idx[j - 1];
        --j;
      }
      t[j] = t0;
      idx[j] = k;
    }
    float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
    float T = 1.f;  // transmittance of the parts in front
    for (int j = 0; j < m; ++j) {
      const float4 p = P.img[idx[j]][i];
      c.x = fmaf(T, p.x, c.x);
      c.y = fmaf(T, p.y, c.y);
      c.z = fmaf(T, p.z, c.z);
      c.w = fmaf(T, p.w, c.w);
      T *= 1.0f - p.w;
    }
    out[i] = c;
  }
}

}  // namespace
}  // namespace sg

extern "C" sg_status sg_composite_over(const sg_view* view, int32_t n_parts,
                                       const float* const* parts, const double* boxes,
                                       float* out_rgba, void* hip_stream) {
  using namespace sg;
  if (!view || !parts || !boxes || !out_rgba)
    return fail(SG_ERR_INVALID_ARG, "sg_composite_over: NULL argument");
  if (n_parts < 1 || n_parts > kMaxParts)
    return fail(SG_ERR_INVALID_ARG, "sg_composite_over: n_parts must be in [1, 8]");
  if (reinterpret_cast<uintptr_t>(out_rgba) % 16 != 0)
    return fail(SG_ERR_INVALID_ARG, "sg_composite_over: out_rgba must be 16-byte aligned");
  Parts P{};
  P.n = n_parts;
  for (int k = 0; k < n_parts; ++k) {
    if (!parts[k] || reinterpret_cast<uintptr_t>(parts[k]) % 16 != 0)
      return fail(SG_ERR_INVALID_ARG, "sg_composite_over: part images must be 16-byte aligned");
    P.img[k] = reinterpret_cast<const float4*>(parts[k]);
    for (int a = 0; a < 6; ++a) {
      if (!std::isfinite(boxes[6 * k + a]))
        return fail(SG_ERR_INVALID_ARG, "sg_composite_over: boxes must be finite");
      P.box[k][a] = boxes[6 * k + a];
    }
    for (int a = 0; a < 3; ++a)
      if (!(P.box[k][a] < P.box[k][a + 3]))
        return fail(SG_ERR_INVALID_ARG, "sg_composite_over: box lo must be below hi");
  }
  ViewDev V;
  sg_status st = view_geometry(*view, &V);
  if (st != SG_OK) return st;
  const int64_t npix = (int64_t)V.W * V.H;
  const int64_t blocks = std::min<int64_t>((npix + 255) / 256, 65536);
  // the caller's current device, selected explicitly for this thread
  int dev = 0;
  SG_HIP(hipGetDevice(&dev));
  SG_HIP(hipSetDevice(dev));
  float4* out = reinterpret_cast<float4*>(out_rgba);
  void* pa[] = {&V, &P, &out};
  SG_HIP(hipLaunchKernel(reinterpret_cast<const void*>(composite_kernel), dim3((unsigned)blocks),
                         dim3(256), pa, 0, (hipStream_t)hip_stream));
  return SG_OK;
}
