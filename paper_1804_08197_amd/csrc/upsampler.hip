// upsampler.hip -- the learned upsampler: inference and training kernels.
//
// Fewer rays per frame (Sec 5.3): the volume is ray cast at half resolution
// one pyramid level coarser and a 4-layer 3x3 convolutional network predicts
// the full-resolution frame (the network is described in
// sg_upsampler.h). Activations are NHWC bfloat16 with 8 (input) or 32
// channels, so one pixel's channels are one contiguous 16- or 64-byte run.
//
// Convolution = implicit GEMM on the matrix cores, taken transposed: 32
// output channels x 32 pixels per v_mfma_f32_32x32x16_bf16, FP32
// accumulators, the weights as the A operand and the pixels as B. The
// GEMM's K runs over (tap, input channel) in steps of 16: with 32 input
// channels a tap is two K-steps; with 8 input channels a K-step covers two
// taps (K = 72 padded to 80). A lane's A operand is 8 consecutive K of one
// output channel (the weights are packed that way, [K / 8][32][8]) and its
// B operand 8 consecutive channels of one pixel at one tap (one 16-byte
// load); its results are 16 channels (four runs of four) of one pixel.
//
// Backward: the input gradient of a 3x3 convolution is a 3x3 convolution of
// the output gradient with the taps mirrored and the channel roles swapped,
// so it runs on the same kernel with weights packed that way and the ReLU
// derivative applied as a mask. Weight gradients sum x (tap-shifted) times
// the output gradient over every pixel: FP32 partial sums per workgroup,
// added in a fixed order (deterministic). Adam keeps FP32 master weights.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/sg_upsampler.h"
#include "sg_internal.h"

namespace sg {

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kLayers = 4;
constexpr int kCin[kLayers] = {8, 32, 32, 32};
constexpr int kCh = 32;       // output channels of every layer
constexpr int kUsed = 20;     // used output channels of the last layer

// packed weights: per layer w[9][cin][32] then b[32]
constexpr int64_t layer_size(int l) { return (int64_t)9 * kCin[l] * kCh + kCh; }
constexpr int64_t kParams = layer_size(0) + layer_size(1) + layer_size(2) + layer_size(3);
int64_t layer_off(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += layer_size(i);
  return o;
}
// K of a layer's GEMM (9 * cin rounded up to a multiple of 32)
constexpr int kdim(int cin) { return ((9 * cin + 31) / 32) * 32; }

__device__ __forceinline__ float bf(bf16 x) { return (float)x; }

// The products run on v_mfma_f32_32x32x16_bf16 (on gfx950 it sustains
// about 1.6x the rate of the 16x16x32 form). Operand layouts (lane l,
// half = l / 32): A[row l % 32][k 8 half .. + 7], B[k 8 half .. + 7][column
// l % 32]; result register r holds row 8 (r / 4) + 4 half + r % 4 of column
// l % 32. A K-step is 16 K; K runs over (tap, input channel), padded to a
// multiple of 16 (72 -> 80 for 8 input channels).
typedef float floatx16 __attribute__((ext_vector_type(16)));
constexpr int ksteps(int cin) { return (9 * cin + 15) / 16; }
__device__ __forceinline__ int acc_channel(int r, int half) {
  return 8 * (r >> 2) + 4 * half + (r & 3);
}
// four floats as four bfloat16 (round to nearest even), packed
__device__ __forceinline__ uint2 pack4(const float (&r)[4]) {
  uint2 pk;
  pk.x = (uint32_t)__builtin_bit_cast(uint16_t, (bf16)r[0]) |
         ((uint32_t)__builtin_bit_cast(uint16_t, (bf16)r[1]) << 16);
  pk.y = (uint32_t)__builtin_bit_cast(uint16_t, (bf16)r[2]) |
         ((uint32_t)__builtin_bit_cast(uint16_t, (bf16)r[3]) << 16);
  return pk;
}

// --------------------------------------------------------------- kernels
// x0 from a render: r, g, b, a, depth code, 0, 0, 0
__global__ void prep_kernel(const float4* rgba, const float* depth, int64_t P, float inv_scale,
                            bf16* x0) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    const float4 c = rgba[p];
    const float d = depth[p];
    const float code = isfinite(d) ? 1.0f / (1.0f + d * inv_scale) : 0.0f;
    bf16x8 v;
    v[0] = (bf16)c.x;
    v[1] = (bf16)c.y;
    v[2] = (bf16)c.z;
    v[3] = (bf16)c.w;
    v[4] = (bf16)code;
    v[5] = v[6] = v[7] = (bf16)0.0f;
    reinterpret_cast<bf16x8*>(x0)[p] = v;
  }
}

// Epilogues of the convolution kernel.
enum { kReluBf16 = 0, kBiasF32 = 1, kMaskBf16 = 2 };

// y[p][co] = bias[co] + sum_{tap, ci} x[p + off(tap)][ci] * w[tap][ci][co]
// (the bias is the accumulator's starting value; the sum runs in K order),
// then the epilogue; zero padding, for N images of H x W. wt: packed
// [K / 8][32][8] bf16. A wave computes 64 pixels (two blocks of 32) x 32
// channels as the transposed product: A = weights (32 channels x 16 K),
// B = pixels (16 K x 32 pixels).
template <int CIN, int EPI>
__global__ __launch_bounds__(256) void conv_kernel(const bf16* __restrict__ x, int N, int H, int W,
                                                   const bf16x8* __restrict__ wt,
                                                   const float* __restrict__ bias,
                                                   void* __restrict__ out,
                                                   const bf16* __restrict__ mask) {
  const int lane = threadIdx.x & 63, col = lane & 31, half = lane >> 5;
  const int64_t P = (int64_t)N * H * W;
  const int64_t p0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64;
  if (p0 >= P) return;  // whole wave
  // the lane's pixel in each of the two blocks
  int py[2], px[2], pn[2];
  bool pv[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    const int64_t p = p0 + mb * 32 + col;
    pv[mb] = p < P;
    const int64_t q = pv[mb] ? p : 0;
    pn[mb] = (int)(q / ((int64_t)H * W));
    const int r = (int)(q - (int64_t)pn[mb] * H * W);
    py[mb] = r / W;
    px[mb] = r - py[mb] * W;
  }
  // the bias is the accumulators' starting value (no bias: 0); register r
  // holds channel acc_channel(r, half)
  floatx16 acc[2];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const float b = EPI == kMaskBf16 ? 0.f : bias[acc_channel(r, half)];
    acc[0][r] = b;
    acc[1][r] = b;
  }
  constexpr int KSTEPS = ksteps(CIN);
  const bf16x8 zero8 = {(bf16)0.f, (bf16)0.f, (bf16)0.f, (bf16)0.f,
                        (bf16)0.f, (bf16)0.f, (bf16)0.f, (bf16)0.f};
#pragma unroll 1
  for (int s = 0; s < KSTEPS; ++s) {
    const int k8 = 2 * s + half;  // this lane's group of 8 K values
    const int tap = CIN == 32 ? k8 >> 2 : k8;
    const int c0 = CIN == 32 ? (k8 & 3) * 8 : 0;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    bf16x8 a[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const int yy = py[mb] + dy, xx = px[mb] + dx;
      const bool in = pv[mb] && tap < 9 && yy >= 0 && yy < H && xx >= 0 && xx < W;
      a[mb] = in ? *reinterpret_cast<const bf16x8*>(
                       x + (((int64_t)pn[mb] * H + yy) * W + xx) * CIN + c0)
                 : zero8;
    }
    const bf16x8 w = wt[(int64_t)k8 * kCh + col];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
      acc[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, a[mb], acc[mb], 0, 0, 0);
  }
  // lane: pixel p0 + 32 mb + col; channels acc_channel(4 g + i, half) =
  // 8 g + 4 half + i, four consecutive per g
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    const int64_t p = p0 + mb * 32 + col;
    if (p >= P) continue;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int c = 8 * g + 4 * half;
      const float v0 = acc[mb][4 * g], v1 = acc[mb][4 * g + 1], v2 = acc[mb][4 * g + 2],
                  v3 = acc[mb][4 * g + 3];
      if (EPI == kBiasF32) {
        *reinterpret_cast<float4*>(reinterpret_cast<float*>(out) + p * kCh + c) =
            make_float4(v0, v1, v2, v3);
      } else {
        float r[4] = {v0, v1, v2, v3};
        if (EPI == kReluBf16) {
#pragma unroll
          for (int i = 0; i < 4; ++i) r[i] = fmaxf(r[i], 0.0f);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) r[i] = bf(mask[p * kCh + c + i]) > 0.0f ? r[i] : 0.0f;
        }
        *reinterpret_cast<uint2*>(reinterpret_cast<bf16*>(out) + p * kCh + c) = pack4(r);
      }
    }
  }
}

// Bilinear x2 (half-pixel centres, clamped) of x0's rgba at full-resolution
// pixel (2y + sy, 2x + sx).
__device__ __forceinline__ float4 base_rgba(const bf16* x0, int n, int H, int W, int y, int x,
                                            int sy, int sx) {
  const int ya = sy ? y : y - 1, xa = sx ? x : x - 1;
  const float fy = sy ? 0.25f : 0.75f, fx = sx ? 0.25f : 0.75f;
  const int y0 = min(max(ya, 0), H - 1), y1 = min(max(ya + 1, 0), H - 1);
  const int x0i = min(max(xa, 0), W - 1), x1 = min(max(xa + 1, 0), W - 1);
  auto at = [&](int yy, int xx, int c) {
    return bf(x0[(((int64_t)n * H + yy) * W + xx) * 8 + c]);
  };
  float o[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float a = at(y0, x0i, c), b = at(y0, x1, c), cc = at(y1, x0i, c), d = at(y1, x1, c);
    const float top = a + (b - a) * fx, bot = cc + (d - cc) * fx;
    o[c] = top + (bot - top) * fy;
  }
  return make_float4(o[0], o[1], o[2], o[3]);
}

// Inference rule: a pixel whose 9 x 9 neighbourhood of x0 (the receptive
// field of the four 3 x 3 layers; outside the image counts as zero) holds
// no nonzero value yields background and a predicted error of 0.
constexpr int kReach = 4;
__device__ __forceinline__ bool x0_nonzero(const bf16x8& v) {
  const uint4 u = __builtin_bit_cast(uint4, v);
  return ((u.x | u.y | u.z | u.w) & 0x7FFF7FFFu) != 0u;  // -0 counts as zero
}
__device__ bool empty_neighbourhood(const bf16* x0, int n, int H, int W, int y, int x) {
  for (int yy = max(y - kReach, 0); yy <= min(y + kReach, H - 1); ++yy)
    for (int xx = max(x - kReach, 0); xx <= min(x + kReach, W - 1); ++xx)
      if (x0_nonzero(reinterpret_cast<const bf16x8*>(x0)[((int64_t)n * H + yy) * W + xx]))
        return false;
  return true;
}

// Inference epilogue: full-resolution rgba and predicted squared error.
// Grid: x = 256-pixel chunks of one image, y = images (strided). With
// partials, each workgroup writes its chunk's sum of the prediction to
// partials[image * gridDim.x + chunk] (a fixed-order tree sum: the result
// does not depend on scheduling); tile_sum_kernel adds them per image.
__global__ __launch_bounds__(256) void shuffle_kernel(const float* o, const bf16* x0, int N, int H,
                                                      int W, float4* out, float* err,
                                                      double* partials) {
  __shared__ double red[256];
  const int64_t HW = (int64_t)H * W;
  for (int n = blockIdx.y; n < N; n += gridDim.y) {
    const int64_t r0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    float zsum = 0.f;
    if (r0 < HW) {
      const int r = (int)r0, y = r / W, x = r - y * W;
      const int64_t p = (int64_t)n * HW + r;
      const float* op = o + p * kCh;
      const bool empty = empty_neighbourhood(x0, n, H, W, y, x);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int sy = s >> 1, sx = s & 1;
        const int64_t q = ((int64_t)n * 2 * H + 2 * y + sy) * (2 * W) + 2 * x + sx;
        if (empty) {  // background, and no predicted error
          out[q] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (err) err[q] = 0.f;
          continue;
        }
        const float4 b = base_rgba(x0, n, H, W, y, x, sy, sx);
        out[q] = make_float4(b.x + op[5 * s], b.y + op[5 * s + 1], b.z + op[5 * s + 2],
                             b.w + op[5 * s + 3]);
        const float z = op[5 * s + 4];
        if (err) err[q] = z * z;
        zsum += z * z;
      }
    }
    if (partials) {  // uniform across the workgroup
      red[threadIdx.x] = (double)zsum;
      __syncthreads();
      for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
      }
      if (threadIdx.x == 0) partials[(int64_t)n * gridDim.x + blockIdx.x] = red[0];
      __syncthreads();
    }
  }
}

// ------------------------------------------------ fused inference kernel
// One workgroup per 16 x 16 tile of low-resolution pixels runs the whole
// network: x0 on the tile plus a 4-pixel halo, h1 on a 3-pixel halo, h2 on
// 2, h3 on 1, o on the tile, every activation in LDS (two buffers used in
// turn: V holds x0, then h2, then o; U holds h1, then h3). Each layer is the
// implicit GEMM of conv_kernel with the same operand layouts, K order,
// epilogue arithmetic and zero padding (activations outside the image are
// stored as 0), so the result equals the layer-by-layer path bit for bit.
// A wave owns up to eight 16-pixel row blocks of a layer's region and keeps
// their accumulators across the K loop, so each weight fragment is loaded
// once per K-step and reused by all of them.
// A hidden pixel's 32 bf16 channels occupy 80 bytes (64 + 16 of padding):
// the 16 pixels of a 16-byte-per-lane read then start on 16 different
// groups of four 4-byte banks (a 64-byte stride would put them on 4).
constexpr int kTile = 16;
constexpr int kE0 = kTile + 8;                               // x0 region edge
constexpr int kPix = kCh + 8;                                // bf16 per hidden pixel (padded)
constexpr int kBufU = (kE0 - 2) * (kE0 - 2) * kPix;          // bf16 elements (h1, h3)
constexpr int kBufV = (kE0 - 4) * (kE0 - 4) * kPix;          // bf16 elements (x0, h2, o)
constexpr int kE1 = kTile + 2;                               // x0 rgba ring edge
constexpr size_t kFusedLds = (size_t)(kBufU + kBufV) * 2 + kE1 * kE1 * 16 + 256 * 8;
static_assert(kE0 * kE0 * 8 <= kBufV, "x0 region fits buffer V");
static_assert(kTile * kTile * kUsed * 2 <= kBufV, "o (FP32, used channels) fits buffer V");
static_assert(kFusedLds <= 80 * 1024, "two workgroups per CU");

// One layer on a region: input region edge EIN in `sin` (CIN channels per
// pixel), output region edge EIN - 2 into `sout` (bf16 x 32 after bias and
// ReLU, or FP32 x kUsed after bias when LAST). (oy0, ox0): image position
// of the output region's first pixel. The product is taken transposed
// (weights as the A operand, pixels as B): the same 32 products per output
// value in the same K order, and each lane ends up holding 4 consecutive
// channels of one pixel, stored with one 8- or 16-byte LDS write.
// A layer's weight fragments for this lane, every K-step (the A operand).
template <int CIN>
__device__ __forceinline__ void load_weights(const bf16x8* __restrict__ wt,
                                             bf16x8 (&wf)[ksteps(CIN)]) {
  const int lane = threadIdx.x & 63, col = lane & 31, half = lane >> 5;
#pragma unroll
  for (int s = 0; s < ksteps(CIN); ++s) wf[s] = wt[(int64_t)(2 * s + half) * kCh + col];
}

// NJ 32-pixel blocks of a layer's output region for this wave (blocks
// wave, wave + 4, ...): input region edge EIN in `sin` (CIN channels per
// pixel), output region edge EIN - 2 into `sout` (bf16 x 32 after ReLU, or
// FP32 x kUsed when LAST). (oy0, ox0): image position of the output
// region's first pixel. wf: this layer's weights; the next layer's (wn from
// wnext, unless LAST) are loaded right after the products, so their latency
// overlaps the epilogue and the barrier.
template <int CIN, int EIN, int NJ, bool LAST>
__device__ __forceinline__ void fused_blocks(const bf16* __restrict__ sin,
                                             void* __restrict__ sout,
                                             const bf16x8 (&wf)[ksteps(CIN)],
                                             const bf16x8* __restrict__ wnext,
                                             bf16x8 (&wn)[ksteps(32)],
                                             const float* __restrict__ bias, int oy0, int ox0,
                                             int H, int W) {
  constexpr int EO = EIN - 2, MO = EO * EO;
  constexpr int PB = CIN == 32 ? kPix * 2 : 16;  // bytes per input pixel
  constexpr int KSTEPS = ksteps(CIN);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, half = lane >> 5;
  const bf16x8 zero8 = {(bf16)0.f, (bf16)0.f, (bf16)0.f, (bf16)0.f,
                        (bf16)0.f, (bf16)0.f, (bf16)0.f, (bf16)0.f};
  // the bias is the accumulators' starting value (as in conv_kernel)
  floatx16 acc[NJ];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const float b = bias[acc_channel(r, half)];
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[j][r] = b;
  }
  // byte address of the top-left input pixel of the lane's 3 x 3 window
  // (with 32 channels, plus the lane's 8-channel group within a tap's
  // 16-K step); every tap is then a constant offset
  const char* base[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int q = min((wave + 4 * j) * 32 + col, MO - 1);  // pixels past the region repeat
    const int qy = q / EO, qx = q - qy * EO;
    base[j] = reinterpret_cast<const char*>(sin) + (qy * EIN + qx) * PB +
              (CIN == 32 ? half * 16 : 0);
  }
  // K-step s: lane K group k8 = 2 s + half. With 32 channels the tap is
  // s / 2 for the whole wave and the channel group 2 (s % 2) + half; with
  // 8 channels the tap is k8 (zero beyond the ninth).
  auto load = [&](int s, bf16x8 (&a)[NJ]) {
    if (CIN == 32) {
      const int tap = s >> 1;
      const int off = ((tap / 3) * EIN + (tap % 3)) * PB + (s & 1) * 32;  // constant
#pragma unroll
      for (int j = 0; j < NJ; ++j) a[j] = *reinterpret_cast<const bf16x8*>(base[j] + off);
    } else {
      const int tap = 2 * s + half;
      const int off = ((tap / 3) * EIN + (tap % 3)) * PB;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        a[j] = tap < 9 ? *reinterpret_cast<const bf16x8*>(base[j] + off) : zero8;
    }
  };
  // the pixel fragments of step s + 1 are read while the products of step
  // s run (two register sets); the scheduling groups keep that order
  bf16x8 a[2][NJ];
  load(0, a[0]);
  __builtin_amdgcn_sched_group_barrier(0x0100, NJ, 0);  // step 0's reads first
#pragma unroll
  for (int s = 0; s < KSTEPS; ++s) {
    if (s + 1 < KSTEPS) load(s + 1, a[(s + 1) & 1]);
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[s], a[s & 1][j], acc[j], 0, 0, 0);
    if (s + 1 < KSTEPS) __builtin_amdgcn_sched_group_barrier(0x0100, NJ, 0);  // LDS reads
    __builtin_amdgcn_sched_group_barrier(0x0008, NJ, 0);                       // products
  }
  if (!LAST) load_weights<32>(wnext, wn);
  __builtin_amdgcn_sched_barrier(0);
  // lane: pixel (block) * 32 + col, channels 8 g + 4 half + i. A region
  // inside the image (most tiles; uniform over the workgroup) needs no mask.
  const bool interior = oy0 >= 0 && ox0 >= 0 && oy0 + EO <= H && ox0 + EO <= W;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int q = (wave + 4 * j) * 32 + col;
    if (q >= MO) continue;
    if (LAST) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int c = 8 * g + 4 * half;
        if (c >= kUsed) continue;
        *reinterpret_cast<float4*>(reinterpret_cast<float*>(sout) + q * kUsed + c) =
            make_float4(acc[j][4 * g], acc[j][4 * g + 1], acc[j][4 * g + 2], acc[j][4 * g + 3]);
      }
    } else {
      bool in = true;
      if (!interior) {
        const int qy = q / EO, qx = q - qy * EO;
        const int iy = oy0 + qy, ix = ox0 + qx;
        in = iy >= 0 && iy < H && ix >= 0 && ix < W;
      }
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        float r[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) r[i] = in ? fmaxf(acc[j][4 * g + i], 0.0f) : 0.0f;
        *reinterpret_cast<uint2*>(reinterpret_cast<bf16*>(sout) + q * kPix + 8 * g + 4 * half) =
            pack4(r);
      }
    }
  }
}

// One layer: a wave takes MAXJ blocks, or MAXJ - 1 when its last one would
// lie past the region (a uniform branch between two branch-free bodies).
template <int CIN, int EIN, int MAXJ, bool LAST>
__device__ __forceinline__ void fused_layer(const bf16* __restrict__ sin, void* __restrict__ sout,
                                            const bf16x8 (&wf)[ksteps(CIN)],
                                            const bf16x8* __restrict__ wnext,
                                            bf16x8 (&wn)[ksteps(32)],
                                            const float* __restrict__ bias, int oy0, int ox0,
                                            int H, int W) {
  constexpr int NBLK = ((EIN - 2) * (EIN - 2) + 31) / 32;
  static_assert(4 * (MAXJ - 1) + 3 >= NBLK - 1, "every block has a wave");
  static_assert(MAXJ == 1 || 4 * (MAXJ - 2) + 3 < NBLK, "only a wave's last block may be idle");
  const int wave = threadIdx.x >> 6;
  if (wave + 4 * (MAXJ - 1) < NBLK)
    fused_blocks<CIN, EIN, MAXJ, LAST>(sin, sout, wf, wnext, wn, bias, oy0, ox0, H, W);
  else
    fused_blocks<CIN, EIN, MAXJ - 1, LAST>(sin, sout, wf, wnext, wn, bias, oy0, ox0, H, W);
}

// Per-image sums of the predicted squared error. The fused kernel writes
// one partial per workgroup (no atomics: device-wide atomics on one address
// serialise across the XCDs); tile_sum_kernel then adds each image's
// partials in a fixed order (deterministic), and takes the fallback
// decision if asked. The layer-by-layer path's epilogue writes one partial
// per 256-pixel chunk of an image and is summed the same way.
struct SumArgs {
  double* sum;        // [images][tiles] partials (fused: tiles; layered: 256-pixel chunks)
  double* result;     // [N] per-image sums of this launch
  int32_t* fallback;  // NULL, or the frame's decision (predicted PSNR < threshold)
  int32_t images;     // N
  int32_t tiles;      // partials per image
  double pixels;      // full-resolution pixels per image
  double threshold_db;
  int32_t* reset;     // NULL, or the tile-list counters, cleared for the next launch
};

// fallback = 1 when 10 log10(1 / m) < threshold, m the mean over the
// images of sum_i / pixels (the frame's predicted mean squared error)
__device__ __forceinline__ int32_t decide(const double* result, int n, double pixels,
                                          double threshold_db) {
  double m = 0.0;
  for (int i = 0; i < n; ++i) m += result[i] / pixels;
  m /= (double)n;
  const double psnr = m <= 0.0 ? INFINITY : 10.0 * log10(1.0 / m);
  return psnr < threshold_db ? 1 : 0;
}

// One workgroup of kSumThreads: result[i] = the partials of image i added
// in a fixed order (deterministic). The 16 waves are split into groups of
// wpi waves, one group per image (a stereo pair: 8 waves each), so that
// the images' loads are in flight together; thread u of a group adds
// partials u, u + 64 wpi, ... (four loads in flight), the 64 lanes of each
// wave fold by xor-shuffles, and the group's waves' sums are added in wave
// order. More images than waves take several rounds.
constexpr int kSumThreads = 1024;
constexpr int kSumWaves = kSumThreads / 64;
__global__ __launch_bounds__(kSumThreads) void tile_sum_kernel(SumArgs a) {
  __shared__ double red[kSumWaves];
  const int t = (int)threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wpi = a.images >= kSumWaves ? 1 : kSumWaves / max(a.images, 1);
  const int ipr = kSumWaves / wpi;  // images per round
  const int g = wave / wpi;         // this wave's group (idle when g >= ipr)
  const int stride = wpi * 64, u = (wave - g * wpi) * 64 + lane;
  for (int r0 = 0; r0 < a.images; r0 += ipr) {
    const int i = r0 + g;
    double v = 0.0;
    if (g < ipr && i < a.images) {
      const double* p = a.sum + (int64_t)i * a.tiles;
      for (int base = 0; base < a.tiles; base += 4 * stride) {
        double x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = base + j * stride + u;
          x[j] = k < a.tiles ? p[k] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) v += x[j];
      }
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (t < ipr && r0 + t < a.images) {
      double r = 0.0;
      for (int w = 0; w < wpi; ++w) r += red[t * wpi + w];
      a.result[r0 + t] = r;
    }
    __syncthreads();
  }
  if (t == 0 && a.fallback) *a.fallback = decide(a.result, a.images, a.pixels, a.threshold_db);
  if (t == 0 && a.reset) {
    a.reset[0] = 0;
    a.reset[1] = 0;
  }
}

// the workgroup's share of the predicted error, into its partial slot
__device__ void tile_partial(const SumArgs& a, double* red, float zsum, int64_t slot) {
  red[threadIdx.x] = (double)zsum;
  __syncthreads();
  for (int st = (int)blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.sum[slot] = red[0];
}

// The network on a tile with content (every layer, then the pixel shuffle,
// bilinear residual and error head); returns this thread's share of the
// predicted squared error.
__device__ __forceinline__ float fused_tile(
    bf16* sU, bf16* sV, const float4* sX, const uint8_t* nzf, uint8_t* rowany,
    const bf16x8 (&wa)[ksteps(8)], bf16x8 (&wb)[ksteps(32)], bf16x8 (&wc)[ksteps(32)],
    const bf16x8* __restrict__ w1, const bf16x8* __restrict__ w2, const bf16x8* __restrict__ w3,
    const float* __restrict__ b0, const float* __restrict__ b1, const float* __restrict__ b2,
    const float* __restrict__ b3, int n, int H, int W, int ty0, int tx0, int qy, int qx, int y,
    int x, float4* __restrict__ out, float* __restrict__ err) {
  // per pixel: any nonzero in its 9 x 9 window (rows qy .. qy+8, columns
  // qx .. qx+8 of the region), as a row pass and a column pass
  for (int e = threadIdx.x; e < kE0 * kTile; e += 256) {
    const int ry = e / kTile, cx = e % kTile;
    uint8_t m = 0;
#pragma unroll
    for (int d = 0; d <= 2 * kReach; ++d) m |= nzf[ry * kE0 + cx + d];
    rowany[e] = m;
  }
  __syncthreads();
  bool empty = true;
#pragma unroll
  for (int d = 0; d <= 2 * kReach; ++d) empty &= rowany[(qy + d) * kTile + qx] == 0;
  fused_layer<8, kE0, 4, false>(sV, sU, wa, w1, wb, b0, ty0 - 3, tx0 - 3, H, W);
  __syncthreads();
  fused_layer<32, kE0 - 2, 4, false>(sU, sV, wb, w2, wc, b1, ty0 - 2, tx0 - 2, H, W);
  __syncthreads();
  fused_layer<32, kE0 - 4, 3, false>(sV, sU, wc, w3, wb, b2, ty0 - 1, tx0 - 1, H, W);
  __syncthreads();
  fused_layer<32, kE0 - 6, 2, true>(sU, sV, wb, nullptr, wc, b3, ty0, tx0, H, W);
  __syncthreads();
  // pixel shuffle, bilinear residual and error head, one thread per pixel
  float zsum = 0.f;
  if (y < H && x < W && empty) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {  // background, and no predicted error
      const int64_t q = ((int64_t)n * 2 * H + 2 * y + (s >> 1)) * (2 * W) + 2 * x + (s & 1);
      out[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (err) err[q] = 0.f;
    }
  } else if (y < H && x < W) {
    const float* op = reinterpret_cast<const float*>(sV) + threadIdx.x * kUsed;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int sy = s >> 1, sx = s & 1;
      const int ya = sy ? y : y - 1, xa = sx ? x : x - 1;
      const float fy = sy ? 0.25f : 0.75f, fx = sx ? 0.25f : 0.75f;
      // neighbours clamped into the image, which keeps them in the ring
      const int r0 = min(max(ya, 0), H - 1) - (ty0 - 1), r1 = min(max(ya + 1, 0), H - 1) - (ty0 - 1);
      const int c0 = min(max(xa, 0), W - 1) - (tx0 - 1), c1 = min(max(xa + 1, 0), W - 1) - (tx0 - 1);
      const float4 A = sX[r0 * kE1 + c0], B = sX[r0 * kE1 + c1], Cc = sX[r1 * kE1 + c0],
                   D = sX[r1 * kE1 + c1];
      const float av[4] = {A.x, A.y, A.z, A.w}, bvv[4] = {B.x, B.y, B.z, B.w},
                  cv[4] = {Cc.x, Cc.y, Cc.z, Cc.w}, dv[4] = {D.x, D.y, D.z, D.w};
      float o[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float top = av[c] + (bvv[c] - av[c]) * fx, bot = cv[c] + (dv[c] - cv[c]) * fx;
        o[c] = top + (bot - top) * fy;
      }
      const int64_t q = ((int64_t)n * 2 * H + 2 * y + sy) * (2 * W) + 2 * x + sx;
      out[q] = make_float4(o[0] + op[5 * s], o[1] + op[5 * s + 1], o[2] + op[5 * s + 2],
                           o[3] + op[5 * s + 3]);
      const float z = op[5 * s + 4];
      if (err) err[q] = z * z;
      zsum += z * z;
    }
  }
  return zsum;
}

// LDS allows two workgroups per CU (two waves per SIMD): the register
// budget is set for that, so a K-step's reads can all be in flight.
// x0 of tile (n, ty0, tx0) with a 4-pixel halo (zero outside the image)
// into LDS: the bf16 region in sV, its nonzero flags in nzf and the rgba of
// the tile plus a 1-pixel ring in sX. Every load is issued before any is
// used. Returns whether this thread saw a nonzero input pixel.
constexpr int kPrep = (kE0 * kE0 + 255) / 256;
__device__ __forceinline__ bool prep_region(const float4* __restrict__ rgba,
                                            const float* __restrict__ depth, int H, int W,
                                            float inv_scale, int n, int ty0, int tx0, bf16* sV,
                                            uint8_t* nzf, float4* sX) {
  float4 pc[kPrep];
  float pd[kPrep];
#pragma unroll
  for (int k = 0; k < kPrep; ++k) {
    const int p = threadIdx.x + 256 * k;
    const int y = ty0 - 4 + p / kE0, x = tx0 - 4 + p % kE0;
    pc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    pd[k] = INFINITY;
    if (p < kE0 * kE0 && y >= 0 && y < H && x >= 0 && x < W) {
      const int64_t q = ((int64_t)n * H + y) * W + x;
      pc[k] = rgba[q];
      pd[k] = depth[q];
    }
  }
  bool any_nz = false;
#pragma unroll
  for (int k = 0; k < kPrep; ++k) {
    const int p = threadIdx.x + 256 * k;
    if (p >= kE0 * kE0) continue;
    const int y = ty0 - 4 + p / kE0, x = tx0 - 4 + p % kE0;
    bf16x8 v;
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = (bf16)0.0f;
    if (y >= 0 && y < H && x >= 0 && x < W) {
      const float4 c = pc[k];
      const float d = pd[k];
      const float code = isfinite(d) ? 1.0f / (1.0f + d * inv_scale) : 0.0f;
      v[0] = (bf16)c.x;
      v[1] = (bf16)c.y;
      v[2] = (bf16)c.z;
      v[3] = (bf16)c.w;
      v[4] = (bf16)code;
    }
    reinterpret_cast<bf16x8*>(sV)[p] = v;
    const bool nz = x0_nonzero(v);
    nzf[p] = nz ? 1 : 0;
    any_nz |= nz;
    const int ry = p / kE0 - 3, rx = p % kE0 - 3;
    if (ry >= 0 && ry < kE1 && rx >= 0 && rx < kE1)
      sX[ry * kE1 + rx] = make_float4(bf(v[0]), bf(v[1]), bf(v[2]), bf(v[3]));
  }
  return any_nz;
}

// Background for every output pixel of tile (n, ty0, tx0): the 32 x 32
// output pixels written row by row (store j of lane i: pixel j * 256 + i),
// so that each store covers whole 512-byte output rows.
__device__ __forceinline__ void clear_tile(int n, int H, int W, int ty0, int tx0,
                                           float4* __restrict__ out, float* __restrict__ err) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int e = j * 256 + (int)threadIdx.x;
    const int oy = 2 * ty0 + e / (2 * kTile), ox = 2 * tx0 + e % (2 * kTile);
    if (oy < 2 * H && ox < 2 * W) {
      const int64_t q = ((int64_t)n * 2 * H + oy) * (2 * W) + ox;
      out[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (err) err[q] = 0.f;
    }
  }
}

// LDS (kFusedLds bytes): U, V, then x0's rgba (bf16-rounded) on the tile and
// a 1-pixel ring for the bilinear base of the last phase, then the reduction
// scratch, which also holds x0's nonzero flags and their 9-wide row maxima
// until the last phase.
extern __shared__ float4 fused_smem[];  // the dynamic LDS of the fused kernel

struct FusedLds {
  bf16* sU;
  bf16* sV;
  float4* sX;
  double* red;
  uint8_t* nzf;
  uint8_t* rowany;
};
__device__ __forceinline__ FusedLds fused_lds(float4* smem) {
  FusedLds l;
  l.sU = reinterpret_cast<bf16*>(smem);
  l.sV = l.sU + kBufU;
  l.sX = reinterpret_cast<float4*>(l.sV + kBufV);
  l.red = reinterpret_cast<double*>(l.sX + kE1 * kE1);
  l.nzf = reinterpret_cast<uint8_t*>(l.red);
  l.rowany = l.nzf + kE0 * kE0;
  return l;
}
static_assert(kE0 * kE0 + kE0 * kTile <= 256 * 8, "flags fit the scratch");

// The tiles of one launch in two lists that share one array: the tiles
// with content in reach from list[0] on, the empty tiles from
// list[tiles - 1] down. A tile is numbered (image, tile row, tile column)
// row-major, which is also its partial-sum slot.
struct TileList {
  int32_t* list;   // [tiles]
  int32_t* count;  // [0]: tiles with content, [1]: empty tiles (zero before the launch)
  int32_t tiles;
  int32_t tiles_x, tiles_y;
};

// The content mask of an input without one, in the layout of the render's
// tile_any mask: one byte per 8 x 8-pixel block, 1 if any of its pixels has
// a nonzero rgba component or a finite depth (a superset of the pixels
// whose x0 is nonzero). One wave per block, four blocks per workgroup.
__global__ __launch_bounds__(256) void content_mask_kernel(const float4* __restrict__ rgba,
                                                           const float* __restrict__ depth, int H,
                                                           int W, int64_t blocks, int mh, int mw,
                                                           uint8_t* __restrict__ mask) {
  const int lane = threadIdx.x & 63;
  const int64_t per = (int64_t)mh * mw;
  // the same trip count for every lane of a wave
  for (int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); blk < blocks;
       blk += (int64_t)gridDim.x * 4) {
    const int64_t n = blk / per;
    const int r = (int)(blk - n * per);
    const int y = (r / mw) * 8 + (lane >> 3), x = (r % mw) * 8 + (lane & 7);
    bool nz = false;
    if (y < H && x < W) {
      const int64_t q = (n * H + y) * W + x;
      const float4 c = rgba[q];
      nz = c.x != 0.f || c.y != 0.f || c.z != 0.f || c.w != 0.f || depth[q] < INFINITY;
    }
    const uint64_t m = __ballot(nz);
    if (lane == 0) mask[blk] = m != 0 ? 1 : 0;
  }
}

static_assert(kTile == 16 && kReach <= 8, "a tile's input region meets at most 4 x 4 blocks");

// One thread per 16 x 16 tile: the tile has content in reach when a block
// of the mask that meets its input region (the tile and a kReach-pixel
// ring, clamped to the image) is nonzero; the tile then joins the first
// list, else the second (with a zero partial sum). A wave appends with one
// atomic per list; the order within a list does not matter, since every
// tile writes only its own pixels and its own partial-sum slot.
__global__ __launch_bounds__(256) void tile_list_kernel(const uint8_t* __restrict__ mask, int H,
                                                        int W, TileList tl, double* sum) {
  const int lane = (int)(threadIdx.x & 63);
  const uint64_t below = (1ull << lane) - 1ull;
  const int per = tl.tiles_x * tl.tiles_y;
  const int mh = (H + 7) >> 3, mw = (W + 7) >> 3;
  // the same trip count for every lane of a wave
  for (int base = (int)blockIdx.x * 256; base < tl.tiles; base += (int)gridDim.x * 256) {
    const int t = base + (int)threadIdx.x;
    const bool valid = t < tl.tiles;
    bool any = false;
    if (valid) {
      const int n = t / per, r = t - n * per, ty = r / tl.tiles_x, tx = r - ty * tl.tiles_x;
      const int y0 = max(ty * kTile - kReach, 0) >> 3;
      const int y1 = min(ty * kTile + kTile - 1 + kReach, H - 1) >> 3;
      const int x0 = max(tx * kTile - kReach, 0) >> 3;
      const int x1 = min(tx * kTile + kTile - 1 + kReach, W - 1) >> 3;
      const uint8_t* m = mask + (int64_t)n * mh * mw;
      // at most 4 x 4 blocks (rows 16 ty - kReach .. 16 ty + 15 + kReach
      // meet blocks 2 ty - 1 .. 2 ty + 2 when kReach <= 8): read as a fixed
      // 4 x 4 with indices clamped into the range
      // (repeats do not change the result), so every load is in flight at once
      uint8_t v[4][4];
#pragma unroll
      for (int dy = 0; dy < 4; ++dy)
#pragma unroll
        for (int dx = 0; dx < 4; ++dx)
          v[dy][dx] = m[min(y0 + dy, y1) * mw + min(x0 + dx, x1)];
#pragma unroll
      for (int dy = 0; dy < 4; ++dy)
#pragma unroll
        for (int dx = 0; dx < 4; ++dx) any |= v[dy][dx] != 0;
      if (!any && sum) sum[t] = 0.0;
    }
    const uint64_t hv = __ballot(valid && any), ev = __ballot(valid && !any);
    int hb = 0, eb = 0;
    if (lane == 0) {
      if (hv) hb = atomicAdd(&tl.count[0], __popcll(hv));
      if (ev) eb = atomicAdd(&tl.count[1], __popcll(ev));
    }
    hb = __shfl(hb, 0);
    eb = __shfl(eb, 0);
    if (valid && any) tl.list[hb + __popcll(hv & below)] = t;
    if (valid && !any) tl.list[tl.tiles - 1 - (eb + __popcll(ev & below))] = t;
  }
}

// Grid: tiles workgroups (enough whatever the split). The lists partition
// the array: entries below c = count[0] are tiles with content, every later
// entry an empty tile. Workgroup b < c runs the network on tile list[b];
// workgroup b >= c stores background (without a look at the input) for the
// kEmptyPerGroup empty entries c + (b - c) kEmptyPerGroup ..., and the
// workgroups past the last empty entry end at once. Workgroups are
// dispatched in grid order, so the tiles that run the network start first
// and the stores stream through the remaining slots beside them, in a
// handful of workgroups (each holds this kernel's 78 KB of LDS, two per
// CU, so every workgroup costs a slot). A tile of the first list whose
// exact input region turns out empty (the mask is per 8 x 8 block) is
// cleared as well: every tile's output is what a test of its own input
// region gives.
constexpr int kEmptyPerGroup = 8;
__global__ __launch_bounds__(256, 2) __attribute__((amdgpu_waves_per_eu(1, 2))) void
fused_forward_kernel(
    const float4* __restrict__ rgba, const float* __restrict__ depth, int H, int W,
    float inv_scale, const bf16x8* __restrict__ w0, const bf16x8* __restrict__ w1,
    const bf16x8* __restrict__ w2, const bf16x8* __restrict__ w3, const float* __restrict__ b0,
    const float* __restrict__ b1, const float* __restrict__ b2, const float* __restrict__ b3,
    float4* __restrict__ out, float* __restrict__ err, SumArgs sums, TileList tl) {
  const int b = (int)blockIdx.x;
  const int c = tl.count[0];
  const int per = tl.tiles_x * tl.tiles_y;
  if (b >= c) {  // empty tiles (their partial sums are already zero)
    const int64_t e0 = c + (int64_t)(b - c) * kEmptyPerGroup;
#pragma unroll
    for (int j = 0; j < kEmptyPerGroup; ++j) {
      if (e0 + j >= tl.tiles) break;  // the same for the whole workgroup
      const int t = tl.list[e0 + j];
      const int n = t / per, r = t - n * per;
      clear_tile(n, H, W, (r / tl.tiles_x) * kTile, (r % tl.tiles_x) * kTile, out, err);
    }
    return;
  }
  const int t = tl.list[b];
  const int n = t / per, r = t - n * per;
  const int ty0 = (r / tl.tiles_x) * kTile, tx0 = (r % tl.tiles_x) * kTile;
  const FusedLds l = fused_lds(fused_smem);
  bf16x8 wa[ksteps(8)], wb[ksteps(32)], wc[ksteps(32)];
  load_weights<8>(w0, wa);
  const bool any_nz = prep_region(rgba, depth, H, W, inv_scale, n, ty0, tx0, l.sV, l.nzf, l.sX);
  if (!__syncthreads_or(any_nz)) {
    clear_tile(n, H, W, ty0, tx0, out, err);
    if (sums.sum && threadIdx.x == 0) sums.sum[t] = 0.0;
    return;
  }
  const int qy = threadIdx.x / kTile, qx = threadIdx.x % kTile;
  const int y = ty0 + qy, x = tx0 + qx;
  const float zsum = fused_tile(l.sU, l.sV, l.sX, l.nzf, l.rowany, wa, wb, wc, w1, w2, w3, b0,
                                b1, b2, b3, n, H, W, ty0, tx0, qy, qx, y, x, out, err);
  if (sums.sum) tile_partial(sums, l.red, zsum, t);
}


// Training loss and its gradient with respect to o (bf16, 32 channels,
// zeros beyond the 20 used): per low-resolution pixel, its four
// full-resolution pixels. loss_sum[0] += the pixel's share.
__global__ __launch_bounds__(256) void loss_kernel(const float* o, const bf16* x0,
                                                   const float4* target, int N, int H, int W,
                                                   float err_weight, bf16* g, double* loss_sum) {
  const int64_t P = (int64_t)N * H * W;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const double Pf = 4.0 * (double)P;  // full-resolution pixels
  double part = 0.0;
  if (p < P) {
    const int n = (int)(p / ((int64_t)H * W));
    const int r = (int)(p - (int64_t)n * H * W), y = r / W, x = r - y * W;
    const float* op = o + p * kCh;
    float gv[kCh];
#pragma unroll
    for (int c = 0; c < kCh; ++c) gv[c] = 0.f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int sy = s >> 1, sx = s & 1;
      const float4 b = base_rgba(x0, n, H, W, y, x, sy, sx);
      const int64_t q = ((int64_t)n * 2 * H + 2 * y + sy) * (2 * W) + 2 * x + sx;
      const float4 t = target[q];
      const float d0 = b.x + op[5 * s] - t.x, d1 = b.y + op[5 * s + 1] - t.y,
                  d2 = b.z + op[5 * s + 2] - t.z, d3 = b.w + op[5 * s + 3] - t.w;
      const float e = sqrtf((d0 * d0 + d1 * d1 + d2 * d2) / 3.0f);
      const float z = op[5 * s + 4];
      // loss = sum d^2 / (4 Pf) + err_weight sum (z - e)^2 / Pf (e held constant)
      part += ((double)d0 * d0 + (double)d1 * d1 + (double)d2 * d2 + (double)d3 * d3) /
                  (4.0 * Pf) +
              (double)err_weight * ((double)(z - e) * (z - e)) / Pf;
      const float k = (float)(2.0 / (4.0 * Pf));
      gv[5 * s] = k * d0;
      gv[5 * s + 1] = k * d1;
      gv[5 * s + 2] = k * d2;
      gv[5 * s + 3] = k * d3;
      gv[5 * s + 4] = (float)(2.0 / Pf) * err_weight * (z - e);
    }
#pragma unroll
    for (int c = 0; c < kCh; ++c) g[p * kCh + c] = (bf16)gv[c];
  }
  __shared__ double red[256];
  red[threadIdx.x] = part;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss_sum) atomicAdd(loss_sum, red[0]);
}

// Weight-gradient partial sums of one workgroup over its pixel chunk:
// part[blk][t][ci][co] = sum_p x[p + off(t)][ci] g[p][co], and the bias
// part[blk][9 CIN 32 + co] = sum_p g[p][co]. 32-pixel tiles are staged in
// LDS (x gathered at the 9 taps, zero outside the image).
template <int CIN>
__global__ __launch_bounds__(256) void wgrad_kernel(const bf16* x, const bf16* g, int N, int H,
                                                    int W, int64_t chunk, float* part) {
  constexpr int PAIRS = CIN * kCh;           // (ci, co)
  constexpr int PER = (PAIRS + 255) / 256;   // pairs per thread
  __shared__ float sx[32][9][CIN];
  __shared__ float sg[32][kCh];
  const int64_t P = (int64_t)N * H * W;
  const int64_t begin = (int64_t)blockIdx.x * chunk, end = min(P, begin + chunk);
  float acc[PER][9];
  float bacc = 0.f;
#pragma unroll
  for (int k = 0; k < PER; ++k)
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[k][t] = 0.f;
  for (int64_t t0 = begin; t0 < end; t0 += 32) {
    const int cnt = (int)min<int64_t>(32, end - t0);
    __syncthreads();
    for (int i = threadIdx.x; i < 32 * 9 * CIN; i += 256) {
      const int pi = i / (9 * CIN), rem = i - pi * 9 * CIN, t = rem / CIN, ci = rem - t * CIN;
      float v = 0.f;
      if (pi < cnt) {
        const int64_t p = t0 + pi;
        const int n = (int)(p / ((int64_t)H * W));
        const int r = (int)(p - (int64_t)n * H * W), y = r / W + t / 3 - 1,
                  xx = r % W + t % 3 - 1;
        if (y >= 0 && y < H && xx >= 0 && xx < W)
          v = bf(x[(((int64_t)n * H + y) * W + xx) * CIN + ci]);
      }
      sx[pi][t][ci] = v;
    }
    for (int i = threadIdx.x; i < 32 * kCh; i += 256) {
      const int pi = i / kCh, co = i - pi * kCh;
      sg[pi][co] = pi < cnt ? bf(g[(t0 + pi) * kCh + co]) : 0.f;
    }
    __syncthreads();
    for (int pi = 0; pi < cnt; ++pi) {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int pair = threadIdx.x + 256 * k;
        if (pair >= PAIRS) continue;
        const int ci = pair / kCh, co = pair - ci * kCh;
        const float gv = sg[pi][co];
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[k][t] = fmaf(sx[pi][t][ci], gv, acc[k][t]);
      }
      if (threadIdx.x < kCh) bacc += sg[pi][threadIdx.x];
    }
  }
  float* out = part + (int64_t)blockIdx.x * (9 * PAIRS + kCh);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int pair = threadIdx.x + 256 * k;
    if (pair >= PAIRS) continue;
    const int ci = pair / kCh, co = pair - ci * kCh;
#pragma unroll
    for (int t = 0; t < 9; ++t) out[((int64_t)t * CIN + ci) * kCh + co] = acc[k][t];
  }
  if (threadIdx.x < kCh) out[9 * PAIRS + threadIdx.x] = bacc;
}

// grads[i] = sum over blocks (in order) of part[blk][i]
__global__ void reduce_kernel(const float* part, int blocks, int64_t n, float* grads) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int b = 0; b < blocks; ++b) s += part[(int64_t)b * n + i];
    grads[i] = s;
  }
}

// Adam on the FP32 master weights.
__global__ void adam_kernel(float* w, const float* g, float* m, float* v, int64_t n, float lr,
                            float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
  }
}

// Pack one layer's FP32 weights w[9][cin][32] into the GEMM layouts:
// forward fw[k / 8][co][k % 8], k = tap cin + ci (zero beyond 9 cin);
// backward (cin == 32 only) bw[k / 8][ci][k % 8], k = tap' 32 + co, with
// element w[8 - tap'][ci][co] (mirrored taps, swapped channel roles).
__global__ void pack_kernel(const float* w, int cin, bf16* fw, bf16* bw) {
  const int K = ((9 * cin + 31) / 32) * 32;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < K * kCh; i += gridDim.x * blockDim.x) {
    const int k = i / kCh, c = i - k * kCh;  // (k, output column)
    const int tap = k / cin, ci = k - tap * cin;
    const float f = k < 9 * cin ? w[((int64_t)tap * cin + ci) * kCh + c] : 0.f;
    fw[((int64_t)(k / 8) * kCh + c) * 8 + (k % 8)] = (bf16)f;
    if (bw && cin == kCh) {
      // column c is the input channel ci' of the backward conv, k = tap' 32 + co
      const int tp = k / kCh, co = k - tp * kCh;
      const float b = w[((int64_t)(8 - tp) * kCh + c) * kCh + co];
      bw[((int64_t)(k / 8) * kCh + c) * 8 + (k % 8)] = (bf16)b;
    }
  }
}

}  // namespace

}  // namespace sg

using namespace sg;

struct sg_upsampler {
  int device = 0;
  int64_t max_pixels = 0;
  float* params = nullptr;  // FP32 master weights (packed)
  float* grads = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  int64_t step = 0;
  bf16* fw[kLayers] = {};   // forward GEMM weights
  bf16* bw[kLayers] = {};   // backward-data GEMM weights (layers 1..3)
  bf16* x0 = nullptr;
  bf16* h[3] = {};          // hidden activations
  float* o = nullptr;
  bf16* ga = nullptr;       // gradient buffers
  bf16* gb = nullptr;
  float* part = nullptr;    // weight-gradient partial sums
  int part_blocks = 0;
  double* acc = nullptr;    // device doubles: loss, partials or sums, per-image results
  int64_t acc_n = 0;
  int32_t* tl = nullptr;    // tile-list counters [4] (zero between launches), list [max_pixels]
  uint8_t* mask = nullptr;  // content mask built from an input without one [max_pixels]
  bool packed = false;
  bool fused = true;        // inference through fused_forward_kernel
};

namespace {

void up_free(sg_upsampler* u) {
  void* ptrs[] = {u->params, u->grads, u->m,    u->v,   u->x0, u->o,
                  u->ga,     u->gb,    u->part, u->acc, u->tl, u->mask};
  for (void* p : ptrs)
    if (p) hipFree(p);
  for (int l = 0; l < kLayers; ++l) {
    if (u->fw[l]) hipFree(u->fw[l]);
    if (u->bw[l]) hipFree(u->bw[l]);
  }
  for (int i = 0; i < 3; ++i)
    if (u->h[i]) hipFree(u->h[i]);
  delete u;
}

int blocks_of(int64_t n, int per = 256) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, 1 << 20));
}

sg_status pack_weights(sg_upsampler* u, hipStream_t s) {
  for (int l = 0; l < kLayers; ++l) {
    const int K = kdim(kCin[l]);
    hipLaunchKernelGGL(pack_kernel, dim3(blocks_of((int64_t)K * kCh)), dim3(256), 0, s,
                       u->params + layer_off(l), kCin[l], u->fw[l], u->bw[l]);
  }
  SG_HIP(hipGetLastError());
  u->packed = true;
  return SG_OK;
}

template <int CIN, int EPI>
sg_status conv(const bf16* x, int N, int H, int W, const bf16* wt, const float* bias, void* out,
               const bf16* mask, hipStream_t s) {
  const int64_t waves = ((int64_t)N * H * W + 63) / 64;
  hipLaunchKernelGGL((conv_kernel<CIN, EPI>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s,
                     x, N, H, W, reinterpret_cast<const bf16x8*>(wt), bias, out, mask);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

sg_status check_batch(sg_upsampler* u, int32_t n, int32_t h, int32_t w, const float* rgba,
                      const float* depth) {
  if (!u || !rgba || !depth || n < 1 || h < 1 || w < 1)
    return fail(SG_ERR_INVALID_ARG, "upsampler: NULL input or empty batch");
  if ((int64_t)n * h * w > u->max_pixels)
    return fail(SG_ERR_INVALID_ARG, "upsampler: batch larger than max_pixels");
  return SG_OK;
}

// x0 and the forward pass (activations kept for the backward pass)
sg_status forward(sg_upsampler* u, int n, int h, int w, const float* rgba, const float* depth,
                  double depth_scale, hipStream_t s) {
  sg_status st;
  if (!u->packed && (st = pack_weights(u, s)) != SG_OK) return st;
  const int64_t P = (int64_t)n * h * w;
  hipLaunchKernelGGL(prep_kernel, dim3(blocks_of(P)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(rgba), depth, P, (float)(1.0 / depth_scale),
                     u->x0);
  SG_HIP(hipGetLastError());
  const float* b = u->params;
  if ((st = conv<8, kReluBf16>(u->x0, n, h, w, u->fw[0], b + layer_off(0) + 9 * 8 * kCh, u->h[0],
                               nullptr, s)) != SG_OK)
    return st;
  for (int l = 1; l < 3; ++l)
    if ((st = conv<32, kReluBf16>(u->h[l - 1], n, h, w, u->fw[l],
                                  b + layer_off(l) + 9 * 32 * kCh, u->h[l], nullptr, s)) != SG_OK)
      return st;
  return conv<32, kBiasF32>(u->h[2], n, h, w, u->fw[3], b + layer_off(3) + 9 * 32 * kCh, u->o,
                            nullptr, s);
}

template <int CIN>
sg_status wgrad(sg_upsampler* u, const bf16* x, const bf16* g, int n, int h, int w, int layer,
                hipStream_t s) {
  const int64_t P = (int64_t)n * h * w;
  const int blocks = (int)std::min<int64_t>(u->part_blocks, (P + 63) / 64);
  const int64_t chunk = (((P + blocks - 1) / blocks + 63) / 64) * 64;
  const int used = (int)((P + chunk - 1) / chunk);
  hipLaunchKernelGGL(wgrad_kernel<CIN>, dim3(used), dim3(256), 0, s, x, g, n, h, w, chunk,
                     u->part);
  const int64_t nn = layer_size(layer);
  hipLaunchKernelGGL(reduce_kernel, dim3(blocks_of(nn)), dim3(256), 0, s, u->part, used, nn,
                     u->grads + layer_off(layer));
  SG_HIP(hipGetLastError());
  return SG_OK;
}

sg_status gradients(sg_upsampler* u, int n, int h, int w, const float* rgba, const float* depth,
                    double depth_scale, const float* target, double err_weight, hipStream_t s) {
  sg_status st = forward(u, n, h, w, rgba, depth, depth_scale, s);
  if (st != SG_OK) return st;
  const int64_t P = (int64_t)n * h * w;
  SG_HIP(hipMemsetAsync(u->acc, 0, sizeof(double), s));
  hipLaunchKernelGGL(loss_kernel, dim3(blocks_of(P)), dim3(256), 0, s, u->o, u->x0,
                     reinterpret_cast<const float4*>(target), n, h, w, (float)err_weight, u->ga,
                     u->acc);
  SG_HIP(hipGetLastError());
  // layer 4 (input h3), then back through the ReLUs
  bf16* g = u->ga;
  bf16* gn = u->gb;
  for (int l = 3; l >= 1; --l) {
    if ((st = wgrad<32>(u, u->h[l - 1], g, n, h, w, l, s)) != SG_OK) return st;
    if ((st = conv<32, kMaskBf16>(g, n, h, w, u->bw[l], nullptr, gn, u->h[l - 1], s)) != SG_OK)
      return st;
    std::swap(g, gn);
  }
  return wgrad<8>(u, u->x0, g, n, h, w, 0, s);
}

// Inference into out_rgba / out_err; with sums, the per-image sums of the
// predicted squared error end up in acc[1 + max_pixels ..] (and, with a
// fallback flag, the frame's decision in *fallback), added in a fixed order
// from per-workgroup partials that every launch overwrites.
sg_status infer(sg_upsampler* up, int32_t n, int32_t h, int32_t w, const float* rgba,
                const float* depth, const uint8_t* content, double depth_scale,
                float* out_rgba, float* out_err, bool sums, int32_t* fallback,
                double threshold_db, hipStream_t s) {
  sg_status st = check_batch(up, n, h, w, rgba, depth);
  if (st != SG_OK) return st;
  if (!out_rgba || !(std::isfinite(depth_scale) && depth_scale > 0.0))
    return fail(SG_ERR_INVALID_ARG, "sg_up_forward: NULL output or bad depth_scale");
  DeviceGuard guard(up->device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  SumArgs sa{};
  if (sums) {
    sa.sum = up->acc + 1;  // per-workgroup partials
    sa.result = up->acc + 1 + up->max_pixels;
    sa.fallback = fallback;
    sa.images = n;
    sa.pixels = 4.0 * (double)h * w;
    sa.threshold_db = threshold_db;
  }
  if (up->fused) {
    if (!up->packed && (st = pack_weights(up, s)) != SG_OK) return st;
    const float* b = up->params;
    // tiles <= n h w <= max_pixels: one list entry and one partial slot each
    TileList tl;
    tl.tiles_x = (w + kTile - 1) / kTile;
    tl.tiles_y = (h + kTile - 1) / kTile;
    tl.tiles = (int32_t)((int64_t)n * tl.tiles_x * tl.tiles_y);
    tl.count = up->tl;
    tl.list = up->tl + 4;
    sa.tiles = tl.tiles_x * tl.tiles_y;
    sa.reset = up->tl;
    const float4* in4 = reinterpret_cast<const float4*>(rgba);
    if (!content) {
      const int mh = (h + 7) / 8, mw = (w + 7) / 8;
      const int64_t blocks = (int64_t)n * mh * mw;  // <= max_pixels
      hipLaunchKernelGGL(content_mask_kernel, dim3(blocks_of(blocks, 4)), dim3(256), 0, s, in4,
                         depth, h, w, blocks, mh, mw, up->mask);
      content = up->mask;
    }
    hipLaunchKernelGGL(tile_list_kernel, dim3(blocks_of(tl.tiles)), dim3(256), 0, s, content, h,
                       w, tl, sums ? sa.sum : nullptr);
    const bf16x8* fw0 = reinterpret_cast<const bf16x8*>(up->fw[0]);
    const bf16x8* fw1 = reinterpret_cast<const bf16x8*>(up->fw[1]);
    const bf16x8* fw2 = reinterpret_cast<const bf16x8*>(up->fw[2]);
    const bf16x8* fw3 = reinterpret_cast<const bf16x8*>(up->fw[3]);
    const float *b0 = b + layer_off(0) + 9 * 8 * kCh, *b1 = b + layer_off(1) + 9 * 32 * kCh,
                *b2 = b + layer_off(2) + 9 * 32 * kCh, *b3 = b + layer_off(3) + 9 * 32 * kCh;
    SG_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(fused_forward_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedLds));
    hipLaunchKernelGGL(fused_forward_kernel, dim3((unsigned)tl.tiles), dim3(256), kFusedLds, s, in4,
                       depth, h, w, (float)(1.0 / depth_scale), fw0, fw1, fw2, fw3, b0, b1, b2,
                       b3, reinterpret_cast<float4*>(out_rgba), out_err, sa, tl);
    // per-image sums and the decision when asked; always the counters' reset
    if (!sums) sa.images = 0;
    hipLaunchKernelGGL(tile_sum_kernel, dim3(1), dim3(kSumThreads), 0, s, sa);
    SG_HIP(hipGetLastError());
  } else {
    if ((st = forward(up, n, h, w, rgba, depth, depth_scale, s)) != SG_OK) return st;
    // chunks of 256 pixels per image: n * chunks <= n * h * w <= max_pixels
    // partial slots
    const int64_t chunks = ((int64_t)h * w + 255) / 256;
    sa.tiles = (int32_t)chunks;
    const dim3 grid((unsigned)chunks, (unsigned)std::min<int32_t>(n, 65535));
    hipLaunchKernelGGL(shuffle_kernel, grid, dim3(256), 0, s, up->o, up->x0, n, h, w,
                       reinterpret_cast<float4*>(out_rgba), out_err, sums ? sa.sum : nullptr);
    if (sums) hipLaunchKernelGGL(tile_sum_kernel, dim3(1), dim3(kSumThreads), 0, s, sa);
    SG_HIP(hipGetLastError());
  }
  return SG_OK;
}

}  // namespace

extern "C" {

int64_t sg_up_param_count(void) { return kParams; }

sg_status sg_up_create(int32_t device, int64_t max_pixels, sg_upsampler** out) {
  if (!out || max_pixels < 1 || max_pixels > ((int64_t)1 << 30))
    return fail(SG_ERR_INVALID_ARG, "sg_up_create: bad arguments");
  *out = nullptr;
  DeviceGuard guard(device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "sg_up_create: cannot select device");
  sg_upsampler* u = new sg_upsampler;
  u->device = device;
  u->max_pixels = max_pixels;
  u->part_blocks = 512;
  // loss, partials or sums [max_pixels] (a tile holds at least one pixel),
  // results [max_pixels]
  u->acc_n = 2 + 2 * max_pixels;
  bool ok = true;
  auto al = [&](void** p, int64_t bytes) {
    ok = ok && hipMalloc(p, (size_t)std::max<int64_t>(bytes, 16)) == hipSuccess;
  };
  al((void**)&u->params, kParams * 4);
  al((void**)&u->grads, kParams * 4);
  al((void**)&u->m, kParams * 4);
  al((void**)&u->v, kParams * 4);
  for (int l = 0; l < kLayers; ++l) {
    al((void**)&u->fw[l], (int64_t)kdim(kCin[l]) * kCh * 2);
    if (kCin[l] == kCh) al((void**)&u->bw[l], (int64_t)kdim(kCh) * kCh * 2);
  }
  al((void**)&u->x0, max_pixels * 8 * 2);
  for (int i = 0; i < 3; ++i) al((void**)&u->h[i], max_pixels * kCh * 2);
  al((void**)&u->o, max_pixels * kCh * 4);
  al((void**)&u->ga, max_pixels * kCh * 2);
  al((void**)&u->gb, max_pixels * kCh * 2);
  al((void**)&u->part, (int64_t)u->part_blocks * (9 * 32 * kCh + kCh) * 4);
  al((void**)&u->acc, u->acc_n * 8);
  al((void**)&u->tl, (4 + max_pixels) * 4);
  al((void**)&u->mask, max_pixels);
  if (!ok) {
    up_free(u);
    (void)hipGetLastError();
    return fail(SG_ERR_OUT_OF_MEMORY, "sg_up_create: device allocation failed");
  }
  if (hipMemset(u->params, 0, kParams * 4) != hipSuccess ||
      hipMemset(u->m, 0, kParams * 4) != hipSuccess ||
      hipMemset(u->v, 0, kParams * 4) != hipSuccess ||
      hipMemset(u->acc, 0, (size_t)u->acc_n * 8) != hipSuccess ||
      hipMemset(u->tl, 0, 16) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    up_free(u);
    return fail(SG_ERR_DEVICE, "sg_up_create: initialisation failed");
  }
  *out = u;
  return SG_OK;
}

sg_status sg_up_destroy(sg_upsampler* up) {
  if (!up) return fail(SG_ERR_INVALID_ARG, "sg_up_destroy: NULL");
  DeviceGuard guard(up->device);
  (void)hipDeviceSynchronize();
  up_free(up);
  return SG_OK;
}

sg_status sg_up_set_weights(sg_upsampler* up, const float* params, int64_t n) {
  if (!up || !params || n != kParams) return fail(SG_ERR_INVALID_ARG, "sg_up_set_weights");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return fail(SG_ERR_INVALID_ARG, "weights must be finite");
  DeviceGuard guard(up->device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  SG_HIP(hipMemcpy(up->params, params, (size_t)n * 4, hipMemcpyHostToDevice));
  SG_HIP(hipMemset(up->m, 0, kParams * 4));
  SG_HIP(hipMemset(up->v, 0, kParams * 4));
  up->step = 0;
  up->packed = false;
  return SG_OK;
}

sg_status sg_up_get_weights(sg_upsampler* up, float* params, int64_t n) {
  if (!up || !params || n != kParams) return fail(SG_ERR_INVALID_ARG, "sg_up_get_weights");
  DeviceGuard guard(up->device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  SG_HIP(hipDeviceSynchronize());
  SG_HIP(hipMemcpy(params, up->params, (size_t)n * 4, hipMemcpyDeviceToHost));
  return SG_OK;
}

sg_status sg_up_forward(sg_upsampler* up, int32_t n, int32_t h, int32_t w, const float* rgba,
                        const float* depth, const uint8_t* content, double depth_scale,
                        float* out_rgba, float* out_err, double* mse_pred, void* hip_stream) {
  hipStream_t s = (hipStream_t)hip_stream;
  sg_status st = infer(up, n, h, w, rgba, depth, content, depth_scale, out_rgba, out_err,
                       mse_pred != nullptr, nullptr, 0.0, s);
  if (st != SG_OK) return st;
  if (mse_pred) {
    DeviceGuard guard(up->device);
    SG_HIP(hipMemcpyAsync(mse_pred, up->acc + 1 + up->max_pixels, sizeof(double) * n,
                          hipMemcpyDeviceToHost, s));
    SG_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i) mse_pred[i] /= 4.0 * (double)h * w;
  }
  return SG_OK;
}

sg_status sg_up_forward_flag(sg_upsampler* up, int32_t n, int32_t h, int32_t w,
                             const float* rgba, const float* depth, const uint8_t* content,
                             double depth_scale, float* out_rgba, float* out_err,
                             double threshold_db, int32_t* fallback, void* hip_stream) {
  if (!fallback || std::isnan(threshold_db))
    return fail(SG_ERR_INVALID_ARG, "sg_up_forward_flag: NULL flag or NaN threshold");
  return infer(up, n, h, w, rgba, depth, content, depth_scale, out_rgba, out_err, true, fallback,
               threshold_db, (hipStream_t)hip_stream);
}

sg_status sg_up_gradients(sg_upsampler* up, int32_t n, int32_t h, int32_t w, const float* rgba,
                          const float* depth, double depth_scale, const float* target,
                          double err_weight, float* grads, double* loss, void* hip_stream) {
  sg_status st = check_batch(up, n, h, w, rgba, depth);
  if (st != SG_OK) return st;
  if (!target || !(std::isfinite(depth_scale) && depth_scale > 0.0) || !std::isfinite(err_weight))
    return fail(SG_ERR_INVALID_ARG, "sg_up_gradients: NULL target or bad scalars");
  DeviceGuard guard(up->device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  hipStream_t s = (hipStream_t)hip_stream;
  if ((st = gradients(up, n, h, w, rgba, depth, depth_scale, target, err_weight, s)) != SG_OK)
    return st;
  if (grads) SG_HIP(hipMemcpyAsync(grads, up->grads, kParams * 4, hipMemcpyDeviceToHost, s));
  if (loss) SG_HIP(hipMemcpyAsync(loss, up->acc, sizeof(double), hipMemcpyDeviceToHost, s));
  if (grads || loss) SG_HIP(hipStreamSynchronize(s));
  return SG_OK;
}

sg_status sg_up_train_step(sg_upsampler* up, int32_t n, int32_t h, int32_t w, const float* rgba,
                           const float* depth, double depth_scale, const float* target,
                           double err_weight, double lr, double* loss, void* hip_stream) {
  if (!(std::isfinite(lr) && lr > 0.0)) return fail(SG_ERR_INVALID_ARG, "sg_up_train_step: lr");
  sg_status st = sg_up_gradients(up, n, h, w, rgba, depth, depth_scale, target, err_weight,
                                 nullptr, loss, hip_stream);
  if (st != SG_OK) return st;
  DeviceGuard guard(up->device);
  hipStream_t s = (hipStream_t)hip_stream;
  up->step += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)up->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)up->step)));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_of(kParams)), dim3(256), 0, s, up->params,
                     up->grads, up->m, up->v, kParams, (float)lr, c1, c2);
  SG_HIP(hipGetLastError());
  return pack_weights(up, s);
}

sg_status sg_up_set_fused(sg_upsampler* up, int32_t fused) {
  if (!up) return fail(SG_ERR_INVALID_ARG, "sg_up_set_fused: NULL upsampler");
  up->fused = fused != 0;
  return SG_OK;
}

sg_status sg_up_read_buffer(sg_upsampler* up, int32_t which, void* host, int64_t bytes) {
  if (!up || !host || which < 0 || which > 4 || bytes < 0)
    return fail(SG_ERR_INVALID_ARG, "sg_up_read_buffer: bad arguments");
  const void* src[5] = {up->x0, up->h[0], up->h[1], up->h[2], up->o};
  const int64_t cap = which == 0 ? up->max_pixels * 8 * 2
                      : which == 4 ? up->max_pixels * kCh * 4
                                   : up->max_pixels * kCh * 2;
  if (bytes > cap) return fail(SG_ERR_INVALID_ARG, "sg_up_read_buffer: more than the buffer");
  DeviceGuard guard(up->device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  SG_HIP(hipDeviceSynchronize());
  SG_HIP(hipMemcpy(host, src[which], (size_t)bytes, hipMemcpyDeviceToHost));
  return SG_OK;
}

}  // extern "C"
