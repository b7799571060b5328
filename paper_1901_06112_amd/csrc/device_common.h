// Device helpers shared by the HIP kernels (guide access, wave reductions,
// XCD-aware block order).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nkf_internal.h"

namespace nkf {

constexpr int kWave = 64;

// numpy-style symmetric padding index: -1 -> 0, n -> n-1 (valid for |pad| <= n).
__device__ __forceinline__ int sym_index(int i, int n) {
  if (i < 0) return -i - 1;
  if (i >= n) return 2 * n - i - 1;
  return i;
}

// Guide value p(x)[d] for pixel x (linear index).
__device__ __forceinline__ float guide_elem(const Guide &g, int64_t x, int d) {
  if (g.kind == GUIDE_EXPLICIT) return g.p[x * g.D + d];
  if (g.kind == GUIDE_SELF) return g.f[x * g.C + d];
  const int T = 2 * g.pr + 1;
  const int c = d % g.C;
  const int q = d / g.C;
  const int dx = q % T - g.pr;
  const int dy = q / T - g.pr;
  const int y = (int)(x / g.W), xx = (int)(x - (int64_t)y * g.W);
  const int yy = sym_index(y + dy, g.H), xq = sym_index(xx + dx, g.W);
  return g.f[((int64_t)yy * g.W + xq) * g.C + c];
}

// exp(-z) for z >= 0 to FP64 accuracy: z = n ln2 - r with n = round(z / ln2)
// and |r| <= ln2 / 2, ln2 split in two parts (the high part has 21
// significant bits, so n * ln2_hi is exact for the n that occur); exp(r) from
// its Taylor polynomial of degree 13 (truncation below 5e-18 relative), then
// a scale by 2^-n.  FP64 accuracy matters when F has large entries: the mix
// u = F^T b cancels, and an FP32 rounding of each b_j would move u_k by up to
// eps sum_j |F_jk| b_j instead of eps |u_k|.
// Branch-free: arguments past the underflow point (and NaN) run the same
// instructions on 0 and select 0 at the end, so lanes never diverge here.
__device__ __forceinline__ double exp_neg64(double z) {
  const bool ok = z < 745.0;
  const double zc = ok ? z : 0.0;
  const double n = rint(zc * 1.4426950408889634);
  const double r = (n * 0.6931467056274414 - zc) + n * 4.7493250390316726e-07;
  double q = 1.6059043836821613e-10;  // 1 / 13!
  q = fma(q, r, 2.08767569878681e-09);
  q = fma(q, r, 2.505210838544172e-08);
  q = fma(q, r, 2.755731922398589e-07);
  q = fma(q, r, 2.7557319223985893e-06);
  q = fma(q, r, 2.48015873015873e-05);
  q = fma(q, r, 0.0001984126984126984);
  q = fma(q, r, 0.001388888888888889);
  q = fma(q, r, 0.008333333333333333);
  q = fma(q, r, 0.041666666666666664);
  q = fma(q, r, 0.16666666666666666);
  q = fma(q, r, 0.5);
  q = fma(q, r, 1.0);
  q = fma(q, r, 1.0);
  return ok ? ldexp(q, -(int)n) : 0.0;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Map the hardware block id to a logical tile id so that each XCD
// receives a contiguous range of logical tiles; neighbouring tiles then share
// halo rows through the same L2.
__device__ __forceinline__ int xcd_swizzle(int b, int nb) {
  constexpr int kXcd = 8;
  const int per = nb / kXcd, rem = nb % kXcd;
  const int xcd = b % kXcd, idx = b / kXcd;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

}  // namespace nkf
