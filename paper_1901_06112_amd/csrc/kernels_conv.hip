// Forward convolutions + contraction + normalisation (Section III,
// Eqs. (finalnum), (finalden); Algorithm 1 accumulation loop).  The kernel
// body is in conv_core.h; this file instantiates it for every window radius
// and picks the plane grouping from the channel count.
#include <hip/hip_runtime.h>

#include "conv_core.h"

namespace nkf {

namespace {

using namespace conv;

// f [N][C] -> fpl [C][N] through a 32 x 32 LDS tile (coalesced on both sides)
__global__ __launch_bounds__(256) void planar_kernel(const float *__restrict__ f, int64_t N, int C,
                                                     float *__restrict__ fpl) {
  __shared__ float t[32][33];
  const int64_t x0 = (int64_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int i = ty; i < 32; i += 8) {
    const int64_t x = x0 + i;
    const int c = c0 + tx;
    t[i][tx] = (x < N && c < C) ? f[x * C + c] : 0.0f;
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int c = c0 + i;
    const int64_t x = x0 + tx;
    if (c < C && x < N) fpl[(int64_t)c * N + x] = t[tx][i];
  }
}

template <int S>
hipError_t launch_S(ConvArgs a, hipStream_t s) {
  const int C = a.C;
  if (C == 1) return launch_one<S, 2, true, 32, MODE_FWD>(a, s, 1, 1);
  if (C <= 3) return launch_one<S, 4, true, 32, MODE_FWD, 512>(a, s, 3, 1);
  // eta pass, then channel chunks that read eta (and f as planes)
  hipError_t e = launch_one<S, 1, true, 32, MODE_FWD>(a, s, 0, 1);
  if (e != hipSuccess) return e;
  ConvArgs b = a;
  b.eta_out = nullptr;
  if (a.fpl) {
    const int64_t N = (int64_t)a.H * a.W;
    hipLaunchKernelGGL(planar_kernel, dim3((unsigned)((N + 31) / 32), (unsigned)((a.C + 31) / 32)), dim3(256), 0, s,
                       a.f, N, a.C, const_cast<float *>(a.fpl));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return launch_one<S, 4, false, 32, MODE_FWD, 512>(b, s, 4, (C + 3) / 4);
}

}  // namespace

hipError_t launch_conv_contract(const ConvProblem &pb, hipStream_t s) {
  ConvArgs a{};
  a.H = pb.H;
  a.W = pb.W;
  a.C = pb.C;
  a.r_eff = pb.r_eff;
  a.f = pb.f;
  a.f0 = pb.f0;
  a.u = pb.u;
  a.out = pb.out;
  a.eta_out = pb.eta_out;
  a.eta_buf = pb.eta_buf;
  a.fpl = pb.C > 3 ? pb.f_planar : nullptr;
  a.force_nch = pb.force_nch;
  for (int t = 0; t < 2 * kMaxRadius + 1; ++t) a.wr[t] = a.wc[t] = (double)pb.taps.w[t];
  switch (pb.S) {
#define NKF_CASE(SV) \
  case SV:           \
    return launch_S<SV>(a, s);
    NKF_CASE(0) NKF_CASE(1) NKF_CASE(2) NKF_CASE(3) NKF_CASE(4) NKF_CASE(5) NKF_CASE(6) NKF_CASE(7)
    NKF_CASE(8) NKF_CASE(9) NKF_CASE(10) NKF_CASE(11) NKF_CASE(12) NKF_CASE(13) NKF_CASE(14)
    NKF_CASE(15) NKF_CASE(16)
#undef NKF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace nkf
