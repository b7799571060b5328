// Backward of the fast filter with landmarks and window radius held fixed.
//
// The paper defines only the forward filter (Section III, Algorithm 1); its
// adjoint follows by differentiating that computation.  In embedding form
// (u = F^T b, b_j(x) = k(c_j, p(x)), F F^T = A^+), with G = dL/dg:
//   a_c = G_c / eta,  beta = -sum_c G_c g~_c / eta                  (ab_kernel)
//   du_dir_k = beta E_k + sum_c a_c Z_kc                            (MODE_DUDIR)
//   du_k = du_dir_k + w*(beta u_k) + sum_c f~_c w*(a_c u_k)         (MODE_ADJ)
//   df_c = sum_k u_k w*(a_c u_k)                                    (MODE_ADJ)
//   db = F du,  dp = -sum_j db_j b_j (p - c_j) / sigma_r^2           (reduce_kernel)
//   dL/dsigma_r (through b) = sum_x sum_j db_j b_j |p - c_j|^2 / sigma_r^3
//   R = sum_x b(x) du_dir(x)^T  -> dL/dsigma_r through A^{-1} on the host
//   dL/dsigma_s = sum_x sum_k u_k [beta (w'*u_k) + sum_c a_c (w'*(u_k f~_c))]
//     with w' = w1'(x)w1 + w1(x)w1', w1'(t) = w1(t) t^2 / sigma_s^3    (MODE_SIGS)
// The convolution passes reuse the streaming FIR of conv_core.h; the r_eff (C+1)
// planes are recomputed rather than stored.
#include <hip/hip_runtime.h>
#include <math.h>

#include "conv_core.h"

namespace nkf {

namespace {

using namespace conv;

// a_c and beta per pixel, [N][4] = (beta, a_0, a_1, a_2); zero where the
// forward took the eta <= 0 guard (the output there is f itself).
__global__ void ab_kernel(int64_t N, int C, const float *__restrict__ G, const float *__restrict__ out,
                          const float *__restrict__ eta, const float *__restrict__ f0,
                          float *__restrict__ ab) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
    const float e = eta[x];
    float r[4] = {0.f, 0.f, 0.f, 0.f};
    if (e > 0.0f && isfinite(e)) {
      const float inv = 1.0f / e;
      float beta = 0.0f;
      for (int c = 0; c < C; ++c) {
        const float g = G[x * C + c];
        r[1 + c] = g * inv;
        beta = fmaf(g, out[x * C + c] - f0[c], beta);
      }
      r[0] = -beta * inv;
    }
    reinterpret_cast<float4 *>(ab)[x] = make_float4(r[0], r[1], r[2], r[3]);
  }
}

constexpr int kRBlock = 256;
constexpr int kRTile = 64;

// exp(-z) for z >= 0 in FP64.
__device__ __forceinline__ double exp_neg64(double z) { return exp(-z); }

// Per 64-pixel tile: b (FP64), db = F du, dp, the sigma_r-through-b sum and
// the block's share of R = sum_x b du_dir^T.  LDS layout (doubles unless
// noted): bs[r][64], d2s[r][64], wj[r][64] (= db_j b_j / sigma_r^2), then the
// block's R accumulator [r * r_eff], then floats pt[D][64], du[r_eff][64],
// dud[r_eff][64].
__global__ __launch_bounds__(kRBlock) void reduce_kernel(Guide g, int64_t N, const float *__restrict__ c, int r,
                                                         const double *__restrict__ F, int r_eff, double sigma_r,
                                                         const float *__restrict__ du, const float *__restrict__ dud,
                                                         float *__restrict__ dp, int want_R,
                                                         double *__restrict__ partials) {
  extern __shared__ double sm[];
  const int D = g.D;
  double *bs = sm;
  double *d2s = bs + (size_t)r * kRTile;
  double *wj = d2s + (size_t)r * kRTile;
  double *Rl = wj + (size_t)r * kRTile;
  const int nR = want_R ? r * r_eff : 0;
  double *red = Rl + nR;                                     // [256]
  float *pt = reinterpret_cast<float *>(red + kRBlock);      // [D][64]
  float *dus = pt + (size_t)D * kRTile;                      // [r_eff][64]
  float *duds = dus + (size_t)r_eff * kRTile;                // [r_eff][64]
  const int tid = threadIdx.x;
  const int px = tid & (kRTile - 1);
  const int kg = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double inv2s2 = 1.0 / (2.0 * sigma_r * sigma_r);
  const double inv_s2 = 1.0 / (sigma_r * sigma_r);
  const double inv_s3 = inv_s2 / sigma_r;
  for (int e = tid; e < nR; e += kRBlock) Rl[e] = 0.0;
  double sr_acc = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * kRTile; base < N; base += (int64_t)gridDim.x * kRTile) {
    __syncthreads();
    for (int e = tid; e < D * kRTile; e += kRBlock) {
      const int d = e / kRTile, q = e - d * kRTile;
      const int64_t x = base + q;
      pt[e] = x < N ? guide_elem(g, x, d) : 0.0f;
    }
    for (int e = tid; e < r_eff * kRTile; e += kRBlock) {
      const int k = e / kRTile, q = e - k * kRTile;
      const int64_t x = base + q;
      dus[e] = x < N ? du[(int64_t)k * N + x] : 0.0f;
      duds[e] = x < N ? dud[(int64_t)k * N + x] : 0.0f;
    }
    __syncthreads();
    const bool valid = base + px < N;
    for (int j = kg; j < r; j += 4) {
      double d2 = 0.0;
      for (int d = 0; d < D; ++d) {
        const double t = (double)pt[d * kRTile + px] - (double)c[j * D + d];
        d2 = fma(t, t, d2);
      }
      const double b = valid ? exp_neg64(d2 * inv2s2) : 0.0;
      double db = 0.0;
      for (int k = 0; k < r_eff; ++k) db = fma(F[j * r_eff + k], (double)dus[k * kRTile + px], db);
      bs[j * kRTile + px] = b;
      d2s[j * kRTile + px] = d2;
      wj[j * kRTile + px] = db * b * inv_s2;
      sr_acc = fma(db * b, d2 * inv_s3, sr_acc);
    }
    __syncthreads();
    // dp_d = -sum_j w_j (p_d - c_jd)
    if (dp) {
      for (int d = kg; d < D; d += 4) {
        const double pd = pt[d * kRTile + px];
        double s = 0.0;
        for (int j = 0; j < r; ++j) s = fma(wj[j * kRTile + px], pd - (double)c[j * D + d], s);
        const int64_t x = base + px;
        if (x < N) dp[x * D + d] = (float)(-s);
      }
    }
    // R[j][k] += sum_px b_j du_dir_k  (each entry owned by one thread)
    for (int e = tid; e < nR; e += kRBlock) {
      const int j = e / r_eff, k = e - j * r_eff;
      double s = Rl[e];
      for (int q = 0; q < kRTile; ++q) s = fma(bs[j * kRTile + q], (double)duds[k * kRTile + q], s);
      Rl[e] = s;
    }
  }
  __syncthreads();
  red[tid] = sr_acc;
  __syncthreads();
  for (int h = kRBlock / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  double *dst = partials + (size_t)blockIdx.x * (nR + 1);
  if (tid == 0) dst[0] = red[0];
  for (int e = tid; e < nR; e += kRBlock) dst[1 + e] = Rl[e];
}

template <int MODE>
hipError_t launch_mode(ConvArgs a, int S, hipStream_t s, int *nblocks) {
  switch (S) {
#define NKF_CASE(SV) \
  case SV:           \
    return launch_one<SV, 4, true, 16, MODE>(a, s, 3, 1, 512, nblocks);
    NKF_CASE(0) NKF_CASE(1) NKF_CASE(2) NKF_CASE(3) NKF_CASE(4) NKF_CASE(5) NKF_CASE(6) NKF_CASE(7)
    NKF_CASE(8) NKF_CASE(9) NKF_CASE(10) NKF_CASE(11) NKF_CASE(12) NKF_CASE(13) NKF_CASE(14)
    NKF_CASE(15) NKF_CASE(16)
#undef NKF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

int bwd_conv_max_blocks(int H, int W) {
  // launch_one uses at least one 16-row chunk per tile
  return ((W + conv::kTW - 1) / conv::kTW) * ((H + 15) / 16);
}

hipError_t launch_bwd_ab(int64_t N, int C, const float *G, const float *out, const float *eta, const float *f0,
                         float *ab, hipStream_t s) {
  int64_t blocks = (N + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(ab_kernel, dim3((int)blocks), dim3(256), 0, s, N, C, G, out, eta, f0, ab);
  return hipGetLastError();
}

hipError_t launch_bwd_conv(const BwdConvProblem &pb, hipStream_t s) {
  ConvArgs a{};
  a.H = pb.H;
  a.W = pb.W;
  a.C = pb.C;
  a.r_eff = pb.r_eff;
  a.f = pb.f;
  a.f0 = pb.f0;
  a.u = pb.u;
  a.ab = pb.ab;
  a.plane_in = pb.plane_in;
  a.plane_out = pb.plane_out;
  a.df = pb.df;
  a.G = pb.G;
  a.eta = pb.eta;
  a.partials = pb.partials;
  for (int t = 0; t < 2 * kMaxRadius + 1; ++t) {
    a.wr[t] = (double)pb.wr.w[t];
    a.wc[t] = (double)pb.wc.w[t];
  }
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (pb.mode) {
    case 1: e = launch_mode<MODE_DUDIR>(a, pb.S, s, &nb); break;
    case 2: e = launch_mode<MODE_SIGS>(a, pb.S, s, &nb); break;
    case 3: e = launch_mode<MODE_ADJ>(a, pb.S, s, &nb); break;
    default: break;
  }
  if (pb.nblocks_out) *pb.nblocks_out = nb;
  return e;
}

int bwd_reduce_blocks(int64_t N) {
  int64_t b = (N + kRTile - 1) / kRTile;
  return (int)(b < 1024 ? b : 1024);
}

size_t bwd_reduce_lds(int r, int r_eff, int D, int want_R) {
  return sizeof(double) * (3 * (size_t)r * kRTile + (want_R ? (size_t)r * r_eff : 0) + kRBlock) +
         sizeof(float) * ((size_t)D + 2 * (size_t)r_eff) * kRTile;
}

hipError_t launch_bwd_reduce(const Guide &g, const float *c, int r, const double *F, int r_eff, double sigma_r,
                             const float *du, const float *dud, float *dp, int want_R, double *partials,
                             hipStream_t s) {
  const int64_t N = (int64_t)g.H * g.W;
  const size_t sm = bwd_reduce_lds(r, r_eff, g.D, want_R);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(reduce_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_kernel, dim3(bwd_reduce_blocks(N)), dim3(kRBlock), sm, s, g, N, c, r, F, r_eff, sigma_r,
                     du, dud, dp, want_R, partials);
  return hipGetLastError();
}

}  // namespace nkf
