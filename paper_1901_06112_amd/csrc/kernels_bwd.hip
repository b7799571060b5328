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
constexpr int kRMaxJ = 16;   // landmarks per thread group (r <= 64)
constexpr int kRS = kRTile + 1;  // padded row stride of the b and du_dir tiles

typedef double double4_t __attribute__((ext_vector_type(4)));

// Per 64-pixel tile: b (FP64), db = F du, dp, the sigma_r-through-b sum and
// the block's share of R = sum_x b du_dir^T.  Thread (px, kg) evaluates the
// landmarks j = kg + 4 m in registers.  R runs on v_mfma_f64_16x16x4f64:
// A = b^T (16 landmarks x 4 pixels), B = du_dir (4 pixels x 16 planes); wave w
// keeps the output tiles w, w + 4, ... of R in registers for the whole launch
// (lane l, element i holds R[16 jt + l/16 + 4 i][16 kt + l%16]).
// LDS (doubles): bs[r][65], wj[r][64] (= db_j b_j / sigma_r^2), red[256],
// Fs[r_eff][4][NJ] (Fs[k][kg][m] = F[kg + 4 m][k], so that the db loop reads
// its F values from LDS, one broadcast read per pair, instead of one scalar
// load and wait per value); floats: pt[D][64], dus[r_eff][64], duds[r_eff][65].
// NJ: landmarks per thread group rounded up (8 or 16), the length of the
// register-blocked loops, so that the accumulators are updated without
// branches (a landmark past r contributes zero).
template <int NJ>
__global__ __launch_bounds__(kRBlock) void reduce_kernel(Guide g, int64_t N, const float *__restrict__ c, int r,
                                                         const double *__restrict__ F, int r_eff, double sigma_r,
                                                         const float *__restrict__ du, const float *__restrict__ dud,
                                                         float *__restrict__ dp, int want_R,
                                                         double *__restrict__ partials) {
  extern __shared__ double sm[];
  const int D = g.D;
  double *bs = sm;
  double *wj = bs + (size_t)r * kRS;
  double *red = wj + (size_t)r * kRTile;                     // [256]
  double *Fs = red + kRBlock;                                // [r_eff][4][NJ]
  float *pt = reinterpret_cast<float *>(Fs + (size_t)4 * NJ * r_eff);  // [D][64]
  float *dus = pt + (size_t)D * kRTile;                      // [r_eff][64]
  float *duds = dus + (size_t)r_eff * kRTile;                // [r_eff][65]
  const int tid = threadIdx.x, lane = tid & 63;
  const int px = tid & (kRTile - 1);
  const int kg = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nj = (r - kg + 3) / 4;  // landmarks j = kg + 4 m of this thread group
  const double inv2s2 = 1.0 / (2.0 * sigma_r * sigma_r);
  const double inv_s2 = 1.0 / (sigma_r * sigma_r);
  const double inv_s3 = inv_s2 / sigma_r;
  const int ntj = (r + 15) / 16, ntk = (r_eff + 15) / 16;
  const int nt = want_R ? ntj * ntk : 0;
  const int nq = nt > kg ? min(4, (nt - kg + 3) / 4) : 0;  // R tiles kg + 4 q of this wave
  double4_t racc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) racc[q] = double4_t{0.0, 0.0, 0.0, 0.0};
  double sr_acc = 0.0;
  for (int e = tid; e < 4 * NJ * r_eff; e += kRBlock) {
    const int k = e / (4 * NJ), rem = e - k * 4 * NJ, q = rem / NJ, m = rem - q * NJ;
    const int j = q + 4 * m;
    Fs[e] = j < r ? F[(size_t)j * r_eff + k] : 0.0;
  }  // ordered before its first use by the barrier after the tile staging
  for (int64_t base = (int64_t)blockIdx.x * kRTile; base < N; base += (int64_t)gridDim.x * kRTile) {
    // stage the tile: thread (px, kg) takes planes k = kg + 4 q of its pixel;
    // every load is issued before the first LDS store, so a tile costs one
    // memory latency
    {
      const int64_t x = base + px;
      const bool xin = x < N;
      float vdu[NJ], vdud[NJ];
      // out-of-range planes and pixels load plane 0 / the last pixel (always
      // in bounds, no branch around the loads) and are zeroed afterwards
      const int64_t xc = xin ? x : N - 1;
#pragma unroll
      for (int q = 0; q < NJ; ++q) {
        const int k = kg + 4 * q;
        const bool ok = xin && k < r_eff;
        const int64_t o = (int64_t)(k < r_eff ? k : 0) * N + xc;
        const float a = du[o], b = dud[o];
        vdu[q] = ok ? a : 0.0f;
        vdud[q] = ok ? b : 0.0f;
      }
      __syncthreads();
      for (int d = kg; d < D; d += 4) pt[d * kRTile + px] = xin ? guide_elem(g, x, d) : 0.0f;
#pragma unroll
      for (int q = 0; q < NJ; ++q) {
        const int k = kg + 4 * q;
        if (k < r_eff) {
          dus[k * kRTile + px] = vdu[q];
          duds[k * kRS + px] = vdud[q];
        }
      }
    }
    __syncthreads();
    const bool valid = base + px < N;
    // db_j = sum_k F[j][k] du_k for this thread's landmarks: each du_k read once
    double db[NJ];
#pragma unroll
    for (int m = 0; m < NJ; ++m) db[m] = 0.0;
    for (int k = 0; k < r_eff; ++k) {
      const double duk = (double)dus[k * kRTile + px];
      const double *fk = Fs + (size_t)(4 * k + kg) * NJ;
#pragma unroll
      for (int m = 0; m < NJ; ++m) db[m] = fma(fk[m], duk, db[m]);
    }
#pragma unroll
    for (int m = 0; m < NJ; ++m) {
      if (m >= nj) continue;
      const int j = kg + 4 * m;
      double d2 = 0.0;
      for (int d = 0; d < D; ++d) {
        const double t = (double)pt[d * kRTile + px] - (double)c[j * D + d];
        d2 = fma(t, t, d2);
      }
      const double b = valid ? exp_neg64(d2 * inv2s2) : 0.0;
      bs[j * kRS + px] = b;
      wj[j * kRTile + px] = db[m] * b * inv_s2;
      sr_acc = fma(db[m] * b, d2 * inv_s3, sr_acc);
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
    // R tiles on the matrix cores, 4 pixels per step, two accumulation chains
    // per tile; the wave's tile count (uniform) picks a loop of fixed length
    auto rtiles = [&](auto qc) {
      constexpr int Q = decltype(qc)::value;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int t = kg + 4 * q;
        const int jt = t / ntk, kt = t - jt * ntk;
        const int ja = 16 * jt + (lane & 15), kb = 16 * kt + (lane & 15);
        // rows past r (r_eff) read row 0 and are zeroed after the load: no
        // branch around the loads
        const bool aok = ja < r, bok = kb < r_eff;
        const double *arow = bs + (aok ? ja : 0) * kRS + (lane >> 4);
        const float *brow = duds + (bok ? kb : 0) * kRS + (lane >> 4);
        double4_t a1 = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int s4 = 0; s4 < kRTile / 4; s4 += 2) {
          const double av0 = aok ? arow[4 * s4] : 0.0;
          const double bv0 = bok ? (double)brow[4 * s4] : 0.0;
          const double av1 = aok ? arow[4 * s4 + 4] : 0.0;
          const double bv1 = bok ? (double)brow[4 * s4 + 4] : 0.0;
          racc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av0, bv0, racc[q], 0, 0, 0);
          a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av1, bv1, a1, 0, 0, 0);
        }
        racc[q] += a1;
      }
    };
    switch (nq) {
      case 4: rtiles(std::integral_constant<int, 4>{}); break;
      case 3: rtiles(std::integral_constant<int, 3>{}); break;
      case 2: rtiles(std::integral_constant<int, 2>{}); break;
      case 1: rtiles(std::integral_constant<int, 1>{}); break;
      default: break;
    }
  }
  __syncthreads();
  red[tid] = sr_acc;
  __syncthreads();
  for (int h = kRBlock / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  const int nR = want_R ? r * r_eff : 0;
  double *dst = partials + (size_t)blockIdx.x * (nR + 1);
  if (tid == 0) dst[0] = red[0];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t = kg + 4 * q;
    if (t >= nt) break;
    const int jt = t / ntk, kt = t - jt * ntk;
    const int k = 16 * kt + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = 16 * jt + (lane >> 4) + 4 * i;
      if (j < r && k < r_eff) dst[1 + j * r_eff + k] = racc[q][i];
    }
  }
}

template <int MODE>
hipError_t launch_mode(ConvArgs a, int S, hipStream_t s, int *nblocks) {
  switch (S) {
  // the fused sigma_s pass holds two tap sets; past S = 10 (past S = 8 when
  // it also forms du_dir) it takes 16-row chunks so that its row windows
  // (RUN + 2S values) still fit in registers
#define NKF_CASE(SV)                                                               \
  case SV:                                                                         \
    if constexpr ((MODE == MODE_SIGS && SV > 10) || (MODE == MODE_DS && SV > 8))   \
      return launch_one<SV, 4, true, 16, MODE, 512>(a, s, 3, 1, nblocks);      \
    else                                                                           \
      return launch_one<SV, 4, true, 32, MODE, 512>(a, s, 3, 1, nblocks);
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
  // launch_one uses at least one 32-row chunk per tile (bound kept at 16 rows)
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
  a.force_nch = pb.force_nch;
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
    case 4: e = launch_mode<MODE_DS>(a, pb.S, s, &nb); break;
    default: break;
  }
  if (pb.nblocks_out) *pb.nblocks_out = nb;
  return e;
}

int bwd_reduce_blocks(int64_t N) {
  int64_t b = (N + kRTile - 1) / kRTile;
  return (int)(b < 1024 ? b : 1024);
}

static int reduce_nj(int r) { return r <= 32 ? 8 : kRMaxJ; }

size_t bwd_reduce_lds(int r, int r_eff, int D, int want_R) {
  (void)want_R;
  return sizeof(double) * ((size_t)r * kRS + (size_t)r * kRTile + kRBlock + (size_t)4 * reduce_nj(r) * r_eff) +
         sizeof(float) * ((size_t)D * kRTile + (size_t)r_eff * kRTile + (size_t)r_eff * kRS);
}

// out[grp][e] = in[b0][e] + in[b0 + 1][e] + ... over the rows b0 = grp * group
// .. min(nrows, b0 + group) - 1, added in row order.
__global__ void sum_rows_kernel(const double *__restrict__ in, int nrows, int width, int group,
                                double *__restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= width) return;
  const int b0 = blockIdx.y * group, b1 = min(nrows, b0 + group);
  double s = 0.0;
  for (int b = b0; b < b1; ++b) s += in[(size_t)b * width + e];
  out[(size_t)blockIdx.y * width + e] = s;
}

constexpr int kSumGroup = 32;

size_t bwd_sum_scratch_doubles(int nrows, int width) {
  return (size_t)((nrows + kSumGroup - 1) / kSumGroup + 1) * width;
}

const double *launch_bwd_sum_partials(const double *partials, int nrows, int width, double *scratch,
                                      hipStream_t s, hipError_t *err) {
  const int ngroups = (nrows + kSumGroup - 1) / kSumGroup;
  const dim3 blk(256), g1((width + 255) / 256, ngroups), g2((width + 255) / 256, 1);
  double *out = scratch + (size_t)ngroups * width;
  hipLaunchKernelGGL(sum_rows_kernel, g1, blk, 0, s, partials, nrows, width, kSumGroup, scratch);
  if ((*err = hipGetLastError()) != hipSuccess) return nullptr;
  hipLaunchKernelGGL(sum_rows_kernel, g2, blk, 0, s, scratch, ngroups, width, ngroups, out);
  *err = hipGetLastError();
  return out;
}

hipError_t launch_bwd_reduce(const Guide &g, const float *c, int r, const double *F, int r_eff, double sigma_r,
                             const float *du, const float *dud, float *dp, int want_R, double *partials,
                             hipStream_t s) {
  const int64_t N = (int64_t)g.H * g.W;
  if (r < 1 || r > 4 * kRMaxJ) return hipErrorInvalidValue;
  const size_t sm = bwd_reduce_lds(r, r_eff, g.D, want_R);
  auto launch = [&](auto kern) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(bwd_reduce_blocks(N)), dim3(kRBlock), sm, s, g, N, c, r, F, r_eff, sigma_r, du,
                       dud, dp, want_R, partials);
    return hipGetLastError();
  };
  return reduce_nj(r) == 8 ? launch(reduce_kernel<8>) : launch(reduce_kernel<kRMaxJ>);
}

}  // namespace nkf
