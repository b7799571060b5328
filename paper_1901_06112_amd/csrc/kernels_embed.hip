// Range embedding (Section III): the cross kernel B(i, x) = k(c_i, p(x))
// (Eq. (defB)) mixed by the FP64 landmark factor F = Q diag(alpha^{-1/2}),
//     u_k(x) = sum_i F[i][k] exp(-|p(x) - c_i|^2 / (2 sigma_r^2)),
// so that u(x).u(y) = b(x)^T A^+ b(y) = K_hat(x, y) (Eqs. (hatK), (vk)).  The
// planes u_k are written planar ([r_eff][N] float32) for the convolution pass.
// Also the per-channel centring offset f0 of the image.
//
// Precision: squared distances are formed in FP64 from the FP32 guide and
// landmarks (exact differences), b = exp(-d^2 / (2 sigma_r^2)) is evaluated
// and kept in FP64, and the r x r_eff mix accumulates in FP64, so the stored
// u_k carries a single FP32 rounding even where F^T b cancels.
#include <hip/hip_runtime.h>
#include <string.h>
#include <float.h>
#include <math.h>

#include <algorithm>

#include "device_common.h"

namespace nkf {

namespace {

constexpr int kBlock = 256;

// Register block of the generic distance pass: clusters per pass.
constexpr int kEmbedRB = 8;

// ct64[d][k] = (double) c[k][d], rows padded to RP = r rounded up to
// kEmbedRB with zeros.
__global__ void transpose_landmarks64_kernel(const float *__restrict__ c, int r, int D, int RP,
                                             double *__restrict__ ct64) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D * RP) return;
  const int d = e / RP, k = e - d * RP;
  ct64[e] = k < r ? (double)c[k * D + d] : 0.0;
}

// Blocks of BT threads (512 for the generic form, whose LDS tile leaves room
// for one or two blocks per CU, so that each SIMD still holds two waves or
// more) on tiles of TPX pixels (64, or 32 when the FP64 b tile of 64 pixels
// would not fit in LDS); thread group kg (a wave when TPX = 64, a half-wave
// when 32) takes landmarks [kg CW, (kg + 1) CW) in the distance pass and
// output planes 8 kg, 8 kg + 8 NG, ... in the mix.
// DS > 0 (D == DS <= 4): the pixel's guide values are held in FP64 registers
// and the landmarks in FP64 in LDS, so a distance term is one subtraction and
// one FMA.  DS == 0: the distances run over kEmbedRB landmarks at a time with
// the transposed FP64 landmarks ct64, eight independent FMA chains per lane.
// An explicit or self guide is staged as float [D][TPX]; a patch guide takes
// tiles of TPX pixels within one image row and stages only the window they
// share, [2 pr + 1][TPX + 2 pr][C] (mirrored at the borders), walking the
// patch dimensions d = (dy T + dx) C + c in that order.
template <int TPX, int DS, int BT>
__global__ __launch_bounds__(BT) void embed_kernel(Guide g, int64_t N, const float *__restrict__ c,
                                                   const double *__restrict__ ct64, int RP, int r,
                                                   const double *__restrict__ F, int r_eff, double inv2s2,
                                                   float *__restrict__ u, double *__restrict__ u64) {
  constexpr int NG = BT / TPX;
  extern __shared__ double smem_d[];
  const int D = g.D;
  double *bs = smem_d;                                              // [r][TPX]
  float *pt = reinterpret_cast<float *>(smem_d + (size_t)r * TPX);  // [D][TPX], or the patch window
  double *c64 = smem_d + (size_t)r * TPX;                           // DS > 0: [r][DS], in place of pt
  const int tid = threadIdx.x;
  const int px = tid & (TPX - 1);
  const int kg = TPX == kWave ? __builtin_amdgcn_readfirstlane(tid / TPX) : tid / TPX;
  const bool patch = DS == 0 && g.kind == GUIDE_PATCH;
  if constexpr (DS > 0) {
    for (int e = tid; e < r * DS; e += BT) c64[e] = (double)c[e];
  }
  const int T = 2 * g.pr + 1, WW = TPX + T - 1;
  const int nch = (g.W + TPX - 1) / TPX;
  const int64_t ntiles = patch ? (int64_t)g.H * nch : (N + TPX - 1) / TPX;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    int64_t x;
    bool valid;
    int ty = 0, tx0 = 0;
    if (patch) {
      ty = (int)(tile / nch);
      tx0 = (int)(tile - (int64_t)ty * nch) * TPX;
      x = (int64_t)ty * g.W + tx0 + px;
      valid = tx0 + px < g.W;
    } else {
      x = tile * TPX + px;
      valid = x < N;
    }
    __syncthreads();
    if constexpr (DS > 0) {
      double pv[DS > 0 ? DS : 1];
#pragma unroll
      for (int d = 0; d < DS; ++d) pv[d] = valid ? (double)guide_elem(g, x, d) : 0.0;
      // two landmarks in flight per thread hide the FP64 exponential's latency
#pragma unroll 2
      for (int k = kg; k < r; k += NG) {
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < DS; ++d) {
          const double t = pv[d] - c64[k * DS + d];
          acc = fma(t, t, acc);
        }
        bs[k * TPX + px] = exp_neg64(acc * inv2s2);
      }
    } else {
      if (patch) {
        // window rows ty - pr .. ty + pr, columns tx0 - pr .. tx0 + TPX - 1 + pr;
        // columns past W - 1 + pr feed no valid pixel and are left at zero
        const int rowlen = WW * g.C;
        for (int e = tid; e < T * rowlen; e += BT) {
          const int wr = e / rowlen, rem = e - wr * rowlen;
          const int wc = rem / g.C, ch = rem - wc * g.C;
          const int xs = tx0 - g.pr + wc;
          float v = 0.0f;
          if (xs < g.W + g.pr) {
            const int yy = sym_index(ty - g.pr + wr, g.H), xq = sym_index(xs, g.W);
            v = g.f[((int64_t)yy * g.W + xq) * g.C + ch];
          }
          pt[e] = v;
        }
      } else {
        for (int e = tid; e < D * TPX; e += BT) {
          const int d = e / TPX, q = e - d * TPX;
          const int64_t xe = tile * TPX + q;
          pt[e] = xe < N ? guide_elem(g, xe, d) : 0.0f;
        }
      }
      __syncthreads();
      const int CW = ((r + NG - 1) / NG + kEmbedRB - 1) / kEmbedRB * kEmbedRB;
      const int k1 = min(r, (kg + 1) * CW);
      for (int j0 = kg * CW; j0 < k1; j0 += kEmbedRB) {
        double acc[kEmbedRB];
#pragma unroll
        for (int q = 0; q < kEmbedRB; ++q) acc[q] = 0.0;
        // runs of dimensions that are evenly spaced in the staged tile and
        // consecutive in ct64: a patch row (T C values, d = (dy T + dx) C + c)
        // per dy, else all D
        const int runs = patch ? T : 1, run = patch ? T * g.C : D;
        const int wstride = patch ? 1 : TPX;
        for (int rw = 0; rw < runs; ++rw) {
          const float *wp = patch ? pt + (rw * WW + px) * g.C : pt + px;
          const double *crow = ct64 + (size_t)rw * run * RP + j0;
#pragma unroll 4
          for (int e = 0; e < run; ++e) {
            const double v = (double)wp[e * wstride];
            const double *cr = crow + (size_t)e * RP;
#pragma unroll
            for (int q = 0; q < kEmbedRB; ++q) {
              const double t = v - cr[q];
              acc[q] = fma(t, t, acc[q]);
            }
          }
        }
#pragma unroll
        for (int q = 0; q < kEmbedRB; ++q)
          if (j0 + q < k1) bs[(j0 + q) * TPX + px] = exp_neg64(acc[q] * inv2s2);
      }
    }
    __syncthreads();
    // thread group kg mixes output planes kb .. kb+7 (kb = 8 kg, 8 kg + 8 NG, ...):
    // one b read and one contiguous row segment of F per k feed 8 FMA chains
    for (int kb = 8 * kg; kb < r_eff; kb += 8 * NG) {
      double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (kb + 8 <= r_eff) {
        // generic form: unrolled so that several F row segments (scalar loads)
        // are in flight together (no gain for D <= 4)
        constexpr int kMixUnroll = DS == 0 ? 4 : 1;
#pragma unroll kMixUnroll
        for (int k = 0; k < r; ++k) {
          const double bv = bs[k * TPX + px];
          const double *Fr = F + (size_t)k * r_eff + kb;
#pragma unroll
          for (int q = 0; q < 8; ++q) acc[q] = fma(Fr[q], bv, acc[q]);
        }
      } else {
        for (int k = 0; k < r; ++k) {
          const double bv = bs[k * TPX + px];
          const double *Fr = F + (size_t)k * r_eff + kb;
#pragma unroll
          for (int q = 0; q < 8; ++q)
            if (kb + q < r_eff) acc[q] = fma(Fr[q], bv, acc[q]);
        }
      }
      if (valid) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (kb + q < r_eff) {
            if (u64)
              u64[(int64_t)(kb + q) * N + x] = acc[q];
            else
              u[(int64_t)(kb + q) * N + x] = (float)acc[q];
          }
      }
    }
  }
}

__device__ __forceinline__ unsigned ord_encode(float v) {
  const unsigned b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord_decode(unsigned k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
static float ord_decode_host(unsigned k) {
  const unsigned b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  float v;
  memcpy(&v, &b, sizeof v);
  return v;
}

// The C <= 4 path keeps kMmReps copies of the (min, max) words, each copy
// in its own 128-byte slot, so that the per-block atomics of a launch spread
// over kMmReps cache lines instead of queueing on one.
constexpr int kMmReps = 32, kMmSlot = 32;

__global__ void mm_init_reps_kernel(unsigned *mm, int C) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMmReps * kMmSlot) mm[i] = i % kMmSlot < C ? 0xffffffffu : 0u;
}

__global__ void mm_init_kernel(unsigned *mm, int C) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < C) {
    mm[i] = 0xffffffffu;  // running min (encoded)
    mm[C + i] = 0u;       // running max (encoded)
  }
}

// C <= 4 with a 16-byte aligned f: the N*C floats as float4 groups of
// G = lcm(4, C) / 4 vectors (whole pixels, so the channel of every component
// is known at compile time), four groups in flight per thread, per-channel
// min / max in registers, then wave and block reductions and one pair of
// atomics per channel and block.  The last N*C mod 4G floats are read one by one.
template <int C>
__global__ __launch_bounds__(256) void minmax_small_kernel(const float *__restrict__ f, int64_t total,
                                                           unsigned *mm) {
  constexpr int G = C == 3 ? 3 : 1;
  constexpr int FG = 4 * G;  // floats per group
  constexpr int UNR = 4;
  __shared__ unsigned slo[4][C], shi[4][C];
  unsigned lo[C], hi[C];
#pragma unroll
  for (int c = 0; c < C; ++c) lo[c] = 0xffffffffu, hi[c] = 0u;
  const float4 *f4 = reinterpret_cast<const float4 *>(f);
  const int64_t ngroups = total / FG;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; g + (UNR - 1) * stride < ngroups; g += UNR * stride) {
    float4 v[UNR][G];
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int j = 0; j < G; ++j) v[u][j] = f4[(g + u * stride) * G + j];
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const float e[4] = {v[u][j].x, v[u][j].y, v[u][j].z, v[u][j].w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int c = (4 * j + t) % C;
          const unsigned k = ord_encode(e[t]);
          lo[c] = min(lo[c], k);
          hi[c] = max(hi[c], k);
        }
      }
  }
  for (; g < ngroups; g += stride)
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const float4 q = f4[g * G + j];
      const float e[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = (4 * j + t) % C;
        const unsigned k = ord_encode(e[t]);
        lo[c] = min(lo[c], k);
        hi[c] = max(hi[c], k);
      }
    }
  // tail floats (fewer than FG), by the first threads of block 0
  if (blockIdx.x == 0 && threadIdx.x < FG) {
    const int64_t e = ngroups * FG + threadIdx.x;
    if (e < total) {
      const unsigned k = ord_encode(f[e]);
#pragma unroll
      for (int c = 0; c < C; ++c)
        if ((int)(e % C) == c) lo[c] = min(lo[c], k), hi[c] = max(hi[c], k);
    }
  }
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1) {
      lo[c] = min(lo[c], (unsigned)__shfl_xor((int)lo[c], m, kWave));
      hi[c] = max(hi[c], (unsigned)__shfl_xor((int)hi[c], m, kWave));
    }
    if (lane == 0) slo[w][c] = lo[c], shi[w][c] = hi[c];
  }
  __syncthreads();
  if (threadIdx.x < C) {
    const int c = threadIdx.x;
    unsigned a = slo[0][c], b = shi[0][c];
    for (int q = 1; q < (int)(blockDim.x / kWave); ++q) a = min(a, slo[q][c]), b = max(b, shi[q][c]);
    unsigned *slot = mm + (blockIdx.x % kMmReps) * kMmSlot;
    atomicMin(&slot[c], a);
    atomicMax(&slot[C + c], b);
  }
}

// Block size is a multiple of C, so a thread's channel is fixed.
__global__ void minmax_kernel(const float *__restrict__ f, int64_t total, int C, unsigned *mm) {
  extern __shared__ unsigned sm[];
  const int B = blockDim.x;
  const int tid = threadIdx.x;
  unsigned lo = 0xffffffffu, hi = 0u;
  for (int64_t e = (int64_t)blockIdx.x * B + tid; e < total; e += (int64_t)gridDim.x * B) {
    const unsigned k = ord_encode(f[e]);
    lo = min(lo, k);
    hi = max(hi, k);
  }
  sm[tid] = lo;
  sm[B + tid] = hi;
  __syncthreads();
  if (tid < C) {
    for (int m = tid + C; m < B; m += C) {
      lo = min(lo, sm[m]);
      hi = max(hi, sm[B + m]);
    }
    atomicMin(&mm[tid], lo);
    atomicMax(&mm[C + tid], hi);
  }
}

__global__ void center_final_kernel(const unsigned *mm, int C, float *f0, int use_value, float value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C) return;
  if (use_value) {
    f0[i] = value;
  } else {
    const double lo = ord_decode(mm[i]), hi = ord_decode(mm[C + i]);
    f0[i] = (float)(0.5 * (lo + hi));
  }
}

// The replicated layout of the C <= 4 path: wave c reduces channel c over
// the kMmReps slots, one slot per lane.
__global__ __launch_bounds__(256) void center_final_reps_kernel(const unsigned *mm, int C, float *f0) {
  const int c = threadIdx.x / kWave, q = threadIdx.x % kWave;
  if (c >= C) return;
  unsigned a = q < kMmReps ? mm[q * kMmSlot + c] : 0xffffffffu;
  unsigned b = q < kMmReps ? mm[q * kMmSlot + C + c] : 0u;
#pragma unroll
  for (int m = kWave / 2; m >= 1; m >>= 1) {
    a = min(a, (unsigned)__shfl_xor((int)a, m, kWave));
    b = max(b, (unsigned)__shfl_xor((int)b, m, kWave));
  }
  if (q == 0) f0[c] = (float)(0.5 * ((double)ord_decode(a) + (double)ord_decode(b)));
}

}  // namespace

hipError_t launch_center(const float *f, int64_t N, int C, double center, float *f0, unsigned *mm,
                         hipStream_t s) {
  const int cb = (C + 255) / 256;
  if (isfinite(center)) {
    hipLaunchKernelGGL(center_final_kernel, dim3(cb), dim3(256), 0, s, mm, C, f0, 1, (float)center);
    return hipGetLastError();
  }
  hipError_t e;
  const int64_t total = N * C;
  if (C <= 4 && (reinterpret_cast<uintptr_t>(f) & 15) == 0) {
    hipLaunchKernelGGL(mm_init_reps_kernel, dim3(kMmReps * kMmSlot / 256), dim3(256), 0, s, mm, C);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int blocks = (int)std::min<int64_t>(std::max<int64_t>((total / 16 + 255) / 256, 1), 1024);
    switch (C) {
      case 1: hipLaunchKernelGGL(minmax_small_kernel<1>, dim3(blocks), dim3(256), 0, s, f, total, mm); break;
      case 2: hipLaunchKernelGGL(minmax_small_kernel<2>, dim3(blocks), dim3(256), 0, s, f, total, mm); break;
      case 3: hipLaunchKernelGGL(minmax_small_kernel<3>, dim3(blocks), dim3(256), 0, s, f, total, mm); break;
      default: hipLaunchKernelGGL(minmax_small_kernel<4>, dim3(blocks), dim3(256), 0, s, f, total, mm); break;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(center_final_reps_kernel, dim3(1), dim3(256), 0, s, mm, C, f0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(mm_init_kernel, dim3(cb), dim3(256), 0, s, mm, C);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int B = C <= 256 ? C * (256 / C) : C;
  int64_t blocks = (total + (int64_t)B * 16 - 1) / ((int64_t)B * 16);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(minmax_kernel, dim3((int)blocks), dim3(B), 2 * B * sizeof(unsigned), s, f, total, C, mm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(center_final_kernel, dim3(cb), dim3(256), 0, s, mm, C, f0, 0, 0.0f);
  return hipGetLastError();
}

size_t center_scratch_words(int C) { return C <= 4 ? (size_t)kMmReps * kMmSlot : 2 * (size_t)C; }

// eta_hat statistics: st[0] = pixels that took the eta_hat <= 0 / non-finite
// guard, st[1] = ord_encode(min eta_hat over the other pixels).
// Landmark Gram matrix A[i][j] = k(c_i, c_j) (Eq. (defA)) in FP64 on the
// device, so that only A crosses to the host for the eigendecomposition:
// one thread per entry (i, j), squared distance from the FP32 landmarks in
// four partial sums over d mod 4 added in a fixed order.
__global__ __launch_bounds__(256) void gram_kernel(const float *__restrict__ c, int r, int D, double inv2s2,
                                                   double *__restrict__ A) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= r * r) return;
  const int i = e / r, j = e - (e / r) * r;
  if (i == j) {
    A[e] = 1.0;
    return;
  }
  const float *ci = c + (size_t)i * D, *cj = c + (size_t)j * D;
  double d4[4] = {0.0, 0.0, 0.0, 0.0};
  int k = 0;
  for (; k + 4 <= D; k += 4)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double t = (double)ci[k + q] - (double)cj[k + q];
      d4[q] = fma(t, t, d4[q]);
    }
  for (; k < D; ++k) {
    const double t = (double)ci[k] - (double)cj[k];
    d4[0] = fma(t, t, d4[0]);
  }
  A[e] = exp_neg64(((d4[0] + d4[1]) + (d4[2] + d4[3])) * inv2s2);
}

hipError_t launch_landmark_gram(const float *c, int r, int D, double sigma_r, double *A, hipStream_t s) {
  const double inv = isinf(sigma_r) ? 0.0 : 1.0 / (2.0 * sigma_r * sigma_r);
  hipLaunchKernelGGL(gram_kernel, dim3((r * r + 255) / 256), dim3(256), 0, s, c, r, D, inv, A);
  return hipGetLastError();
}

__global__ void eta_stats_init_kernel(unsigned *st) {
  if (threadIdx.x == 0) {
    st[0] = 0u;
    st[1] = 0xffffffffu;
  }
}

__global__ __launch_bounds__(256) void eta_stats_kernel(const float *__restrict__ eta, int64_t N, unsigned *st) {
  unsigned cnt = 0u, mn = 0xffffffffu;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
    const float e = eta[x];
    if (e > 0.0f && isfinite(e))
      mn = min(mn, ord_encode(e));
    else
      ++cnt;
  }
#pragma unroll
  for (int m = kWave / 2; m >= 1; m >>= 1) {
    cnt += (unsigned)__shfl_xor((int)cnt, m, kWave);
    mn = min(mn, (unsigned)__shfl_xor((int)mn, m, kWave));
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (cnt) atomicAdd(&st[0], cnt);
    atomicMin(&st[1], mn);
  }
}

hipError_t launch_eta_stats(const float *eta, int64_t N, unsigned *st, hipStream_t s) {
  hipLaunchKernelGGL(eta_stats_init_kernel, dim3(1), dim3(64), 0, s, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t blocks = (N + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(eta_stats_kernel, dim3((unsigned)blocks), dim3(256), 0, s, eta, N, st);
  return hipGetLastError();
}

double eta_stats_min(unsigned code) { return code == 0xffffffffu ? NAN : (double)ord_decode_host(code); }

size_t embed_scratch_doubles(const Guide &g, int r) {
  const bool small = g.D <= 4 && g.kind != GUIDE_PATCH;
  return small ? 0 : (size_t)g.D * (size_t)((r + kEmbedRB - 1) / kEmbedRB * kEmbedRB);
}

hipError_t launch_embed(const Guide &g, const float *c, int r, const double *F, int r_eff, double sigma_r,
                        float *u, double *ct64, hipStream_t s, double *u64) {
  const int64_t N = (int64_t)g.H * g.W;
  const double inv2s2 = isinf(sigma_r) ? 0.0 : 1.0 / (2.0 * sigma_r * sigma_r);
  // DS > 0 keeps the landmarks as FP64 [r][D] where the generic form stages the guide tile
  const bool small = g.D <= 4 && g.kind != GUIDE_PATCH;
  const bool patch = g.kind == GUIDE_PATCH;
  const int T = 2 * g.pr + 1;
  auto lds = [&](int tpx) {
    const size_t stage = small ? sizeof(double) * r * g.D
                         : patch ? sizeof(float) * T * (tpx + T - 1) * g.C
                                 : sizeof(float) * g.D * tpx;
    return sizeof(double) * r * tpx + stage;
  };
  const bool wide = lds(64) <= 160 * 1024;
  const int tpx = wide ? 64 : 32;
  const size_t sm = lds(tpx);
  int64_t blocks = patch ? (int64_t)g.H * ((g.W + tpx - 1) / tpx) : (N + tpx - 1) / tpx;
  if (blocks > 16384) blocks = 16384;
  const int ds = small ? g.D : 0;
  const int key = (wide ? 100 : 0) + ds;
  const int RP = (r + kEmbedRB - 1) / kEmbedRB * kEmbedRB;
  hipError_t e = hipSuccess;
  if (!small) {
    hipLaunchKernelGGL(transpose_landmarks64_kernel, dim3((g.D * RP + 255) / 256), dim3(256), 0, s, c, r, g.D, RP,
                       ct64);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  switch (key) {
#define NKF_EMBED(K, T, DSV)                                                                                  \
  case K:                                                                                                     \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(embed_kernel<T, DSV, DSV ? 256 : 512>),            \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);                             \
    if (e != hipSuccess) return e;                                                                            \
    hipLaunchKernelGGL((embed_kernel<T, DSV, DSV ? 256 : 512>), dim3((unsigned)blocks), dim3(DSV ? 256 : 512), \
                       sm, s, g, N, c, ct64, RP, r, F, r_eff, inv2s2, u, u64);                                \
    break;
    NKF_EMBED(100, 64, 0) NKF_EMBED(101, 64, 1) NKF_EMBED(102, 64, 2) NKF_EMBED(103, 64, 3) NKF_EMBED(104, 64, 4)
    NKF_EMBED(0, 32, 0) NKF_EMBED(1, 32, 1) NKF_EMBED(2, 32, 2) NKF_EMBED(3, 32, 3) NKF_EMBED(4, 32, 4)
#undef NKF_EMBED
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nkf
