// Windowed Nystrom-kernel filter for many channels on the matrix cores: Eq.
// (num1) with the range kernel replaced by its Nystrom approximation
// K_hat(x, y) = u(x).u(y) (Eq. (hatK), u = F^T b), evaluated per window
// before the sum switch of Eqs. (finalnum), (finalden):
//     eta_hat(x) = sum_y w(x - y) K_hat(x, y),
//     zeta(x)    = sum_y w(x - y) K_hat(x, y) (f(y) - f0),
//     g_hat(x)   = f0 + zeta(x) / eta_hat(x)      (eta_hat <= 0: f(x)).
// The FIR form convolves r_eff (C + 1) planes; this form costs two GEMMs per
// window, K_hat = U_keys U_queries^T and zeta = W_t^T F_keys, whose size
// grows with r_eff + C instead of r_eff C, which pays for hyperspectral
// cubes.  It serves the 16-bit precision forms (BF16 or FP16 operands, FP32
// accumulation): the embedding values enter as 16-bit hi + lo pairs (three
// MFMA passes, hi.hi + lo.hi + hi.lo), the weighted kernel values
// w(x - y) K_hat(x, y) and the centred image values as single 16-bit values,
// and eta_hat is summed in FP32 from the unrounded weighted values.
//
// Tiles.  A block (8 waves, two per SIMD) owns 8 query rows by 32 query
// columns: two 16-column halves; wave w takes half w & 1 and rows
// (w >> 1) + 4j, j = 0, 1, so each wave carries two 16-query units whose
// query operands stay in registers for the whole launch.  The block walks the
// 8 + 2S key rows its windows reach; each key row's 64 columns
// [x0 - 16, x0 + 48) (S <= 16) are staged in LDS (embedding hi/lo pixel-major,
// centred image channel-major), double-buffered, the next row's loads in
// flight while the current one is used.  Per key row and unit: GEMM1 on the
// three 16-key tiles that can meet the unit's windows (A = keys, B = queries;
// the accumulator holds K_hat for 4 keys of one query per lane), the spatial
// weights (row tap x column tap, zero outside the window) applied in FP32,
// then GEMM2 with those values as the A operand straight from the
// accumulators: their K slots are keys {4q + i} of two tiles, and the staged
// image values are read in the same key order for the B operand.
// Channels run in chunks of 128 (GEMM1 recomputed per chunk).
//
// Inputs are prepared once per call into zero-padded buffers, so that the
// staging needs no bounds checks: the embedding as [H][WP][RP] hi and lo
// (RP = r_eff rounded up to 32 or 64), the centred image as
// [CP][H][WP] (CP = C rounded up to 16); storage column = x + 16 and
// WP = 32 ceil(W / 32) + 32, so every block's key columns lie inside.
#include <hip/hip_runtime.h>
#include <math.h>

#include "device_common.h"
#include "nkf_internal.h"

namespace nkf {

namespace {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

template <typename T>
struct WkOp;
template <>
struct WkOp<__bf16> {
  typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 V8;
  typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 V4;
  static __device__ __forceinline__ f32x4 mma(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct WkOp<_Float16> {
  typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 V8;
  typedef __attribute__((__vector_size__(4 * sizeof(_Float16)))) _Float16 V4;
  static __device__ __forceinline__ f32x4 mma(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

constexpr int kWT = 512;     // threads per block
constexpr int kNJ = 2;       // 16-query units per wave
constexpr int kQC = 32;      // query columns per block
constexpr int kQR = 8;       // query rows per block
constexpr int kKC = 64;      // key columns per block
constexpr int kCB = 128;     // channels per chunk
constexpr int kFS = kKC + 8; // LDS row stride of the staged image (elements): 144 B
constexpr int kColOff = 16;  // storage column of x = 0

__host__ __device__ __forceinline__ int wk_wp(int W) { return (W + kQC - 1) / kQC * kQC + kQC; }

struct WkArgs {
  int H, W, C, CP, S, WP, tiles_x, ntiles;
  const void *uh, *ul;  // [H][WP][RP]
  const void *ft;       // [CP][H][WP]
  const float *f, *f0;
  Taps taps;
  float *out, *eta_out;
};

template <typename T, int RS>
struct WkStage {
  static constexpr int RP = 32 * RS;
  T su[2][kKC][RP + 8];  // embedding hi / lo of the key row (row stride RP + 8: 16-byte reads conflict-free)
  T sf[kCB][kFS];        // centred image of the key row, channel-major
};

// ---- preparation: zero-padded 16-bit operands -------------------------------
// Both kernels walk the H x WP storage slots (slot = y WP + storage column) in
// groups of 64 and transpose through LDS, so that the reads (planes of u,
// pixels of f) and the writes (pixel-major u, channel planes of f) are
// contiguous runs.

constexpr int kPrepPx = 64;

template <typename T>
__global__ __launch_bounds__(256) void wk_prep_u_kernel(const float *__restrict__ u, int64_t N, int r_eff, int H,
                                                        int W, int WP, int RP, T *__restrict__ uh,
                                                        T *__restrict__ ul) {
  __shared__ float tile[64][kPrepPx + 1];  // [plane][slot]
  const int64_t nslots = (int64_t)H * WP;
  const int64_t s0 = (int64_t)blockIdx.x * kPrepPx;
  const int tid = threadIdx.x;
  // read: plane k, 64 consecutive slots (pixels of one image row or two)
  for (int e = tid; e < RP * kPrepPx; e += 256) {
    const int k = e / kPrepPx, px = e % kPrepPx;
    const int64_t sl = s0 + px;
    float v = 0.0f;
    if (sl < nslots && k < r_eff) {
      const int y = (int)(sl / WP), x = (int)(sl % WP) - kColOff;
      if (x >= 0 && x < W) v = u[(int64_t)k * N + (int64_t)y * W + x];
    }
    tile[k][px] = v;
  }
  __syncthreads();
  // write: 8 planes of one slot per thread-step, consecutive threads along the
  // slot's RP values, then the next slot
  const int KC = RP / 8;
  for (int e = tid; e < KC * kPrepPx; e += 256) {
    const int px = e / KC, kc = e % KC;
    const int64_t sl = s0 + px;
    if (sl >= nslots) continue;
    typename WkOp<T>::V8 hi, lo;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float v = tile[8 * kc + i][px];
      hi[i] = (T)v;
      lo[i] = (T)(v - (float)hi[i]);
    }
    *reinterpret_cast<typename WkOp<T>::V8 *>(uh + sl * RP + 8 * kc) = hi;
    *reinterpret_cast<typename WkOp<T>::V8 *>(ul + sl * RP + 8 * kc) = lo;
  }
}

// grid: (slot groups, channel groups of 128)
template <typename T>
__global__ __launch_bounds__(256) void wk_prep_f_kernel(const float *__restrict__ f, const float *__restrict__ f0,
                                                        int C, int CP, int H, int W, int WP, T *__restrict__ ft) {
  __shared__ T tile[kCB][kPrepPx + 8];  // [channel][slot]
  const int64_t nslots = (int64_t)H * WP;
  const int64_t s0 = (int64_t)blockIdx.x * kPrepPx;
  const int cb = blockIdx.y * kCB, nc = min(kCB, CP - cb);
  const int tid = threadIdx.x;
  // read: the slots' pixels, channels cb .. cb + nc - 1 (contiguous per pixel)
  for (int e = tid; e < nc * kPrepPx; e += 256) {
    const int px = e / nc, c = e % nc;
    const int64_t sl = s0 + px;
    float v = 0.0f;
    if (sl < nslots && cb + c < C) {
      const int y = (int)(sl / WP), x = (int)(sl % WP) - kColOff;
      if (x >= 0 && x < W) v = f[((int64_t)y * W + x) * C + cb + c] - f0[cb + c];
    }
    tile[c][px] = (T)v;
  }
  __syncthreads();
  // write: 8 slots of one channel per thread-step
  for (int e = tid; e < nc * (kPrepPx / 8); e += 256) {
    const int c = e / (kPrepPx / 8), q = e % (kPrepPx / 8);
    const int64_t sl = s0 + 8 * q;
    if (sl >= nslots) continue;  // nslots is a multiple of 8 (WP is)
    *reinterpret_cast<typename WkOp<T>::V8 *>(ft + (int64_t)(cb + c) * nslots + sl) =
        *reinterpret_cast<const typename WkOp<T>::V8 *>(&tile[c][8 * q]);
  }
}

// ---- the windowed kernel ----------------------------------------------------

template <typename T, int RS>
__global__ __launch_bounds__(kWT) void wk_kernel(WkArgs a) {
  using V8 = typename WkOp<T>::V8;
  using V4 = typename WkOp<T>::V4;
  constexpr int RP = 32 * RS;
  constexpr int NU = 2 * kKC * RP / 8 / kWT;  // 16-byte embedding chunks per thread and key row
  constexpr int NF = kCB * kKC / 8 / kWT;     // 16-byte image chunks per thread and key row (max)
  __shared__ WkStage<T, RS> st[2];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  const int y0 = (tile / a.tiles_x) * kQR, x0 = (tile % a.tiles_x) * kQC;
  const int qt = w & 1;
  const int S = a.S;
  const T *uh = static_cast<const T *>(a.uh);
  const T *ul = static_cast<const T *>(a.ul);
  const T *ft = static_cast<const T *>(a.ft);

  // query operands (B of GEMM1): unit j = query row y0 + (w >> 1) + 4j,
  // columns x0 + 16 qt + col, embedding chunk 8 kq of each 32-wide step
  V8 qh[kNJ][RS], ql[kNJ][RS];
#pragma unroll
  for (int j = 0; j < kNJ; ++j) {
    const int qy = y0 + (w >> 1) + 4 * j;
    const int64_t o = ((int64_t)(qy < a.H ? qy : 0) * a.WP + x0 + 16 * qt + col + kColOff) * RP + 8 * kq;
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      V8 h = *reinterpret_cast<const V8 *>(uh + o + 32 * s);
      V8 l = *reinterpret_cast<const V8 *>(ul + o + 32 * s);
      if (qy >= a.H) {
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = (T)0.0f, l[e] = (T)0.0f;
      }
      qh[j][s] = h;
      ql[j][s] = l;
    }
  }
  // column taps of the lane's accumulator entries: key tile kt (0..2, key
  // columns x0 + 16 (qt + kt) - 16 + 4 kq + i) against query column
  // x0 + 16 qt + col
  float wx[3][4];
#pragma unroll
  for (int kt = 0; kt < 3; ++kt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int dx = 16 * kt - 16 + 4 * kq + i - col;
      wx[kt][i] = (dx >= -S && dx <= S) ? a.taps.w[dx + S] : 0.0f;
    }

  const int nky = kQR + 2 * S;
  for (int c0 = 0; c0 < a.CP; c0 += kCB) {
    const int CB = min(kCB, a.CP - c0);  // multiple of 16
    const int CT = CB / 16;
    f32x4 z[kNJ][kCB / 16];
    float eta[kNJ];
#pragma unroll
    for (int j = 0; j < kNJ; ++j) {
      eta[j] = 0.0f;
#pragma unroll
      for (int ct = 0; ct < kCB / 16; ++ct) z[j][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

    uint4 ru[NU], rf[NF];
    auto load_row = [&](int ky) {
      const bool in = ky >= 0 && ky < a.H;
#pragma unroll
      for (int q = 0; q < NU; ++q) {
        const int e = tid + kWT * q;
        const int hl = e / (8 * RP), rem = e % (8 * RP);
        const int px = rem / (RP / 8), kc = rem % (RP / 8);
        const T *src = (hl ? ul : uh) + ((int64_t)(in ? ky : 0) * a.WP + x0 + px) * RP + 8 * kc;
        ru[q] = in ? *reinterpret_cast<const uint4 *>(src) : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        const int e = tid + kWT * q;
        const int c = e >> 3, qq = e & 7;
        const bool ok = in && c < CB;
        const T *src = ft + ((int64_t)(c0 + (ok ? c : 0)) * a.H + (in ? ky : 0)) * a.WP + x0 + 8 * qq;
        rf[q] = ok ? *reinterpret_cast<const uint4 *>(src) : make_uint4(0u, 0u, 0u, 0u);
      }
    };
    auto store_row = [&](WkStage<T, RS> &sg) {
#pragma unroll
      for (int q = 0; q < NU; ++q) {
        const int e = tid + kWT * q;
        const int hl = e / (8 * RP), rem = e % (8 * RP);
        const int px = rem / (RP / 8), kc = rem % (RP / 8);
        *reinterpret_cast<uint4 *>(&sg.su[hl][px][8 * kc]) = ru[q];
      }
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        const int e = tid + kWT * q;
        const int c = e >> 3, qq = e & 7;
        if (c < CB) *reinterpret_cast<uint4 *>(&sg.sf[c][8 * qq]) = rf[q];
      }
    };

    load_row(y0 - S);
    store_row(st[0]);
    __syncthreads();
    for (int it = 0; it < nky; ++it) {
      const int ky = y0 - S + it;
      if (it + 1 < nky) load_row(ky + 1);
      const WkStage<T, RS> &sg = st[it & 1];
      float wy[kNJ];
      bool any = false;
#pragma unroll
      for (int j = 0; j < kNJ; ++j) {
        const int dy = ky - (y0 + (w >> 1) + 4 * j);
        const bool act = dy >= -S && dy <= S;
        wy[j] = act ? a.taps.w[dy + S] : 0.0f;
        any |= act;
      }
      if (any) {
        // GEMM1 per key tile, weights applied, packed as GEMM2 A operands
        V4 wt16[kNJ][3];
#pragma unroll
        for (int kt = 0; kt < 3; ++kt) {
          const int kc0 = 16 * (qt + kt);
          V8 ah[RS], al[RS];
#pragma unroll
          for (int s = 0; s < RS; ++s) {
            ah[s] = *reinterpret_cast<const V8 *>(&sg.su[0][kc0 + col][32 * s + 8 * kq]);
            al[s] = *reinterpret_cast<const V8 *>(&sg.su[1][kc0 + col][32 * s + 8 * kq]);
          }
          f32x4 acc[kNJ];
#pragma unroll
          for (int j = 0; j < kNJ; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < RS; ++s) {
#pragma unroll
            for (int j = 0; j < kNJ; ++j) acc[j] = WkOp<T>::mma(ah[s], qh[j][s], acc[j]);
#pragma unroll
            for (int j = 0; j < kNJ; ++j) acc[j] = WkOp<T>::mma(al[s], qh[j][s], acc[j]);
#pragma unroll
            for (int j = 0; j < kNJ; ++j) acc[j] = WkOp<T>::mma(ah[s], ql[j][s], acc[j]);
          }
#pragma unroll
          for (int j = 0; j < kNJ; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float v = acc[j][i] * (wy[j] * wx[kt][i]);
              eta[j] += v;
              wt16[j][kt][i] = (T)v;
            }
          // keep each tile's operand loads next to their use (register pressure)
          __builtin_amdgcn_sched_barrier(0);
        }
        // GEMM2: key pairs (tile qt, qt + 1) and (qt + 2, zeros)
        V8 a0[kNJ], a1[kNJ];
        const V4 zero4 = {(T)0.0f, (T)0.0f, (T)0.0f, (T)0.0f};
#pragma unroll
        for (int j = 0; j < kNJ; ++j) {
          a0[j] = __builtin_shufflevector(wt16[j][0], wt16[j][1], 0, 1, 2, 3, 4, 5, 6, 7);
          a1[j] = __builtin_shufflevector(wt16[j][2], zero4, 0, 1, 2, 3, 4, 5, 6, 7);
        }
#pragma unroll
        for (int ct = 0; ct < kCB / 16; ++ct) {
          if (ct < CT) {
            const T *fr = &sg.sf[16 * ct + col][0];
            const V4 f0v = *reinterpret_cast<const V4 *>(fr + 16 * qt + 4 * kq);
            const V4 f1v = *reinterpret_cast<const V4 *>(fr + 16 * (qt + 1) + 4 * kq);
            const V4 f2v = *reinterpret_cast<const V4 *>(fr + 16 * (qt + 2) + 4 * kq);
            const V8 b0 = __builtin_shufflevector(f0v, f1v, 0, 1, 2, 3, 4, 5, 6, 7);
            const V8 b1 = __builtin_shufflevector(f2v, f2v, 0, 1, 2, 3, 0, 1, 2, 3);
#pragma unroll
            for (int j = 0; j < kNJ; ++j) {
              z[j][ct] = WkOp<T>::mma(a0[j], b0, z[j][ct]);
              z[j][ct] = WkOp<T>::mma(a1[j], b1, z[j][ct]);
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if (it + 1 < nky) store_row(st[(it + 1) & 1]);
      __syncthreads();
    }

    // epilogue: eta_hat of query col is spread over the four lanes col + 16 kq
#pragma unroll
    for (int j = 0; j < kNJ; ++j) {
      float e = eta[j];
      e += __shfl_xor(e, 16, 64);
      e += __shfl_xor(e, 32, 64);
      const int qy = y0 + (w >> 1) + 4 * j;
      if (qy >= a.H) continue;
      if (c0 == 0 && a.eta_out && kq == 0) {
        const int x = x0 + 16 * qt + col;
        if (x < a.W) a.eta_out[(int64_t)qy * a.W + x] = e;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = 4 * kq + i;  // query of accumulator entry i
        const float eq = __shfl(e, q, 64);
        const int x = x0 + 16 * qt + q;
        if (x >= a.W) continue;
        const bool ok = eq > 0.0f && isfinite(eq);
        const int64_t px = (int64_t)qy * a.W + x;
#pragma unroll
        for (int ct = 0; ct < kCB / 16; ++ct) {
          const int c = c0 + 16 * ct + col;
          if (ct < CT && c < a.C)
            a.out[px * a.C + c] = ok ? a.f0[c] + z[j][ct][i] / eq : a.f[px * a.C + c];
        }
      }
    }
  }
}

int wk_rs(int r_eff) { return r_eff <= 32 ? 1 : 2; }

template <typename T>
hipError_t launch_wk_t(const WkProblem &pb, hipStream_t s) {
  const int WP = wk_wp(pb.W), RP = 32 * wk_rs(pb.r_eff), CP = (pb.C + 15) / 16 * 16;
  const int64_t N = (int64_t)pb.H * pb.W;
  // scratch: the centred image first (prepared by launch_wk_prep_f, which
  // needs no landmarks), then the embedding hi and lo
  T *ft = static_cast<T *>(pb.scratch);
  T *uh = ft + (size_t)CP * pb.H * WP;
  T *ul = uh + (size_t)pb.H * WP * RP;
  const unsigned groups = (unsigned)(((int64_t)pb.H * WP + kPrepPx - 1) / kPrepPx);
  hipLaunchKernelGGL(wk_prep_u_kernel<T>, dim3(groups), dim3(256), 0, s, pb.u, N, pb.r_eff, pb.H, pb.W, WP, RP,
                     uh, ul);

  WkArgs a{};
  a.H = pb.H;
  a.W = pb.W;
  a.C = pb.C;
  a.CP = CP;
  a.S = pb.S;
  a.WP = WP;
  a.tiles_x = (pb.W + kQC - 1) / kQC;
  a.ntiles = a.tiles_x * ((pb.H + kQR - 1) / kQR);
  a.uh = uh;
  a.ul = ul;
  a.ft = ft;
  a.f = pb.f;
  a.f0 = pb.f0;
  a.taps = pb.taps;
  a.out = pb.out;
  a.eta_out = pb.eta_out;
  if (wk_rs(pb.r_eff) == 1)
    hipLaunchKernelGGL((wk_kernel<T, 1>), dim3(a.ntiles), dim3(kWT), 0, s, a);
  else
    hipLaunchKernelGGL((wk_kernel<T, 2>), dim3(a.ntiles), dim3(kWT), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wk_prep_f_t(const WkProblem &pb, hipStream_t s) {
  const int WP = wk_wp(pb.W), CP = (pb.C + 15) / 16 * 16;
  const unsigned groups = (unsigned)(((int64_t)pb.H * WP + kPrepPx - 1) / kPrepPx);
  hipLaunchKernelGGL(wk_prep_f_kernel<T>, dim3(groups, (unsigned)((CP + kCB - 1) / kCB)), dim3(256), 0, s, pb.f,
                     pb.f0, pb.C, CP, pb.H, pb.W, WP, static_cast<T *>(pb.scratch));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_wk_prep_f(const WkProblem &pb, hipStream_t s) {
  return pb.prec == 1 ? launch_wk_prep_f_t<__bf16>(pb, s) : launch_wk_prep_f_t<_Float16>(pb, s);
}

bool wk_supported(int C, int r, int S, int prec) {
  return prec != 0 && C >= 4 && r <= kWkMaxRank && S <= kMaxRadius;
}

size_t wk_scratch_bytes(int H, int W, int C, int r) {
  const size_t WP = wk_wp(W), RP = 32 * wk_rs(r), CP = (C + 15) / 16 * 16;
  return 2 * ((size_t)2 * H * WP * RP + CP * H * WP);
}

hipError_t launch_wk(const WkProblem &pb, hipStream_t s) {
  if (pb.r_eff < 1 || pb.r_eff > kWkMaxRank || pb.S > kMaxRadius || pb.S < 0) return hipErrorInvalidValue;
  return pb.prec == 1 ? launch_wk_t<__bf16>(pb, s) : launch_wk_t<_Float16>(pb, s);
}

}  // namespace nkf
