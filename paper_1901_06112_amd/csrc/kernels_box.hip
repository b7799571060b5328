// Box-window convolutions + contraction + normalisation (Section III,
// Eqs. (finalnum), (finalden); the box window of the nonlocal-means
// experiments, Section IV) for images with up to three channels, with FP64
// storage and accumulation from the embedding planes to the output.
//
// For embedding plane u_k and image channel c,
//   E_k = box * u_k,   Z_kc = box * (u_k f_c),
//   eta(x) = sum_k u_k(x) E_k(x),   zeta_c(x) = sum_k u_k(x) Z_kc(x),
//   g_c(x) = zeta_c(x) / eta(x)        (f_c(x) where eta <= 0 or not finite),
// the box being the (2S+1)^2 window of ones intersected with the image (zero
// extension of numerator and denominator alike).  The image is not centred
// here: every stage is FP64, so the uncentred numerator costs no accuracy and
// g = zeta / eta directly.
//
// A block owns an output tile of TW = 64 - 2S columns by 56 rows (32 to 48
// for the larger radii); the 64 columns of the tile plus S on each side are the threads'
// columns.  For each plane k:
//   vertical pass    thread (column, plane p, half of the rows) walks down its
//                    rows keeping an FP64 sliding sum of u_k f_p (plane 0: u_k)
//                    over 2S + 1 rows; the term of the row that leaves the
//                    window is recomputed from the u_k value the thread still
//                    holds, and the sums of the output rows go to LDS, with
//                    u_k at the tile's own pixels;
//   horizontal pass  thread (output row, plane, half of the columns) slides an
//                    FP64 window along the vertical sums and adds u_k(x) times
//                    the window sum to its FP64 accumulators.
// Each register that held u_k of a row that has left the window is reloaded
// at once with u_{k+1} of that row, so a whole plane's loads are in flight
// behind the current plane's arithmetic.
//
// Per pixel and plane k (P = C + 1 planes): 4P flops of sliding sums, P
// products and 2P contraction flops; compulsory HBM traffic is the u_k value
// (8 bytes in the FP64 form), so the kernel streams r_eff * 8 bytes per pixel
// plus the image and the output.
#include <hip/hip_runtime.h>
#include <math.h>

#include "device_common.h"

namespace nkf {

namespace {

constexpr int kBT = 512;        // threads per block
constexpr int kXW = 64;         // tile width including the 2S halo columns
// Output rows per tile: 56, fewer for the larger radii, whose longer column
// windows would not leave registers for 56 (a register spill puts scratch
// loads on the counter the plane prefetch relies on).
constexpr int tile_rows(int S, bool u_fp64) {
  return u_fp64 ? (S <= 8 ? 56 : S <= 10 ? 48 : S <= 12 ? 40 : 32) : (S <= 10 ? 56 : S <= 13 ? 48 : 40);
}
constexpr int kNP = 4;          // planes per k: E and up to three channels
// LDS strides of the vertical sums vbuf[row][plane][column] in doubles.  An
// 8-byte access is served 32 lanes at a time over 64 four-byte banks, so 32
// lanes conflict-free need 32 distinct addresses mod 32.  The vertical pass
// stores 8 columns x 4 planes per half-wave (plane stride == 8 mod 32), the
// horizontal pass reads 8 rows x 4 planes (row stride == 1 mod 32).
constexpr int kPS = 72;
constexpr int kRS = 289;
constexpr int kMaxSplits = 8;   // k ranges per tile (blocks of one tile)
constexpr unsigned kOffInvalid = 0x80000000u;

// u_k at the tile's pixels, ubuf[row][column] over all 64 columns; an odd row
// stride puts the 8 rows a horizontal-pass half-wave reads in distinct banks.
constexpr int kUS = kXW + 1;
static_assert(kPS % 32 == 8 && kRS % 32 == 1 && kRS >= kNP * kPS, "vbuf strides");

struct BoxArgs {
  int H, W, C, r_eff;
  int tiles_x, ntiles, nks, nblocks;
  const float *f;
  const void *u;        // [r_eff][N] of UT
  float *out;
  float *eta_out;       // nullable
  double *part;         // [nks][N][4] when nks > 1
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, int nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, nbytes, 0x00020000);
}

// One element at byte offset `off` of a buffer resource; an offset at or past
// the resource's size reads 0 without touching memory.
template <typename UT>
__device__ __forceinline__ UT ld(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ double ld<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float ld<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Marks a per-lane register as redefined, in place.  Applied once per plane to
// the image values, it keeps their FP32 -> FP64 conversions at their use
// instead of a hoisted FP64 copy of every row.
__device__ __forceinline__ void touch_v(float &v) { asm volatile("" : "+v"(v)); }
// The same for a wave-uniform value, in a scalar register (an in-place asm on
// a vector register that feeds the loads makes the compiler drain every
// pending load at the loop head).
__device__ __forceinline__ unsigned opaque_s(unsigned v) {
  v = __builtin_amdgcn_readfirstlane(v);
  asm volatile("" : "+s"(v));
  return v;
}

// Value of lane J of each quad (four consecutive lanes), in every lane of the
// quad: DPP quad_perm [J, J, J, J] on each 32-bit half.
template <int J>
__device__ __forceinline__ double quad_bcast(double v) {
  constexpr int ctl = J * 0x55;
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, ctl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctl, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// quad_bcast for a lane index known after unrolling
__device__ __forceinline__ double quad_bcast_at(double v, int j) {
  switch (j & 3) {
    case 0: return quad_bcast<0>(v);
    case 1: return quad_bcast<1>(v);
    case 2: return quad_bcast<2>(v);
    default: return quad_bcast<3>(v);
  }
}

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left free): the image values are in
// registers before the first plane's loads are issued, so that at most one
// plane's loads per thread (fewer than the 63 the counter tracks) are ever in
// flight and the plane loop waits for each row's load alone.
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

template <int S, typename UT>
__global__ __launch_bounds__(kBT) void box_kernel(BoxArgs a) {
  constexpr int TW = kXW - 2 * S;        // output columns of a tile
  constexpr int kTH = tile_rows(S, sizeof(UT) == 8);  // output rows of a tile
  constexpr int kTHH = kTH / 2;          // output rows per half of the vertical pass
  constexpr int G = 2 * S + 1;           // window length
  constexpr int IRH = kTHH + 2 * S;      // input rows of one half of the vertical pass
  constexpr int RUN = TW / 2;            // output columns per horizontal-pass thread
  static_assert(kTH % 8 == 0 && kTH <= 64, "horizontal pass: 8 rows per wave, 8 waves");
  __shared__ double vbuf[kTH * kRS];
  __shared__ double ubuf[kTH * kUS];

  const int tid = threadIdx.x;
  const int L = xcd_swizzle(blockIdx.x, a.nblocks);
  const int ks = L / a.ntiles, tile = L - ks * a.ntiles;
  const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
  const int H = a.H, W = a.W, C = a.C;
  const int64_t N = (int64_t)H * W;
  const int k0 = (int)((int64_t)a.r_eff * ks / a.nks);
  const int k1 = (int)((int64_t)a.r_eff * (ks + 1) / a.nks);

  // ---- vertical-pass role: 16 columns x 4 planes per wave ------------------
  const int vp = tid & 3, vc = (tid >> 2) & (kXW - 1);
  const int vh = __builtin_amdgcn_readfirstlane(tid >> 8);
  const int gx = tx * TW - S + vc;
  const bool colok = gx >= 0 && gx < W;
  const int gy0 = ty * kTH - S + vh * kTHH;   // image row of the half's first input row
  const UT *ub = static_cast<const UT *>(a.u);
  // One buffer resource per plane, based at the half's first row inside the
  // image and covering the half's rows inside it; row q of the half is at
  // byte offset voff0 + q * rowbytes.  Rows above the image give negative
  // offsets (>= 2^31 as unsigned), rows below it offsets past the resource,
  // and columns outside it start from kOffInvalid: all read 0 without a
  // branch.  Offsets stay within 2^31 of their start (IRH rows of at most
  // 2^21 FP64 values), and the resource holds at most IRH rows.
  const int gyb = gy0 > 0 ? gy0 : 0;
  const int rows_in = min(H - gyb, IRH);
  const int nrec = rows_in > 0 ? rows_in * W * (int)sizeof(UT) : 0;
  const unsigned rowbytes = (unsigned)W * (unsigned)sizeof(UT);
  const unsigned voff0 =
      colok ? (unsigned)(((int64_t)(gy0 - gyb) * W + gx) * (int64_t)sizeof(UT)) : kOffInvalid;
  auto plane_rsrc = [&](int k) { return buf_rsrc(ub + (int64_t)k * N + (int64_t)gyb * W, nrec); };

  // the thread's multiplier down its column: 1 for the E plane, f_{p-1}
  // otherwise (0 for planes past C and outside the image, where u_k is 0 too)
  float freg[IRH];
#pragma unroll
  for (int q = 0; q < IRH; ++q) {
    const int gy = gy0 + q;
    const bool ok = colok && (unsigned)gy < (unsigned)H && vp <= C;
    freg[q] = vp == 0 ? 1.0f : (ok ? a.f[((int64_t)gy * W + gx) * C + (vp - 1)] : 0.0f);
  }
  wait_vm_all();

  // The four threads of a column (a quad of lanes, one per plane) split its
  // rows: thread p loads rows p, p + 4, ..., M of them, and each row's value
  // reaches the other three by a quad broadcast.  Two register sets
  // alternate: the loads of plane k + 1 are issued at the start of plane k.
  constexpr int M = (IRH + 3) / 4;
  const unsigned voffp = voff0 + (unsigned)vp * rowbytes;
  UT own[2][M];
  auto load_plane = [&](UT (&dst)[M], int k) {
    const __amdgpu_buffer_rsrc_t rk = plane_rsrc(k);
    // the row stride is opaque per plane so that the M offsets are not hoisted
    const unsigned rb4 = opaque_s(4u * rowbytes);
    unsigned vo = voffp;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      dst[m] = ld<UT>(rk, vo);
      vo += rb4;
      // issued in row order, so that each use waits for its own row alone
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  load_plane(own[0], k0);

  // ---- horizontal-pass role: 8 rows x 4 planes x 2 column halves per wave --
  const int ho = (tid >> 6) * 8 + (tid & 7);
  const int hp = (tid >> 3) & 3, hs = (tid >> 5) & 1;
  const bool hact = __builtin_amdgcn_readfirstlane(tid >> 6) < kTH / 8;
  double acc[RUN];
#pragma unroll
  for (int j = 0; j < RUN; ++j) acc[j] = 0.0;

  // one plane: the vertical pass from `cur`, the next plane's loads into `nxt`,
  // then the horizontal pass
  auto plane = [&](UT (&cur)[M], UT (&nxt)[M], int k) {
    // the next plane's loads (the last plane reloads itself: no branch)
    load_plane(nxt, k + 1 < k1 ? k + 1 : k);
#pragma unroll
    for (int q = 0; q < IRH; ++q) touch_v(freg[q]);
    // u of the last G rows, a ring indexed by row mod G
    double fifo[G];
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < IRH; ++q) {
      const double uq = quad_bcast_at((double)cur[q >> 2], q);
      s = fma(uq, (double)freg[q], s);
      if (q >= G) s = fma(-fifo[q % G], (double)freg[q - G], s);  // the row leaving the window
      fifo[q % G] = uq;
      if (q >= 2 * S) {
        const int o = vh * kTHH + q - 2 * S;  // output row centred on input row q - S
        vbuf[o * kRS + vp * kPS + vc] = s;
        // the four plane threads of a column store the same value
        ubuf[o * kUS + vc] = fifo[(q - S) % G];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    if (hact) {
      const double *vr = vbuf + ho * kRS + hp * kPS + hs * RUN;
      const double *ur = ubuf + ho * kUS + S + hs * RUN;
      double w = 0.0;
#pragma unroll
      for (int t = 0; t < G; ++t) w += vr[t];
#pragma unroll
      for (int j = 0; j < RUN; ++j) {
        if (j > 0) w += vr[j + 2 * S] - vr[j - 1];
        acc[j] = fma(ur[j], w, acc[j]);
      }
    }
    __syncthreads();
  };

  for (int k = k0; k < k1; k += 2) {
    plane(own[0], own[1], k);
    if (k + 1 < k1) plane(own[1], own[0], k + 1);
  }

  // ---- epilogue -------------------------------------------------------------
  const int oy = ty * kTH + ho;
  const int ox0 = tx * TW + hs * RUN;
  if (a.nks > 1) {
    // this k range's FP64 sums; the combine kernel adds the ranges in order
    if (hact && oy < H && hp <= C) {
      double *dst = a.part + ((int64_t)ks * N + (int64_t)oy * W) * kNP + hp;
#pragma unroll
      for (int j = 0; j < RUN; ++j)
        if (ox0 + j < W) dst[(int64_t)(ox0 + j) * kNP] = acc[j];
    }
    return;
  }
  double *eb = vbuf;  // eta of the tile, [kTH][TW]
  if (hact && hp == 0) {
#pragma unroll
    for (int j = 0; j < RUN; ++j) eb[ho * TW + hs * RUN + j] = acc[j];
  }
  __syncthreads();
  if (hact && oy < H && hp <= C) {
#pragma unroll
    for (int j = 0; j < RUN; ++j) {
      const int ox = ox0 + j;
      if (ox >= W) continue;
      const int64_t pix = (int64_t)oy * W + ox;
      const double e = eb[ho * TW + hs * RUN + j];
      if (hp == 0) {
        if (a.eta_out) a.eta_out[pix] = (float)e;
      } else {
        const int ch = hp - 1;
        a.out[pix * C + ch] = (e > 0.0 && isfinite(e)) ? (float)(acc[j] / e) : a.f[pix * C + ch];
      }
    }
  }
}

// Sums of the k ranges (in range order), the normalisation and the guard.
__global__ __launch_bounds__(256) void box_combine_kernel(const double *__restrict__ part, int nks, int64_t N,
                                                          int C, const float *__restrict__ f,
                                                          float *__restrict__ out, float *__restrict__ eta_out) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
    double z[kNP] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < nks; ++s) {
      const double *pp = part + ((int64_t)s * N + x) * kNP;
#pragma unroll
      for (int p = 0; p < kNP; ++p)
        if (p <= C) z[p] += pp[p];
    }
    const double e = z[0];
    if (eta_out) eta_out[x] = (float)e;
    const bool ok = e > 0.0 && isfinite(e);
    for (int c = 0; c < C; ++c) out[x * C + c] = ok ? (float)(z[1 + c] / e) : f[x * C + c];
  }
}

int box_tile_width(int S) { return kXW - 2 * S; }

template <int S, typename UT>
hipError_t launch_S(const BoxArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((box_kernel<S, UT>), dim3(a.nblocks), dim3(kBT), 0, s, a);
  return hipGetLastError();
}

template <typename UT>
hipError_t launch_T(const BoxArgs &a, int S, hipStream_t s) {
  switch (S) {
#define NKF_CASE(SV) \
  case SV:           \
    return launch_S<SV, UT>(a, s);
    NKF_CASE(0) NKF_CASE(1) NKF_CASE(2) NKF_CASE(3) NKF_CASE(4) NKF_CASE(5) NKF_CASE(6) NKF_CASE(7)
    NKF_CASE(8) NKF_CASE(9) NKF_CASE(10) NKF_CASE(11) NKF_CASE(12) NKF_CASE(13) NKF_CASE(14)
    NKF_CASE(15) NKF_CASE(16)
#undef NKF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

// Number of k ranges a tile is split into: one block per CU is resident (the
// tile's LDS), so the grid runs in ceil(blocks / CUs) rounds of r_eff / nks
// planes each; the smallest split within 3% of the best round count wins
// (each extra range costs 64 bytes of partial sums per pixel).
int box_splits(int H, int W, int S, int r_eff, int num_cu, int u_fp64) {
  if (S < 0 || S > kMaxRadius) return 1;
  const int TH = tile_rows(S, u_fp64 != 0);
  const int64_t tiles = (int64_t)((W + box_tile_width(S) - 1) / box_tile_width(S)) * ((H + TH - 1) / TH);
  const int cu = num_cu > 0 ? num_cu : 256;
  const int kmax = r_eff < kMaxSplits ? r_eff : kMaxSplits;
  double best = 1e300;
  double cost[kMaxSplits + 1];
  for (int k = 1; k <= kmax; ++k) {
    cost[k] = (double)((tiles * k + cu - 1) / cu) / k;
    if (cost[k] < best) best = cost[k];
  }
  for (int k = 1; k <= kmax; ++k)
    if (cost[k] <= best * 1.03) return k;
  return 1;
}

size_t box_partials_doubles(int H, int W, int S, int r_eff, int num_cu, int u_fp64) {
  const int nks = box_splits(H, W, S, r_eff, num_cu, u_fp64);
  return nks > 1 ? (size_t)nks * H * W * kNP : 0;
}

hipError_t launch_box(const BoxProblem &pb, hipStream_t s) {
  if (pb.C < 1 || pb.C > 3 || pb.S < 0 || pb.S > kMaxRadius) return hipErrorInvalidValue;
  BoxArgs a{};
  a.H = pb.H;
  a.W = pb.W;
  a.C = pb.C;
  a.r_eff = pb.r_eff;
  a.f = pb.f;
  a.u = pb.u;
  a.out = pb.out;
  a.eta_out = pb.eta_out;
  const int TW = box_tile_width(pb.S);
  a.tiles_x = (pb.W + TW - 1) / TW;
  const int TH = tile_rows(pb.S, pb.u_fp64 != 0);
  const int64_t ntiles = (int64_t)a.tiles_x * ((pb.H + TH - 1) / TH);
  a.nks = box_splits(pb.H, pb.W, pb.S, pb.r_eff, pb.num_cu, pb.u_fp64);
  if (a.nks > 1 && !pb.part) return hipErrorInvalidValue;
  a.part = pb.part;
  if (ntiles * a.nks > 0x7fffffff) return hipErrorInvalidValue;
  a.ntiles = (int)ntiles;
  a.nblocks = (int)(ntiles * a.nks);
  hipError_t e = pb.u_fp64 ? launch_T<double>(a, pb.S, s) : launch_T<float>(a, pb.S, s);
  if (e != hipSuccess || a.nks == 1) return e;
  const int64_t N = (int64_t)pb.H * pb.W;
  int64_t blocks = (N + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(box_combine_kernel, dim3((unsigned)blocks), dim3(256), 0, s, pb.part, a.nks, N, pb.C, pb.f,
                     pb.out, pb.eta_out);
  return hipGetLastError();
}

}  // namespace nkf
