// Shared core of the fused convolution kernels: the streaming separable FIR
// (row pass into an LDS ring, column pass out of it) and its per-k epilogues
// for the forward filter and for the adjoint passes of the backward.
//
// Forward (Section III, Eqs. (finalnum), (finalden); Algorithm 1
// accumulation loop), in embedding form: with u_k the planes of the range
// embedding and f~ = f - f0,
//     Z_kc = w * (u_k f~_c),   E_k = w * u_k,
//     zeta_c(x) = sum_k u_k(x) Z_kc(x),   eta(x) = sum_k u_k(x) E_k(x),
//     g(x) = zeta(x) / eta(x) + f0        (f(x) where eta <= 0 or not finite).
// w(z) = w1(z1) w1(z2) on the (2S+1)^2 window intersected with the image.
//
// Backward modes (NP = 4 planes, C <= 3), with a_c = G_c / eta and
// beta = -sum_c G_c g~_c / eta per pixel (see kernels_bwd.hip):
//   MODE_DUDIR  du_dir_k(x) = beta E_k(x) + sum_c a_c Z_kc(x)        -> HBM
//   MODE_SIGS   sum_x u_k(x) [beta (w' * u_k) + sum_c a_c (w' * u_k f~_c)]
//               with w' = dw/dsigma_s = w1' (x) w1 + w1 (x) w1' (taps w1 in
//               wr, w1' in wc): the row pass keeps both w1 and w1' rows in two
//               rings, the column pass takes w1' over the first and w1 over
//               the second                                          -> partials
//   MODE_DS     MODE_DUDIR and MODE_SIGS in one pass: the w1 column pass over
//               the w1 rows gives du_dir, the w1' one the sigma_s terms
//   MODE_ADJ    Yb_k = w * (beta u_k), Ya_kc = w * (a_c u_k):
//               du_k(x) = du_dir_k(x) + Yb_k(x) + sum_c f~_c(x) Ya_kc(x) -> HBM
//               df_c(x) = sum_k u_k(x) Ya_kc(x)                  -> registers
//
// One block owns a 32-column x TH-row output tile and a set of NP planes.
// For each k it streams the tile's input rows (plus S-row halos) through LDS
// in chunks of RC rows:
//   stage   the NP plane inputs for RC rows x (32 + 2S) columns into LDS
//           (loaded into registers one chunk ahead);
//   row     horizontal FIR of those rows (register sliding window) into a
//           ring of RC (1 + ceil(2S/RC)) rows in LDS;
//   column  vertical FIR down the ring for the previous output chunk, then
//           the mode's per-pixel contraction.
// The r_eff NP convolved planes never reach HBM.
//
// Precision: each FIR pass accumulates its taps in FP64 (FP64 FMA issues at
// the FP32 rate on CDNA4 without packed math) and stores its result as FP32,
// so each convolved value carries one rounding instead of 2S+1.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <math.h>

#include "device_common.h"

namespace nkf {
namespace conv {

constexpr int kBlock = 256;
constexpr int kTW = 32;
constexpr int kTWP = kTW + 4;  // ring row stride (floats): rows shift by 4 banks

enum Mode { MODE_FWD = 0, MODE_DUDIR = 1, MODE_SIGS = 2, MODE_ADJ = 3, MODE_DS = 4 };

struct ConvArgs {
  int H, W, C, r_eff;
  int nch;          // output chunks (of RC rows) per tile
  int force_nch;    // > 0: chunks per tile requested by the caller (0: chosen from the grid size)
  int tiles_x, tiles_y, nblocks;
  int ch_per_block; // channel planes per block
  const float *f;
  const float *fpl;  // nullable: f as planes [C][N] (channel loads coalesced across pixels)
  const float *f0;
  const float *u;
  float *out;
  float *eta_out;   // nullable
  float *eta_buf;   // eta written (HAS_E, NP == 1) or read (!HAS_E)
  // backward modes
  const float *ab;        // [N][4]: beta, a_0, a_1, a_2
  const float *plane_in;  // ADJ: du_dir [r_eff][N]
  float *plane_out;       // DUDIR: du_dir, ADJ: du  [r_eff][N]
  float *df;              // ADJ: [N][C]
  const float *G;         // ADJ: dL/dg [N][C] (guard pixels)
  const float *eta;       // ADJ: eta_hat [N] (guard test)
  double *partials;       // SIGS: one double per block
  double wr[2 * kMaxRadius + 1];  // row-pass taps (FP32 values widened to FP64)
  double wc[2 * kMaxRadius + 1];  // column-pass taps
};

template <int S, int NP, bool HAS_E, int RC, int MODE, int BT = kBlock, bool BOX = false>
struct Cfg {
  static constexpr int T = 2 * S + 1;
  // LDS has 64 banks of 4 bytes; a b128 access is served 16 lanes at a time.
  // The row-pass lanes of one such group are 4 segments (8 floats apart) x 2
  // rows x 2 planes, so rows are offset by 4 mod 32 floats and planes by
  // 32 mod 64 floats: the 16 lanes then cover all 64 banks.
  static constexpr int SW0 = ((kTW + 2 * S + 3) / 4) * 4;
  static constexpr int SW = SW0 + ((4 - SW0 % 32) + 32) % 32;   // >= 32 + 2S, == 4 mod 32
  static constexpr int PSTG0 = RC * SW;
  static constexpr int PSTG = PSTG0 + ((32 - PSTG0 % 64) + 64) % 64;  // plane stride, == 32 mod 64
  static constexpr int RUN = RC * NP * kTW / BT;              // outputs per thread per pass
  static constexpr int SEGS = kTW / RUN;                      // row-pass segments per row
  static constexpr int SUBS = BT / (kTW * NP);                // column-pass row groups
  static constexpr int LAG = (2 * S + RC - 1) / RC;           // input chunks ahead of output
  static constexpr int RING = RC * (1 + LAG);
  static constexpr int RINGX = RING + 2 * S;                  // ring rows + mirrored head
  static constexpr int PR0 = RINGX * kTWP;
  static constexpr int PR = PR0 + ((32 - PR0 % 64) + 64) % 64;     // ring plane stride, == 32 mod 64
  static constexpr int NCH_MAX = 64 / RUN;                    // accumulator budget: 64 floats
  static constexpr int NCHAN = NP - (HAS_E ? 1 : 0);          // channel planes
  static constexpr bool FWD = MODE == MODE_FWD;
  static constexpr bool RAWU_SEP = !HAS_E;                    // raw u needs its own plane
  static constexpr int NPU = NP + (RAWU_SEP ? 1 : 0);         // staged planes
  static constexpr int UPL = RAWU_SEP ? NP : 0;               // index of the raw-u staged plane
  static constexpr int WIN = ((RUN + 2 * S + 3) / 4) * 4;
  static constexpr int STG = NPU * PSTG;                      // staging floats
  static constexpr bool TWO_RINGS = MODE == MODE_SIGS || MODE == MODE_DS;  // w1 and w1' rows
  static constexpr int RINGF = NP * PR * (TWO_RINGS ? 2 : 1);  // convolved-row ring floats
  static constexpr int URINGF = FWD ? RINGX * kTWP : 0;       // raw-u ring floats (forward)
  static constexpr int EXF = (MODE == MODE_DUDIR || MODE == MODE_ADJ || MODE == MODE_DS) ? NP * RC * kTW : 0;
  static constexpr int ETAB = FWD ? NCH_MAX * RC * kTW : 0;   // epilogue eta tile
  static constexpr int MAIN = STG + RINGF + URINGF + EXF;
  static constexpr int SMEM = MAIN > ETAB ? MAIN : ETAB;
  static_assert(RUN * SEGS == kTW, "row pass split");
  // Ring rows as 16-byte stores (row stride == 4 mod 32 and plane stride ==
  // 32 mod 64: each 16 lanes of a store cover all 64 banks, where single-float
  // stores of the same lanes meet 4 to a bank).  Measured faster for the box
  // window and the channel-chunk kernels, slightly slower for the Gaussian
  // kernels with the E plane, which keep single-float stores.
  static constexpr bool VEC_RING = BOX || !HAS_E;
  static_assert(kTWP % 4 == 0 && PR % 4 == 0 && PSTG % 4 == 0, "ring and staging rows hold whole float4s");
  static_assert(SUBS * RUN == RC, "column pass split");
  static_assert(RC * NP * SEGS == BT, "row pass threads");
  static_assert(FWD || (NP == 4 && HAS_E), "backward modes use the E plane + 3 channel planes");
};

// Hides a value from the optimiser so that address arithmetic and loads that
// depend on it are redone each k instead of being hoisted out of the k loop
// (hoisting them keeps hundreds of registers live).
template <class V>
__device__ __forceinline__ V opaque(V v) {
  asm volatile("" : "+v"(v));
  return v;
}

// The same for a wave-uniform value, kept in a scalar register.
__device__ __forceinline__ int opaque_s(int v) {
  return __builtin_amdgcn_readfirstlane(opaque(v));
}

// Raw buffer resource (no stride, gfx9 data format field) over 2^31 - 256
// bytes from base.  A buffer load whose offset is at or past that range
// returns 0 instead of touching memory; kOffInvalid is such an offset.
constexpr unsigned kOffInvalid = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, 0x7FFFFF00, 0x00020000);
}
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// sum_t w[t] x[t] for a symmetric window (w[t] == w[2S - t]): the mirrored
// pair x[t] + x[2S - t] of two FP32 values is exact in FP64, so folding halves
// the taps held in scalar registers without changing the VALU operation count.
template <int S>
__device__ __forceinline__ double fir_sym(const double *w, const double *x) {
  double s = w[S] * x[S];
#pragma unroll
  for (int t = 0; t < S; ++t) s = fma(w[t], x[t] + x[2 * S - t], s);
  return s;
}

// Output i of a run of consecutive outputs over win[i .. i + 2S], called for
// i = 0, 1, ... in order: the symmetric FIR with taps w, or for the box
// kernel (all taps 1) a sliding FP64 sum that adds the entering and drops
// the leaving value (2 operations per output instead of 2S + 1).
template <int S, bool BOX>
struct Window {
  double s = 0.0;
  __device__ __forceinline__ double at(const double *w, const double *win, int i) {
    if constexpr (BOX) {
      if (i == 0) {
        s = 0.0;
#pragma unroll
        for (int t = 0; t <= 2 * S; ++t) s += win[t];
      } else {
        s += win[i + 2 * S] - win[i - 1];
      }
      return s;
    } else {
      return fir_sym<S>(w, &win[i]);
    }
  }
};

// RUN floats (RUN % 4 == 0) to the 16-byte aligned run at dst as 16-byte
// stores, and again at dst + mirror_off when mirror is set.
template <int RUN>
__device__ __forceinline__ void store_run4(float *dst, const float *v, bool mirror, int mirror_off) {
  static_assert(RUN % 4 == 0, "runs are whole float4s");
  float4 *d4 = reinterpret_cast<float4 *>(dst);
#pragma unroll
  for (int j = 0; j < RUN / 4; ++j) {
    const float4 q = make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
    d4[j] = q;
    if (mirror) d4[mirror_off / 4 + j] = q;
  }
}

template <int S, int NP, bool HAS_E, int RC, int MODE, int BT = kBlock, bool BOX = false>
__global__ __launch_bounds__(BT) void conv_kernel(ConvArgs a) {
  using K = Cfg<S, NP, HAS_E, RC, MODE, BT, BOX>;
  constexpr int SW = K::SW, RUN = K::RUN, SEGS = K::SEGS, LAG = K::LAG, RING = K::RING;
  constexpr int NCH_MAX = K::NCH_MAX, NCHAN = K::NCHAN, UPL = K::UPL;
  constexpr bool FWD = K::FWD;
  constexpr bool BWD_AB = MODE == MODE_DUDIR || MODE == MODE_SIGS || MODE == MODE_DS;  // weights a, beta
  constexpr bool SIGT = MODE == MODE_SIGS || MODE == MODE_DS;     // the sigma_s terms
  __shared__ __attribute__((aligned(16))) float smem[K::SMEM];
  float *stg = smem;                        // [NPU][RC][SW], plane stride PSTG
  float *ring = smem + K::STG;              // [NP][RINGX][kTWP], plane stride PR
  float *uring = ring + K::RINGF;           // [RINGX][kTWP] (forward)
  float *ex = uring + K::URINGF;            // [NP][RC][32] (DUDIR, ADJ)

  const int tid = threadIdx.x;
  const int L = xcd_swizzle(blockIdx.x, a.nblocks);
  const int per_chunk = a.tiles_x * a.tiles_y;
  const int cchunk = L / per_chunk;
  const int rem = L - cchunk * per_chunk;
  const int ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
  const int TH = a.nch * RC;
  const int tx0 = tx * kTW;
  const int c0 = cchunk * a.ch_per_block;
  const int H = a.H, W = a.W, C = a.C;
  const int64_t N = (int64_t)H * W;

  // row-pass role: tid bits = [segment][row bit 0][plane bit 0][row bits 1..][plane bits 1..]
  int r_sg, r_rr, r_p;
  {
    int t = tid;
    r_sg = t % SEGS;
    t /= SEGS;
    const int rr0 = t & 1;
    t >>= 1;
    int p0 = 0;
    if constexpr (NP >= 2) {
      p0 = t & 1;
      t >>= 1;
    }
    r_rr = rr0 + 2 * (t % (RC / 2));
    t /= RC / 2;
    r_p = NP >= 2 ? p0 + 2 * t : t;
  }
  // column-pass role
  const int c_x = tid % kTW;
  const int c_p = (tid / kTW) % NP;
  const int c_sub = tid / (kTW * NP);

  float f0c[NCHAN > 0 ? NCHAN : 1], chm[NCHAN > 0 ? NCHAN : 1];
#pragma unroll
  for (int ch = 0; ch < NCHAN; ++ch) {
    f0c[ch] = c0 + ch < C ? a.f0[c0 + ch] : 0.0f;
    chm[ch] = c0 + ch < C ? 1.0f : 0.0f;
  }

  float acc[NCH_MAX][RUN];
#pragma unroll
  for (int j = 0; j < NCH_MAX; ++j)
#pragma unroll
    for (int i = 0; i < RUN; ++i) acc[j][i] = 0.0f;
  double sacc = 0.0;  // MODE_SIGS

  const int nin = a.nch + LAG;
  // Staging data of one input chunk lives in registers between its global
  // loads and its LDS store: the loads of chunk i+1 are issued right after
  // chunk i is stored, so their latency hides behind chunk i's FIR passes.
  // pm[q][p] is the multiplier of plane p (forward: 1, f~_c; adjoint: beta, a_c).
  constexpr int NPOS = (RC * SW + BT - 1) / BT;
  constexpr int NCH1 = NCHAN > 0 ? NCHAN : 1;
  float pu[NPOS], pf[NPOS][NCH1], pb[NPOS];
  // Loads go through buffer resources based at the first image row of the
  // chunk, with 32-bit byte offsets relative to it.  A position outside the
  // image (or past the staging tile) takes kOffInvalid and reads 0, so the
  // loads are issued without branches or masks, and nothing waits for them
  // until the store one chunk later.  relq[q] = rr * W + gx of position q;
  // colv[q]: its column lies in the image.
  int relq[NPOS];
  bool colv[NPOS];
#pragma unroll
  for (int q = 0; q < NPOS; ++q) {
    const int e = tid + q * BT;
    const int rr = e / SW, j = e - rr * SW;
    const int gx = tx0 - S + j;
    colv[q] = e < RC * SW && j < kTW + 2 * S && gx >= 0 && gx < W;
    relq[q] = rr * W + gx;
  }
  auto fetch = [&](int kk, int icc) {
    // redefined per call, so that no offset is hoisted out of the k loop
    const int gy0 = opaque_s(ty * TH) - S + icc * RC;   // image row of staging row 0
    const int gyb = gy0 > 0 ? gy0 : 0;                  // resource base row
    const int dW = (gy0 - gyb) * W;                     // staging row 0 relative to it
    const int64_t rowoff = (int64_t)gyb * W;
    const __amdgpu_buffer_rsrc_t ru = buf_rsrc(a.u + (int64_t)kk * N + rowoff);
    unsigned off[NPOS];
#pragma unroll
    for (int q = 0; q < NPOS; ++q) {
      const int rr = (tid + q * BT) / SW;
      const bool in = colv[q] && (unsigned)(gy0 + rr) < (unsigned)H;
      const unsigned rel = (unsigned)(relq[q] + dW);   // pixel offset from the base row
      off[q] = in ? rel : kOffInvalid;
      pu[q] = buf_ld(ru, in ? rel * 4u : kOffInvalid);
    }
    if constexpr (MODE == MODE_ADJ) {
      // (beta, a_1..a_3) of a pixel: four dword loads at one offset (the
      // 16-byte buffer load builtin is not used: this compiler lowers it to a
      // single dword)
      const __amdgpu_buffer_rsrc_t rab = buf_rsrc(a.ab + rowoff * 4);
#pragma unroll
      for (int q = 0; q < NPOS; ++q) {
        const unsigned ob = off[q] != kOffInvalid ? off[q] * 16u : kOffInvalid;
        pb[q] = buf_ld(rab, ob);
#pragma unroll
        for (int ch = 0; ch < NCHAN; ++ch) pf[q][ch] = buf_ld(rab, ob + 4u * (unsigned)(1 + ch));
      }
    } else if (a.fpl) {
      // planar f: each channel load is contiguous across the lanes
#pragma unroll
      for (int ch = 0; ch < NCHAN; ++ch) {
        const int cc = c0 + ch < C ? c0 + ch : C - 1;
        const __amdgpu_buffer_rsrc_t rc = buf_rsrc(a.fpl + (int64_t)cc * N + rowoff);
#pragma unroll
        for (int q = 0; q < NPOS; ++q) pf[q][ch] = buf_ld(rc, off[q] != kOffInvalid ? off[q] * 4u : kOffInvalid);
      }
    } else {
      // interleaved f (C <= 3); channels past C re-read channel C-1 and are zeroed by chm
      const __amdgpu_buffer_rsrc_t rf = buf_rsrc(a.f + rowoff * C);
#pragma unroll
      for (int q = 0; q < NPOS; ++q) {
        const unsigned of = off[q] != kOffInvalid ? off[q] * (unsigned)(4 * C) : kOffInvalid;
#pragma unroll
        for (int ch = 0; ch < NCHAN; ++ch) pf[q][ch] = buf_ld(rf, of + 4u * (unsigned)(c0 + ch < C ? c0 + ch : C - 1));
      }
    }
  };
  fetch(0, 0);
  for (int k = 0; k < a.r_eff; ++k) {
#pragma unroll
    for (int ic = 0; ic < NCH_MAX + LAG; ++ic) {
      if (ic < nin) {
        // ---- stage the plane inputs for R rows [ic*RC, ic*RC + RC) -----------
        // (the previous row pass finished reading the staging buffer before the
        // barrier that preceded the previous column pass)
#pragma unroll
        for (int q = 0; q < NPOS; ++q) {
          const int e = tid + q * BT;
          if (e < RC * SW) {
            const int rr = e / SW, j = e - rr * SW;
            const float uq = pu[q];  // 0 outside the image
            if constexpr (MODE == MODE_ADJ)
              stg[rr * SW + j] = pb[q] * uq;  // plane 0: beta u_k
            else
              stg[UPL * K::PSTG + rr * SW + j] = uq;
#pragma unroll
            for (int ch = 0; ch < NCHAN; ++ch) {
              // forward modes: f~ = f - f0; channels past C are zero
              const float fv = MODE == MODE_ADJ ? pf[q][ch] : (pf[q][ch] - f0c[ch]) * chm[ch];
              stg[((HAS_E ? 1 : 0) + ch) * K::PSTG + rr * SW + j] = fv * uq;
            }
          }
        }
        if (ic + 1 < nin)
          fetch(k, ic + 1);
        else if (k + 1 < a.r_eff)
          fetch(k + 1, 0);
        __syncthreads();
        // ---- row pass: horizontal FIR into the ring ---------------------------
        {
          // ring slot of R row q = ic*RC + rr; rows with slot < 2S are mirrored
          // at slot + RING so that column windows never wrap
          const int slot = (ic % (1 + LAG)) * RC + r_rr;
          const bool mirror = slot < 2 * S;
          double win[K::WIN];
          const float4 *src = reinterpret_cast<const float4 *>(&stg[r_p * K::PSTG + r_rr * SW + r_sg * RUN]);
#pragma unroll
          for (int v4 = 0; v4 < K::WIN / 4; ++v4) {
            const float4 q = src[v4];
            win[4 * v4 + 0] = (double)q.x;
            win[4 * v4 + 1] = (double)q.y;
            win[4 * v4 + 2] = (double)q.z;
            win[4 * v4 + 3] = (double)q.w;
          }
          float *dst = &ring[r_p * K::PR + slot * kTWP + r_sg * RUN];
          Window<S, BOX> rw;
          if constexpr (K::VEC_RING) {
            float ov[RUN];
#pragma unroll
            for (int i = 0; i < RUN; ++i) ov[i] = (float)rw.at(a.wr, win, i);
            store_run4<RUN>(dst, ov, mirror, RING * kTWP);
          } else {
            // each output stored as soon as it is formed
#pragma unroll
            for (int i = 0; i < RUN; ++i) {
              const float sf = (float)rw.at(a.wr, win, i);
              dst[i] = sf;
              if (mirror) dst[RING * kTWP + i] = sf;
            }
          }
          if constexpr (SIGT) {
            // the w1' rows, in the second ring
            float *dst2 = dst + NP * K::PR;
#pragma unroll
            for (int i = 0; i < RUN; ++i) {
              const float sf = (float)fir_sym<S>(a.wc, &win[i]);
              dst2[i] = sf;
              if (mirror) dst2[RING * kTWP + i] = sf;
            }
          }
          if constexpr (FWD) {
            if (r_p == 0) {
              // raw u_k at the tile's own columns, for the contraction
              const float *us = &stg[UPL * K::PSTG + r_rr * SW + S + r_sg * RUN];
              float *ud = &uring[slot * kTWP + r_sg * RUN];
              if constexpr (K::VEC_RING) {
                float ov[RUN];
#pragma unroll
                for (int i = 0; i < RUN; ++i) ov[i] = us[i];
                store_run4<RUN>(ud, ov, mirror, RING * kTWP);
              } else {
#pragma unroll
                for (int i = 0; i < RUN; ++i) {
                  const float uv = us[i];
                  ud[i] = uv;
                  if (mirror) ud[RING * kTWP + i] = uv;
                }
              }
            }
          }
        }
        __syncthreads();
        // ---- column pass for output chunk oc = ic - LAG -----------------------
        if (ic >= LAG) {
          const int oc = ic - LAG;
          // local output rows o0 .. o0+RUN-1 need R rows o0 .. o0+RUN+2S-1
          const int o0 = oc * RC + c_sub * RUN;
          const int b0 = (oc * RC) % RING + c_sub * RUN;   // < RING, window ends < RINGX
          const float *col = &ring[c_p * K::PR + b0 * kTWP + c_x];
          double win[RUN + 2 * S];
#pragma unroll
          for (int j = 0; j < RUN + 2 * S; ++j) win[j] = col[j * kTWP];
          // the forward and the adjoint passes use one tap set for both passes
          const double *wcol = a.wr;
          if constexpr (FWD) {
            const float *ucol = &uring[(b0 + S) * kTWP + c_x];
            Window<S, BOX> cw;
#pragma unroll
            for (int i = 0; i < RUN; ++i) {
              const double z = cw.at(wcol, win, i);
              acc[oc][i] = fmaf(ucol[i * kTWP], (float)z, acc[oc][i]);
            }
          } else {
            const int ty0k = opaque(ty * TH);
            const int gx = tx0 + c_x;
            const float *uk = a.u + (int64_t)k * N;
            float cu[SIGT ? RUN : 1];
#pragma unroll
            for (int i = 0; i < RUN; ++i) {
              // SIGS: w1' down the w1 rows here, w1 down the w1' rows below
              const double z = fir_sym<S>(SIGT ? a.wc : wcol, &win[i]);
              const int gy = ty0k + o0 + i;
              const bool inpix = oc < a.nch && gy < H && gx < W;
              const int pix = inpix ? gy * W + gx : 0;
              if constexpr (BWD_AB) {
                const float coef = inpix ? a.ab[(int64_t)pix * 4 + c_p] : 0.0f;
                if constexpr (MODE == MODE_DUDIR) {
                  ex[(c_p * RC + c_sub * RUN + i) * kTW + c_x] = coef * (float)z;
                } else {
                  const float uo = inpix ? uk[pix] : 0.0f;
                  sacc = fma((double)(uo * coef), z, sacc);
                  if constexpr (SIGT) cu[i] = uo * coef;
                  if constexpr (MODE == MODE_DS)  // du_dir from the w1 column pass of the same rows
                    ex[(c_p * RC + c_sub * RUN + i) * kTW + c_x] = coef * (float)fir_sym<S>(wcol, &win[i]);
                }
              } else {  // MODE_ADJ
                float coef = 1.0f;
                if (c_p > 0) {
                  const int ch = c_p - 1;
                  coef = (inpix && ch < C) ? a.f[(int64_t)pix * C + ch] - f0c[ch] : 0.0f;
                  const float uo = inpix ? uk[pix] : 0.0f;
                  acc[oc][i] = fmaf(uo, (float)z, acc[oc][i]);
                }
                ex[(c_p * RC + c_sub * RUN + i) * kTW + c_x] = coef * (float)z;
              }
            }
            if constexpr (SIGT) {
#pragma unroll
              for (int j = 0; j < RUN + 2 * S; ++j) win[j] = col[NP * K::PR + j * kTWP];
#pragma unroll
              for (int i = 0; i < RUN; ++i) sacc = fma((double)cu[i], fir_sym<S>(wcol, &win[i]), sacc);
            }
          }
          if constexpr (MODE == MODE_DUDIR || MODE == MODE_ADJ || MODE == MODE_DS) {
            // combine the NP planes of each pixel of the chunk
            __syncthreads();
            const int ty0k = opaque(ty * TH);
            float *outk = a.plane_out + (int64_t)k * N;
#pragma unroll
            for (int m = 0; m < RC * kTW / BT; ++m) {
              const int pl = tid + m * BT;
              const int row = pl / kTW, cx = pl % kTW;
              const int gy = ty0k + oc * RC + row, gx = tx0 + cx;
              if (oc < a.nch && gy < H && gx < W) {
                float s = 0.0f;
#pragma unroll
                for (int p = 0; p < NP; ++p) s += ex[(p * RC + row) * kTW + cx];
                const int64_t pix = (int64_t)gy * W + gx;
                if constexpr (MODE == MODE_ADJ) s += a.plane_in[(int64_t)k * N + pix];
                outk[pix] = s;
              }
            }
          }
        }
      }
    }
  }

  // ---- epilogues ----------------------------------------------------------
  const int ty0 = ty * TH;
  const int gx = tx0 + c_x;
  if constexpr (MODE == MODE_DUDIR) {
    return;
  } else if constexpr (SIGT) {
    // block sum of the per-thread FP64 partials, in a fixed order
    __syncthreads();
    double *red = reinterpret_cast<double *>(smem);
    red[tid] = sacc;
    __syncthreads();
    for (int h = BT / 2; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) a.partials[blockIdx.x] = red[0];
    return;
  } else if constexpr (MODE == MODE_ADJ) {
    // df_c = sum_k u_k Ya_kc; pixels that took the eta <= 0 guard output f,
    // so dL/df there is G itself
    const int ch = c_p - 1;
    if (ch >= 0 && ch < C && gx < W) {
#pragma unroll
      for (int oc = 0; oc < NCH_MAX; ++oc)
#pragma unroll
        for (int i = 0; i < RUN; ++i) {
          const int gy = ty0 + oc * RC + c_sub * RUN + i;
          if (oc < a.nch && gy < H) {
            const int64_t pix = (int64_t)gy * W + gx;
            const float e = a.eta[pix];
            float v = acc[oc][i];
            if (!(e > 0.0f && isfinite(e))) v += a.G[pix * C + ch];
            a.df[pix * C + ch] = v;
          }
        }
    }
    return;
  } else if constexpr (HAS_E && NP == 1) {
#pragma unroll
    for (int oc = 0; oc < NCH_MAX; ++oc)
#pragma unroll
      for (int i = 0; i < RUN; ++i) {
        const int gy = ty0 + oc * RC + c_sub * RUN + i;
        if (oc < a.nch && gy < H && gx < W) {
          const int64_t pix = (int64_t)gy * W + gx;
          if (a.eta_buf) a.eta_buf[pix] = acc[oc][i];
          if (a.eta_out) a.eta_out[pix] = acc[oc][i];
        }
      }
    return;
  } else {
    float *etab = smem;  // [TH][32], reuses the staging and ring buffers
    if constexpr (HAS_E) {
      __syncthreads();
      if (c_p == 0) {
#pragma unroll
        for (int oc = 0; oc < NCH_MAX; ++oc)
#pragma unroll
          for (int i = 0; i < RUN; ++i) {
            const int o = oc * RC + c_sub * RUN + i;
            if (oc < a.nch) {
              etab[o * kTW + c_x] = acc[oc][i];
              const int gy = ty0 + o;
              if (a.eta_out && gy < H && gx < W) a.eta_out[(int64_t)gy * W + gx] = acc[oc][i];
            }
          }
      }
      __syncthreads();
    }
    const int ch = c_p - (HAS_E ? 1 : 0);
    const int gc = c0 + ch;
    if (ch >= 0 && gc < C && gx < W) {
      const float f0 = a.f0[gc];
#pragma unroll
      for (int oc = 0; oc < NCH_MAX; ++oc)
#pragma unroll
        for (int i = 0; i < RUN; ++i) {
          const int o = oc * RC + c_sub * RUN + i;
          const int gy = ty0 + o;
          if (oc < a.nch && gy < H) {
            const int64_t pix = (int64_t)gy * W + gx;
            const float eta = HAS_E ? etab[o * kTW + c_x] : a.eta_buf[pix];
            float g;
            if (eta > 0.0f && isfinite(eta))
              g = acc[oc][i] / eta + f0;
            else
              g = a.f[pix * C + gc];
            a.out[pix * C + gc] = g;
          }
        }
    }
  }
}

// Compute units of the current device (cached per device; contexts on other
// host threads may fill the cache concurrently, each storing the same value).
inline int device_cus() {
  static std::atomic<int> cus[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = cus[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    int n = 0;
    v = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0 ? n : 256;
    cus[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}

// Tile geometry and launch of one kernel instantiation.
template <int S, int NP, bool HAS_E, int RC, int MODE, int BT = kBlock, bool BOX = false>
hipError_t launch_one(ConvArgs a, hipStream_t s, int ch_per_block, int nchunks_c, int *nblocks_out = nullptr) {
  using K = Cfg<S, NP, HAS_E, RC, MODE, BT, BOX>;
  a.ch_per_block = ch_per_block;
  a.tiles_x = (a.W + kTW - 1) / kTW;
  auto blocks = [&](int n) {
    const int th = n * RC;
    return (int64_t)a.tiles_x * ((a.H + th - 1) / th) * nchunks_c;
  };
  // do not use more chunks than the image needs
  const int need = (a.H + RC - 1) / RC;
  int nch = 1;
  if (a.force_nch > 0) {
    nch = a.force_nch < K::NCH_MAX ? a.force_nch : K::NCH_MAX;
  } else {
    // a block streams nch + LAG input chunks for its nch output chunks, and
    // blocks run in rounds of one per CU (512 threads: a whole CU's LDS) or
    // two (256 threads): take the chunk count of the fewest chunk-steps,
    // rounds x (nch + LAG), the larger one on ties
    const int64_t slots = (int64_t)device_cus() * (BT == 512 ? 1 : 2);
    int64_t best = -1;
    for (int n = 1; n <= K::NCH_MAX && n <= need; ++n) {
      const int64_t cost = (blocks(n) + slots - 1) / slots * (n + K::LAG);
      if (best < 0 || cost <= best) {
        best = cost;
        nch = n;
      }
    }
  }
  if (nch > need) nch = need;
  a.nch = nch;
  a.tiles_y = (a.H + nch * RC - 1) / (nch * RC);
  const int64_t nb = (int64_t)a.tiles_x * a.tiles_y * nchunks_c;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  a.nblocks = (int)nb;
  if (nblocks_out) *nblocks_out = a.nblocks;
  hipLaunchKernelGGL((conv_kernel<S, NP, HAS_E, RC, MODE, BT, BOX>), dim3(a.nblocks), dim3(BT), 0, s, a);
  return hipGetLastError();
}

}  // namespace conv
}  // namespace nkf
