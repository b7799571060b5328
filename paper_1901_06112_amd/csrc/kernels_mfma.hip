// Distance step on the matrix cores for high-dimensional guides (hyperspectral
// bands, nonlocal-means patches): the cross kernel B(i, x) = k(c_i, p(x)) of
// Eq. (defB) and the k-means assignment (Section III) in GEMM form,
//     |p - c|^2 = |p~|^2 + |c~|^2 - 2 p~.c~,   p~ = p - mu, c~ = c - mu,
// with the centred guide and landmarks rounded to BF16 or FP16 for the MFMA
// product (FP32 accumulation), the squared norms taken in FP32 from the
// unrounded centred values, and the result clamped at zero.  mu is the mean
// guide value (per channel for patch guides), which makes |p~| and |c~| small
// next to |p| and |c| and keeps the cancellation in the GEMM form within the
// 16-bit rounding.
//
// Tiles.  A block of NW waves walks tiles of TP = 16 NW pixels; wave w owns
// pixels 16w .. 16w+15 of the tile.  The tile's guide data is staged once in
// LDS as centred FP32 (the "raw tile"):
//   explicit / self guides: TP consecutive pixels, D values each;
//   patch guides: TP consecutive pixels of one image row plus the rows and
//     columns their patches reach (symmetric padding), so that the
//     (2pr+1)^2 C patch values of a pixel are 2pr+1 runs of (2pr+1) C
//     contiguous floats of the raw tile.
// The GEMM runs over a permuted dimension axis: each run (one patch row, or
// the whole vector of an explicit guide) is padded to a multiple of 8 so that
// every 8-element MFMA operand chunk lies inside one run and is read straight
// from the raw tile.  The landmarks are permuted the same way; a distance
// does not depend on the order of the dimensions.
//
// k-means: the argmin of |c~|^2 - 2 p~.c~ (lowest index on ties), then each
// wave adds its pixels' centred guide vectors to the block's per-cluster FP32
// sums in LDS (lanes over dimensions, so the atomics of one instruction hit
// distinct words), written out once per block as FP64 partials.
// Embedding: the products as 16-bit hi + lo pairs (three MFMA passes, about
// twice the bits of the k-means products, whose decisions only need the
// nearest landmark), b = exp(-d^2 / (2 sigma_r^2)) into an LDS tile, then
// u^T = F^T b^T on v_mfma_f32_16x16x4_f32, each wave keeping its rows of F^T
// in registers for the whole launch.
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>

#include <type_traits>

#include "device_common.h"

namespace nkf {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int kMaxChunks = 64;   // 8-element chunks of the permuted axis (Dp <= 512)
constexpr int kMaxDc = 4;        // dimensions per lane in the accumulation (D <= 256)
constexpr int kMaxBlocks = 256;  // k-means partial slots
constexpr int kMeanBlocks = 1024;
constexpr int kEmbedBlocks = 512;
constexpr size_t kLdsMax = 160 * 1024;

template <int PREC>
struct Half;
template <>
struct Half<1> {
  using T = __bf16;
  using V = bf16x8;
  static __device__ __forceinline__ floatx4 mma(V a, V b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Half<2> {
  using T = _Float16;
  using V = f16x8;
  static __device__ __forceinline__ floatx4 mma(V a, V b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

struct MArgs {
  Guide g;
  int64_t N;
  const float *c;    // [r][D] landmarks (guide order)
  const float *mu;   // centring offsets: [C] for patch guides, [D] otherwise
  int r, RP;         // RP = 16 NT >= r: landmark rows of the MFMA tiles
  // permuted axis: NR runs of RL values, each padded to RLP (multiple of 8);
  // Dp = NR * RLP rounded up to 32; DS = Dp + 8 (landmark row stride, halves)
  int NR, RL, RLP, Dp, DS;
  // raw tile: value (pixel i, run q, element e) at q * rowstride + i * pxstride + e
  int rowstride, pxstride, raw_floats;  // raw_floats includes muf floats for the offsets
  int muf;
  int tiles_x;       // patch guides: tiles per image row
  int ntiles;
  const void *ctg;   // [RP][DS] 16-bit centred landmarks on the permuted axis
  const void *ctg_lo;  // [RP][DS] their rounding remainders, also 16-bit (embedding)
  const float *cn2g; // [RP] their FP32 squared norms (FLT_MAX for padding)
  // k-means
  int *labels;       // nullable
  double *partials;  // [gridDim][r][D+1]
  int lds_acc;       // per-cluster sums in LDS (else FP64 atomics into the block's slot)
  // embedding
  const float *F32;  // [r][r_eff]
  int r_eff, RE;     // RE = r_eff rounded up to 16
  float inv2s2;
  float *u;          // [r_eff][N]
  float *bbuf;       // [ntiles][TP][RP] cross-kernel tiles of the split embedding
};

__device__ __forceinline__ float mu_of(const MArgs &a, int d) {
  return a.mu[a.g.kind == GUIDE_PATCH ? d % a.g.C : d];
}

// Pixels of tile t: linear indices x0 .. x0 + nvalid - 1 (consecutive in
// both layouts); patch tiles also record their image row and first column.
struct TileInfo {
  int64_t x0;
  int nvalid, y, col0;
};

template <int TP>
__device__ __forceinline__ TileInfo tile_info(const MArgs &a, int t) {
  TileInfo ti;
  if (a.g.kind == GUIDE_PATCH) {
    ti.y = t / a.tiles_x;
    ti.col0 = (t - ti.y * a.tiles_x) * TP;
    ti.x0 = (int64_t)ti.y * a.g.W + ti.col0;
    ti.nvalid = a.g.W - ti.col0 < TP ? a.g.W - ti.col0 : TP;
  } else {
    ti.y = ti.col0 = 0;
    ti.x0 = (int64_t)t * TP;
    ti.nvalid = a.N - ti.x0 < TP ? (int)(a.N - ti.x0) : TP;
  }
  return ti;
}

// Centred FP32 guide data of one tile into raw; mus is the block's LDS copy
// of the centring offsets.  For explicit and self guides every thread issues
// its loads in batches of eight (float4 where D % 4 == 0) before storing any,
// so a tile costs about one memory latency instead of one per element.
template <int TP, int BT>
__device__ __forceinline__ void stage_raw(const MArgs &a, const TileInfo &ti, float *raw, const float *mus) {
  const Guide &g = a.g;
  const int tid = threadIdx.x;
  if (g.kind == GUIDE_PATCH) {
    const int C = g.C, PW = 2 * g.pr + 1, TPR = TP + 2 * g.pr;
    // (patch row q, tile column j) pairs; the C channels of a column are contiguous
    for (int idx = tid; idx < PW * TPR; idx += BT) {
      const int q = idx / TPR, j = idx - q * TPR;
      const int yy = sym_index(ti.y + q - g.pr, g.H);
      const int xs = ti.col0 + j - g.pr;
      float *dst = raw + q * a.rowstride + j * C;
      if (xs < g.W + g.pr) {  // columns past the padded image edge are never read
        const float *src = g.f + ((int64_t)yy * g.W + sym_index(xs, g.W)) * C;
        for (int ch = 0; ch < C; ++ch) dst[ch] = src[ch] - mus[ch];
      } else {
        for (int ch = 0; ch < C; ++ch) dst[ch] = 0.0f;
      }
    }
  } else {
    const int D = g.D;
    const float *src = (g.kind == GUIDE_EXPLICIT ? g.p : g.f) + ti.x0 * D;
    const int ntot = TP * D, nval = ti.nvalid * D;
    if ((D & 3) == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
      // float4 groups (never across pixels: D % 4 == 0), walked with
      // incremental (pixel, dimension) indices
      constexpr int NB = 8, STEP = 4 * BT;
      const int di = STEP / D, dd = STEP - di * D;
      int i = (4 * tid) / D, d = 4 * tid - i * D;
      for (int b = 4 * tid; b < ntot; b += NB * STEP) {
        float4 v[NB];
        int pi[NB], pd[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int e = b + k * STEP;
          pi[k] = i;
          pd[k] = d;
          v[k] = e < nval ? *reinterpret_cast<const float4 *>(src + e) : make_float4(0.f, 0.f, 0.f, 0.f);
          i += di;
          d += dd;
          if (d >= D) {
            d -= D;
            ++i;
          }
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int e = b + k * STEP;
          if (e >= ntot) break;
          float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
          if (e < nval) {
            const float *m = mus + pd[k];
            o = make_float4(v[k].x - m[0], v[k].y - m[1], v[k].z - m[2], v[k].w - m[3]);
          }
          *reinterpret_cast<float4 *>(raw + pi[k] * a.pxstride + pd[k]) = o;
        }
      }
    } else {
      // element e = i D + d of the tile, walked with incremental (i, d)
      constexpr int NB = 8;
      const int di = BT / D, dd = BT - (BT / D) * D;
      int i = tid / D, d = tid - (tid / D) * D;
      for (int b = tid; b < ntot; b += NB * BT) {
        float v[NB];
        int pi[NB], pd[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int e = b + k * BT;
          pi[k] = i;
          pd[k] = d;
          v[k] = e < nval ? src[e] : 0.0f;
          i += di;
          d += dd;
          if (d >= D) {
            d -= D;
            ++i;
          }
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int e = b + k * BT;
          if (e >= ntot) break;
          raw[pi[k] * a.pxstride + pd[k]] = e < nval ? v[k] - mus[pd[k]] : 0.0f;
        }
      }
    }
  }
}

// Register prefetch of an explicit / self guide tile in one batch of float4
// groups (D % 4 == 0, 16-byte aligned rows, TP D <= 32 BT): the k-means loop
// issues the loads of its next tile before processing the current one, so
// they are in flight during its products and sums.
template <int TP, int BT>
struct TilePrefetch {
  float4 v[8];
  static __host__ __device__ __forceinline__ bool usable(const MArgs &a) {
    const float *base = a.g.kind == GUIDE_EXPLICIT ? a.g.p : a.g.f;
    return a.g.kind != GUIDE_PATCH && (a.g.D & 3) == 0 && (reinterpret_cast<uintptr_t>(base) & 15) == 0 &&
           TP * a.g.D <= 32 * BT;
  }
  __device__ __forceinline__ void load(const MArgs &a, const TileInfo &ti) {
    const int D = a.g.D;
    const float *src = (a.g.kind == GUIDE_EXPLICIT ? a.g.p : a.g.f) + ti.x0 * D;
    const int nval = ti.nvalid * D;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = 4 * (int)threadIdx.x + k * 4 * BT;
      v[k] = e < nval ? *reinterpret_cast<const float4 *>(src + e) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  __device__ __forceinline__ void store(const MArgs &a, const TileInfo &ti, float *raw, const float *mus) const {
    const int D = a.g.D, nval = ti.nvalid * D, ntot = TP * D;
    const int di = 4 * BT / D, dd = 4 * BT - di * D;
    int i = (4 * (int)threadIdx.x) / D, d = 4 * (int)threadIdx.x - i * D;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = 4 * (int)threadIdx.x + k * 4 * BT;
      if (e >= ntot) break;
      float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < nval) o = make_float4(v[k].x - mus[d], v[k].y - mus[d + 1], v[k].z - mus[d + 2], v[k].w - mus[d + 3]);
      *reinterpret_cast<float4 *>(raw + i * a.pxstride + d) = o;
      i += di;
      d += dd;
      if (d >= D) {
        d -= D;
        ++i;
      }
    }
  }
};

// The same for patch guides with C <= 4 whose tile window (2pr+1 rows of
// TP + 2pr columns) has at most 2 BT columns: each thread holds the centred
// C values of up to two (patch row, column) pairs (zeros past the padded
// image edge, as stage_raw writes them).
template <int TP, int BT>
struct PatchPrefetch {
  float v[2][4];
  static __host__ __device__ __forceinline__ bool usable(const MArgs &a) {
    return a.g.kind == GUIDE_PATCH && a.g.C <= 4 && (2 * a.g.pr + 1) * (TP + 2 * a.g.pr) <= 2 * BT;
  }
  __device__ __forceinline__ void load(const MArgs &a, const TileInfo &ti, const float *mus) {
    const Guide &g = a.g;
    const int C = g.C, TPR = TP + 2 * g.pr, npair = (2 * g.pr + 1) * TPR;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int idx = (int)threadIdx.x + k * BT;
      const int q = idx / TPR, j = idx - q * TPR;
      const int xs = ti.col0 + j - g.pr;
      const bool ok = idx < npair && xs < g.W + g.pr;  // columns past the padded edge are never read
      const float *src =
          g.f + ((int64_t)sym_index(ok ? ti.y + q - g.pr : 0, g.H) * g.W + sym_index(ok ? xs : 0, g.W)) * C;
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) v[k][ch] = ok && ch < C ? src[ch] - mus[ch] : 0.0f;
    }
  }
  __device__ __forceinline__ void store(const MArgs &a, float *raw) const {
    const Guide &g = a.g;
    const int C = g.C, TPR = TP + 2 * g.pr, npair = (2 * g.pr + 1) * TPR;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int idx = (int)threadIdx.x + k * BT;
      if (idx >= npair) break;
      const int q = idx / TPR, j = idx - q * TPR;
      float *dst = raw + q * a.rowstride + j * C;
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
        if (ch < C) dst[ch] = v[k][ch];
    }
  }
};

// The block's copy of the centring offsets sits at the end of the raw area.
__device__ __forceinline__ float *raw_mu(const MArgs &a, float *raw) { return raw + a.raw_floats - a.muf; }
__device__ __forceinline__ void load_mu(const MArgs &a, float *mus, int BT) {
  const int M = a.g.kind == GUIDE_PATCH ? a.g.C : a.g.D;
  for (int e = threadIdx.x; e < M; e += BT) mus[e] = a.mu[e];
}

// Chunk table of the permuted axis (raw offset without the pixel term, and
// number of valid elements of each 8-element chunk) and, when dmap is given,
// the raw offset of each guide dimension d (for the accumulation).
__device__ __forceinline__ void build_tables(const MArgs &a, int *tab_off, int *tab_nv, int *dmap, int BT) {
  for (int q8 = threadIdx.x; q8 < a.Dp / 8; q8 += BT) {
    const int d0 = 8 * q8, q = d0 / a.RLP, e0 = d0 - q * a.RLP;
    int nv = 0;
    if (q < a.NR) nv = a.RL - e0 >= 8 ? 8 : (a.RL - e0 > 0 ? a.RL - e0 : 0);
    tab_off[q8] = q < a.NR ? q * a.rowstride + e0 : 0;
    tab_nv[q8] = nv;
  }
  if (dmap)
    for (int d = threadIdx.x; d < a.g.D; d += BT) {
      const int q = d / a.RL;
      dmap[d] = q * a.rowstride + (d - q * a.RL);
    }
}

// Centred 16-bit landmarks on the permuted axis, the 16-bit rounding of what
// the first rounding left (hi + lo carries about twice the bits), and their
// FP32 squared norms (padded landmarks get FLT_MAX so that they never win an
// argmin), once per launch: one wave per landmark row.
template <int PREC>
__global__ __launch_bounds__(64) void prep_landmarks_kernel(MArgs a, typename Half<PREC>::T *ctg,
                                                            typename Half<PREC>::T *ctg_lo, float *cn2g) {
  using T = typename Half<PREC>::T;
  const int k = blockIdx.x, lane = threadIdx.x, D = a.g.D;
  float s = 0.0f;
  for (int dd = lane; dd < a.DS; dd += 64) {
    const int q = dd / a.RLP, el = dd - q * a.RLP;
    float v = 0.0f;
    if (k < a.r && dd < a.Dp && q < a.NR && el < a.RL) {
      const int d = q * a.RL + el;
      v = a.c[k * D + d] - mu_of(a, d);
    }
    s = fmaf(v, v, s);
    const T hv = (T)v;
    ctg[k * a.DS + dd] = hv;
    ctg_lo[k * a.DS + dd] = (T)(v - (float)hv);
  }
  s = wave_sum(s);
  if (lane == 0) cn2g[k] = k < a.r ? s : FLT_MAX;
}

// copy the prepared landmarks into LDS (16-byte vectors)
__device__ __forceinline__ void load_landmarks(const MArgs &a, void *ct, float *cn2, int BT,
                                               void *ct_lo = nullptr) {
  const int n16 = a.RP * a.DS * 2 / 16;  // RP * DS halves, DS a multiple of 8
  const uint4 *src = reinterpret_cast<const uint4 *>(a.ctg);
  uint4 *dst = reinterpret_cast<uint4 *>(ct);
  for (int e = threadIdx.x; e < n16; e += BT) dst[e] = src[e];
  if (ct_lo) {
    const uint4 *sl = reinterpret_cast<const uint4 *>(a.ctg_lo);
    uint4 *dl = reinterpret_cast<uint4 *>(ct_lo);
    for (int e = threadIdx.x; e < n16; e += BT) dl[e] = sl[e];
  }
  for (int k = threadIdx.x; k < a.RP; k += BT) cn2[k] = a.cn2g[k];
}

// acc[t][i] = p~(pixel 16w + 4 rq + i) . c~(landmark 16t + col) for this
// wave's 16 pixels and all RP landmarks; with NORMS, s2 = |p~|^2 (FP32, from
// the unrounded values) of pixel 16w + (lane & 15).  With SPLIT (ct_lo holds
// the landmarks' 16-bit remainders) each operand is a 16-bit pair hi + lo and
// the product takes hi.hi + lo.hi + hi.lo: three MFMA passes whose result
// carries about twice the bits of one (lo.lo is below their rounding).
template <int PREC, int NT, bool NORMS, bool SPLIT = false>
__device__ __forceinline__ void tile_products(const MArgs &a, const float *raw, const int *tab_off,
                                              const int *tab_nv, const typename Half<PREC>::T *ct,
                                              floatx4 (&acc)[NT], float &s2,
                                              const typename Half<PREC>::T *ct_lo = nullptr) {
  using T = typename Half<PREC>::T;
  using V = typename Half<PREC>::V;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4;
  const int pofs = (16 * w + row) * a.pxstride;
  const bool aligned = a.g.kind != GUIDE_PATCH;  // explicit rows: 16-byte aligned chunks
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  s2 = 0.0f;
  for (int s = 0; s < a.Dp / 32; ++s) {
    const int q8 = 4 * s + kq;
    const float *src = raw + tab_off[q8] + pofs;
    const int nv = tab_nv[q8];
    float x[8];
    if (aligned) {
      const float4 lo = *reinterpret_cast<const float4 *>(src);
      const float4 hi = *reinterpret_cast<const float4 *>(src + 4);
      x[0] = lo.x, x[1] = lo.y, x[2] = lo.z, x[3] = lo.w;
      x[4] = hi.x, x[5] = hi.y, x[6] = hi.z, x[7] = hi.w;
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) x[j] = src[j];
    }
    V av, avl;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float v = j < nv ? x[j] : 0.0f;
      if constexpr (NORMS) s2 = fmaf(v, v, s2);
      av[j] = (T)v;
      if constexpr (SPLIT) avl[j] = (T)(v - (float)av[j]);
    }
    V bv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bv[t] = *reinterpret_cast<const V *>(&ct[(16 * t + row) * a.DS + 32 * s + 8 * kq]);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = Half<PREC>::mma(av, bv[t], acc[t]);
    if constexpr (SPLIT) {
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = Half<PREC>::mma(avl, bv[t], acc[t]);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        bv[t] = *reinterpret_cast<const V *>(&ct_lo[(16 * t + row) * a.DS + 32 * s + 8 * kq]);
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = Half<PREC>::mma(av, bv[t], acc[t]);
    }
  }
  if constexpr (NORMS) {
    s2 += __shfl_xor(s2, 16, 64);
    s2 += __shfl_xor(s2, 32, 64);
  }
}

// ---- k-means: assignment fused with the per-cluster sums --------------------
// LDS bytes of the k-means kernel before the one-hot matrix (halves of size hb)
__host__ __device__ __forceinline__ size_t lloyd_base_bytes(const MArgs &a, int TP, int hb) {
  return (size_t)hb * a.RP * a.DS + sizeof(float) * ((size_t)a.raw_floats + 8 + a.RP) +
         sizeof(int) * (2 * kMaxChunks + TP + a.g.D + a.RP);
}

// Minimum of (value, index) over the 16 lanes of a DPP row, lowest index on
// ties (rotations by 8 and 4 within the row, then quad swaps): every lane of
// the row ends with the row's minimum.
__device__ __forceinline__ void row16_argmin(float &best, int &bi) {
  auto step = [&](auto ctrl) {
    constexpr int C = decltype(ctrl)::value;
    const float ob = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(best), C, 0xf, 0xf, false));
    const int oi = __builtin_amdgcn_update_dpp(0, bi, C, 0xf, 0xf, false);
    const bool take = (ob < best) | ((ob == best) & (oi < bi));  // no short circuit: no branch
    best = take ? ob : best;
    bi = take ? oi : bi;
  };
  step(std::integral_constant<int, 0x128>{});  // row_ror:8
  step(std::integral_constant<int, 0x124>{});  // row_ror:4
  step(std::integral_constant<int, 0x4E>{});   // quad_perm [2,3,0,1]
  step(std::integral_constant<int, 0xB1>{});   // quad_perm [1,0,3,2]
}

// Split of an FP32 value into 16-bit parts whose sum restores it to about
// 2^-22 (FP16: hi + lo) or 2^-24 (BF16: hi + mid + lo) relative.
template <int PREC>
struct Split;
template <>
struct Split<1> {
  static constexpr int NPART = 3;
  static __device__ __forceinline__ void parts(float v, __bf16 *o) {
    const __bf16 h = (__bf16)v;
    const float r1 = v - (float)h;
    const __bf16 m = (__bf16)r1;
    o[0] = h;
    o[1] = m;
    o[2] = (__bf16)(r1 - (float)m);
  }
};
template <>
struct Split<2> {
  static constexpr int NPART = 2;
  static __device__ __forceinline__ void parts(float v, _Float16 *o) {
    const _Float16 h = (_Float16)v;
    o[0] = h;
    o[1] = (_Float16)(v - (float)h);
  }
};

// MDT == 0: per-cluster sums with LDS (or global FP64) atomics, lanes over the
// dimensions.  MDT > 0: the sums as a GEMM on the matrix cores,
//     S[k][d] += sum_px [label(px) == k] p~(px, d),
// A = one-hot labels (16 clusters x 32 pixels), B = the centred guide values
// split into 16-bit parts (32 pixels x 16 dimensions), FP32 accumulators held
// by the waves for the whole launch: wave w owns the dimension tiles
// w + NW m (m < MDT) for all NT cluster tiles.  The counts are integer LDS
// increments in the argmin (exact, order-free), so D = 16 n guides need no
// extra tile for a count column and every wave owns the same number of tiles.
template <int PREC, int NT, int BT, int MDT, int PF>
__global__ __launch_bounds__(BT) void lloyd_mfma_kernel(MArgs a) {
  using T = typename Half<PREC>::T;
  using V = typename Half<PREC>::V;
  constexpr int NW = BT / 64, TP = 16 * NW;
  constexpr int NPART = Split<PREC>::NPART;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T *ct = reinterpret_cast<T *>(smem_raw);                                    // [RP][DS]
  float *raw = reinterpret_cast<float *>(ct + (size_t)a.RP * a.DS);           // [raw_floats + 8]
  float *cn2 = raw + a.raw_floats + 8;                                        // [RP]
  int *tab_off = reinterpret_cast<int *>(cn2 + a.RP);                         // [kMaxChunks]
  int *tab_nv = tab_off + kMaxChunks;                                         // [kMaxChunks]
  int *labs = tab_nv + kMaxChunks;                                            // [TP]
  int *dmap = labs + TP;                                                      // [D]
  int *cnt = dmap + a.g.D;                                                    // [RP] (GEMM path)
  float *sacc = reinterpret_cast<float *>(cnt + a.RP);                        // [r][D+1] (lds_acc)
  // GEMM path: one-hot label matrix [RP][TP + 8] (16-bit 0 / 1), 16-byte aligned
  T *oh = reinterpret_cast<T *>(smem_raw + ((lloyd_base_bytes(a, TP, sizeof(T)) + 15) & ~(size_t)15));
  constexpr int OHS = TP + 8;
  const int D = a.g.D, DA = D + 1;
  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = lane & 15, rq = lane >> 4;
  double *slot = a.partials + (size_t)blockIdx.x * a.r * DA;

  load_landmarks(a, ct, cn2, BT);
  build_tables(a, tab_off, tab_nv, dmap, BT);
  load_mu(a, raw_mu(a, raw), BT);
  for (int e = tid; e < TP; e += BT) labs[e] = -1;
  if constexpr (MDT > 0) {
    for (int e = tid; e < a.RP * OHS; e += BT) oh[e] = (T)0.0f;
    for (int e = tid; e < a.RP; e += BT) cnt[e] = 0;
  } else {
    if (a.lds_acc) {
      for (int e = tid; e < a.r * DA; e += BT) sacc[e] = 0.0f;
    } else {
      for (int e = tid; e < a.r * DA; e += BT) slot[e] = 0.0;
    }
  }
  __syncthreads();
  // raw-tile offsets: atomic path, dimensions d = lane + 64 m; GEMM path,
  // dimension 16 (w + NW m) + col (-2: the count column, -1: padding)
  int doff[MDT > 0 ? MDT : kMaxDc];
  if constexpr (MDT == 0) {
#pragma unroll
    for (int m = 0; m < kMaxDc; ++m) doff[m] = lane + 64 * m < D ? dmap[lane + 64 * m] : -1;
  } else {
#pragma unroll
    for (int m = 0; m < MDT; ++m) {
      const int d = 16 * (w + NW * m) + col;
      doff[m] = d < D ? dmap[d] : -1;
    }
  }
  const int ndt = (D + 15) / 16;  // dimension tiles of the GEMM sums
  // dimension tiles w + NW m (m < MDT) owned by this wave
  const int nown = MDT > 0 ? max(0, min(MDT, (ndt - w + NW - 1) / NW)) : 0;
  floatx4 sacc_r[MDT > 0 ? MDT : 1][NT];
#pragma unroll
  for (int m = 0; m < (MDT > 0 ? MDT : 1); ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) sacc_r[m][t] = floatx4{0.f, 0.f, 0.f, 0.f};

  // PF (chosen by the host): 1 = TilePrefetch, 2 = PatchPrefetch, 0 = none;
  // the offsets in LDS are complete after the barrier at the loop head
  TilePrefetch<TP, BT> pre;
  PatchPrefetch<TP, BT> ppre;
  if constexpr (PF == 2) __syncthreads();
  if ((int)blockIdx.x < a.ntiles) {
    if constexpr (PF == 1) pre.load(a, tile_info<TP>(a, blockIdx.x));
    if constexpr (PF == 2) ppre.load(a, tile_info<TP>(a, blockIdx.x), raw_mu(a, raw));
  }
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const TileInfo ti = tile_info<TP>(a, t);
    __syncthreads();
    if constexpr (PF == 1)
      pre.store(a, ti, raw, raw_mu(a, raw));
    else if constexpr (PF == 2)
      ppre.store(a, raw);
    else
      stage_raw<TP, BT>(a, ti, raw, raw_mu(a, raw));
    __syncthreads();
    if (t + (int)gridDim.x < a.ntiles) {
      if constexpr (PF == 1) pre.load(a, tile_info<TP>(a, t + gridDim.x));
      if constexpr (PF == 2) ppre.load(a, tile_info<TP>(a, t + gridDim.x), raw_mu(a, raw));
    }
    {
      floatx4 acc[NT];
      float s2;
      tile_products<PREC, NT, false>(a, raw, tab_off, tab_nv, ct, acc, s2);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float best = FLT_MAX;
        int bi = 0x7fffffff;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
          const int k = 16 * tt + col;
          const float v = cn2[k] - 2.0f * acc[tt][i];  // padded landmarks: cn2 = FLT_MAX
          const bool take = v < best;
          best = take ? v : best;
          bi = take ? k : bi;
        }
        row16_argmin(best, bi);
        if (bi >= a.r) bi = 0;  // non-finite guide values: no comparison succeeded
        if (col == 0) {
          const int pxl = 16 * w + 4 * rq + i;
          const bool valid = pxl < ti.nvalid;
          if constexpr (MDT > 0) {
            // move this pixel's one-hot entry from the previous tile's label
            const int old = labs[pxl];
            if (old >= 0) oh[old * OHS + pxl] = (T)0.0f;
            if (valid) {
              oh[bi * OHS + pxl] = (T)1.0f;
              atomicAdd(&cnt[bi], 1);
            }
          }
          labs[pxl] = valid ? bi : -1;
          if (valid && a.labels) a.labels[ti.x0 + pxl] = bi;
        }
      }
    }
    __syncthreads();
    if constexpr (MDT > 0) {
      // one-hot GEMM over the tile's pixels, 32 per K step.  The number of
      // dimension tiles this wave owns is uniform and picks a loop of fixed
      // length: no branches between the accumulators' updates, which kept
      // them moving between registers
      auto sums = [&](auto mc) {
        constexpr int M = decltype(mc)::value;
#pragma unroll
        for (int ks = 0; ks < TP / 32; ++ks) {
          const int px0 = 32 * ks + 8 * rq;  // this lane's 8 pixels (K rows)
          V bp[M][NPART];
#pragma unroll
          for (int m = 0; m < M; ++m) {
            // v = raw value (dimension column) or 0 (padding); the padding
            // lanes read dimension 0 (in bounds), so no branch around the load
            const bool dim = doff[m] >= 0;
            const float *src = raw + px0 * a.pxstride + (dim ? doff[m] : 0);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const float lv = src[j * a.pxstride];
              const float v = dim ? lv : 0.0f;
              T pp[NPART];
              Split<PREC>::parts(v, pp);
#pragma unroll
              for (int q = 0; q < NPART; ++q) bp[m][q][j] = pp[q];
            }
          }
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) {
            const V av = *reinterpret_cast<const V *>(&oh[(16 * tt + col) * OHS + px0]);
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
              for (int q = 0; q < NPART; ++q) sacc_r[m][tt] = Half<PREC>::mma(av, bp[m][q], sacc_r[m][tt]);
          }
        }
      };
      if (nown == MDT) {
        sums(std::integral_constant<int, MDT>{});
      } else if constexpr (MDT == 2) {
        if (nown == 1) sums(std::integral_constant<int, 1>{});
      }
    } else {
      // per-cluster sums of the centred guide vectors with atomics: wave w
      // walks its own 16 pixels, lanes over the dimensions d = lane + 64 m
      const int npx = ti.nvalid - 16 * w < 16 ? ti.nvalid - 16 * w : 16;
      for (int pi = 0; pi < npx; ++pi) {
        const int pxl = 16 * w + pi;
        const int L = labs[pxl];
        const float *src = raw + pxl * a.pxstride;
        float v[kMaxDc];
#pragma unroll
        for (int m = 0; m < kMaxDc; ++m) v[m] = src[doff[m] >= 0 ? doff[m] : 0];
        if (a.lds_acc) {
          float *dst = sacc + L * DA + lane;
#pragma unroll
          for (int m = 0; m < kMaxDc; ++m)
            if (doff[m] >= 0) atomicAdd(&dst[64 * m], v[m]);
          if (lane == 0) atomicAdd(&sacc[L * DA + D], 1.0f);
        } else {
          double *dst = slot + (size_t)L * DA + lane;
#pragma unroll
          for (int m = 0; m < kMaxDc; ++m)
            if (doff[m] >= 0) atomicAdd(&dst[64 * m], (double)v[m]);
          if (lane == 0) atomicAdd(&slot[(size_t)L * DA + D], 1.0);
        }
      }
    }
  }
  if constexpr (MDT > 0) {
    // lane holds S[k = 16 tt + 4 rq + i][d = 16 (w + NW m) + col]
#pragma unroll
    for (int m = 0; m < MDT; ++m) {
      const int d = 16 * (w + NW * m) + col;
      if (d >= D) continue;
#pragma unroll
      for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = 16 * tt + 4 * rq + i;
          if (k < a.r) slot[(size_t)k * DA + d] = (double)sacc_r[m][tt][i];
        }
    }
    // the counts are complete: the last tile's increments precede the barrier
    // ahead of its sums
    for (int k = tid; k < a.r; k += BT) slot[(size_t)k * DA + D] = (double)cnt[k];
  } else if (a.lds_acc) {
    __syncthreads();
    for (int e = tid; e < a.r * DA; e += BT) slot[e] = (double)sacc[e];
  }
}

// ---- FP32 assignment on the matrix cores (the FP32 form, D > 32) -----------
// Labels of the FP32 form for wide guides with the tiles, staging, permuted
// axis and argmin of the 16-bit k-means, the products p~.c~ on
// v_mfma_f32_16x16x4f32 (FP32 operands and sums; 16 pixels x 16 landmarks x 4
// dimensions per instruction) and the landmarks as FP32 [RP][DS] in LDS.  The
// distances take the GEMM form |c~|^2 - 2 p~.c~ about an offset near the data,
// landmark 0 of the current centroids (the distances do not depend on it), where
// the VALU kernel sums (p - c)^2 directly; the labels differ from it only inside
// the FP32 tie band.  Labels only: the FP32 form keeps its deterministic
// owned-dimension cluster sums.
__global__ __launch_bounds__(64) void prep_landmarks32_kernel(MArgs a, float *ctg, float *cn2g) {
  const int k = blockIdx.x, lane = threadIdx.x, D = a.g.D;
  float s = 0.0f;
  for (int dd = lane; dd < a.DS; dd += 64) {
    const int q = dd / a.RLP, el = dd - q * a.RLP;
    float v = 0.0f;
    if (k < a.r && q < a.NR && el < a.RL) {
      const int d = q * a.RL + el;
      v = a.c[k * D + d] - mu_of(a, d);
    }
    s = fmaf(v, v, s);
    ctg[k * a.DS + dd] = v;
  }
  s = wave_sum(s);
  if (lane == 0) cn2g[k] = k < a.r ? s : FLT_MAX;
}

// acc[t][i] = p~(pixel 16w + 4 rq + i) . c~(landmark 16t + col), FP32: lane
// (row, kq) gives operand A = p~(pixel 16w + row, dimension 4s + kq) and B =
// c~(landmark 16t + row, dimension 4s + kq) on the permuted axis.
template <int NT>
__device__ __forceinline__ void tile_products32(const MArgs &a, const float *raw, const int *tab_off,
                                                const int *tab_nv, const float *ct, floatx4 (&acc)[NT]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4;
  const int pofs = (16 * w + row) * a.pxstride;
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nsteps = a.NR * a.RLP / 4;
  for (int s = 0; s < nsteps; ++s) {
    const int e = 4 * s + kq, q8 = e >> 3, o = e & 7;
    const float lv = raw[tab_off[q8] + pofs + o];  // in bounds; past the chunk's valid count it is zeroed
    const float av = o < tab_nv[q8] ? lv : 0.0f;
    float bv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bv[t] = ct[(16 * t + row) * a.DS + e];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[t], acc[t], 0, 0, 0);
  }
}

size_t assign32_lds(const MArgs &a) {
  return sizeof(float) * ((size_t)a.RP * a.DS + a.raw_floats + 8 + a.RP) + sizeof(int) * 2 * kMaxChunks;
}

template <int NT, int BT, int PF>
__global__ __launch_bounds__(BT) void assign_f32_kernel(MArgs a) {
  constexpr int NW = BT / 64, TP = 16 * NW;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  float *ct = reinterpret_cast<float *>(smem_raw);                  // [RP][DS]
  float *raw = ct + (size_t)a.RP * a.DS;                           // [raw_floats + 8]
  float *cn2 = raw + a.raw_floats + 8;                             // [RP]
  int *tab_off = reinterpret_cast<int *>(cn2 + a.RP);              // [kMaxChunks]
  int *tab_nv = tab_off + kMaxChunks;                              // [kMaxChunks]
  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = lane & 15, rq = lane >> 4;
  {
    const int n4 = a.RP * a.DS / 4;  // DS is a multiple of 8
    const float4 *src = reinterpret_cast<const float4 *>(a.ctg);
    float4 *dst = reinterpret_cast<float4 *>(ct);
    for (int e = tid; e < n4; e += BT) dst[e] = src[e];
    for (int k = tid; k < a.RP; k += BT) cn2[k] = a.cn2g[k];
  }
  build_tables(a, tab_off, tab_nv, nullptr, BT);
  load_mu(a, raw_mu(a, raw), BT);
  TilePrefetch<TP, BT> pre;
  PatchPrefetch<TP, BT> ppre;
  __syncthreads();  // the offsets in LDS before the first prefetch
  if ((int)blockIdx.x < a.ntiles) {
    if constexpr (PF == 1) pre.load(a, tile_info<TP>(a, blockIdx.x));
    if constexpr (PF == 2) ppre.load(a, tile_info<TP>(a, blockIdx.x), raw_mu(a, raw));
  }
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const TileInfo ti = tile_info<TP>(a, t);
    __syncthreads();
    if constexpr (PF == 1)
      pre.store(a, ti, raw, raw_mu(a, raw));
    else if constexpr (PF == 2)
      ppre.store(a, raw);
    else
      stage_raw<TP, BT>(a, ti, raw, raw_mu(a, raw));
    __syncthreads();
    if (t + (int)gridDim.x < a.ntiles) {
      if constexpr (PF == 1) pre.load(a, tile_info<TP>(a, t + gridDim.x));
      if constexpr (PF == 2) ppre.load(a, tile_info<TP>(a, t + gridDim.x), raw_mu(a, raw));
    }
    floatx4 acc[NT];
    tile_products32<NT>(a, raw, tab_off, tab_nv, ct, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float best = FLT_MAX;
      int bi = 0x7fffffff;
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        const int k = 16 * tt + col;
        const float v = cn2[k] - 2.0f * acc[tt][i];  // padded landmarks: cn2 = FLT_MAX
        const bool take = v < best;
        best = take ? v : best;
        bi = take ? k : bi;
      }
      row16_argmin(best, bi);
      if (bi >= a.r) bi = 0;  // non-finite guide values: no comparison succeeded
      const int pxl = 16 * w + 4 * rq + i;
      if (col == 0 && pxl < ti.nvalid) a.labels[ti.x0 + pxl] = bi;
    }
  }
}

template <int NT>
hipError_t launch_assign32_nt(const MArgs &a, size_t lds, hipStream_t s) {
  constexpr int BT = 512, TP = 16 * BT / 64;
  const int nb = a.ntiles < 1024 ? (a.ntiles < 1 ? 1 : a.ntiles) : 1024;
  auto go = [&](auto kern) {
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(BT), lds, s, a);
    return hipGetLastError();
  };
  if (TilePrefetch<TP, BT>::usable(a)) return go(assign_f32_kernel<NT, BT, 1>);
  if (PatchPrefetch<TP, BT>::usable(a)) return go(assign_f32_kernel<NT, BT, 2>);
  return go(assign_f32_kernel<NT, BT, 0>);
}

// ---- embedding --------------------------------------------------------------
// MAXT2: output tiles (16 planes of u) per wave.  The wave's rows of F^T stay
// in registers when they fit (FREG), else they are read from memory.
// EM: 0 = the whole embedding; 1 = the cross-kernel tiles only, written to
// bbuf (they need the landmarks but not F, so they can run while the host
// decomposes A); 2 = the mix only, from the tiles in bbuf.
template <int PREC, int NT, int BT, int MAXT2, int EM = 0>
__global__ __launch_bounds__(BT) void embed_mfma_kernel(MArgs a) {
  using T = typename Half<PREC>::T;
  constexpr int NW = BT / 64, TP = 16 * NW;
  constexpr int KS = NT * 4;                     // K steps of the mix (RP / 4)
  constexpr bool FREG = KS * MAXT2 <= 64 && NT <= 8;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T *ct = reinterpret_cast<T *>(smem_raw);                                    // [RP][DS]
  T *ct_lo = ct + (size_t)a.RP * a.DS;                                        // [RP][DS]
  float *raw = reinterpret_cast<float *>(ct_lo + (size_t)a.RP * a.DS);        // [raw_floats + 8]
  // [TP][RP + 4]; the mix-only form keeps nothing else in LDS
  float *bs = EM == 2 ? reinterpret_cast<float *>(smem_raw) : raw + a.raw_floats + 8;
  float *cn2 = bs + TP * (a.RP + 4);                                          // [RP]
  int *tab_off = reinterpret_cast<int *>(cn2 + a.RP);                         // [kMaxChunks]
  int *tab_nv = tab_off + kMaxChunks;                                         // [kMaxChunks]
  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = lane & 15, rq = lane >> 4;
  // b-tile row stride == 4 (mod 16): the exp stores (rows 4 rq + i, columns
  // col) and the mix reads (rows col, columns 4 s + rq) hit distinct banks
  const int BS = a.RP + 4;
  // output tiles w + NW m (m < MAXT2) of this wave with 16 (w + NW m) < RE
  const int nmix = max(0, min(MAXT2, (a.RE / 16 - w + NW - 1) / NW));

  if constexpr (EM != 2) {
    load_landmarks(a, ct, cn2, BT, ct_lo);
    build_tables(a, tab_off, tab_nv, nullptr, BT);
    load_mu(a, raw_mu(a, raw), BT);
  }
  // mix operand A = F^T: A[k'][j] = F[j][k']; lane (col, rq) takes
  // A[16 t2 + col][4 s + rq] for the wave's tiles t2 = w + NW m
  auto fval = [&](int m, int s) {
    const int kk = 16 * (w + NW * m) + col, j = 4 * s + rq;
    return (kk < a.r_eff && j < a.r) ? a.F32[j * a.r_eff + kk] : 0.0f;
  };
  float fa[FREG ? MAXT2 : 1][FREG ? KS : 1];
  if constexpr (FREG && EM != 1) {
#pragma unroll
    for (int m = 0; m < MAXT2; ++m)
#pragma unroll
      for (int s = 0; s < KS; ++s) fa[m][s] = fval(m, s);
  }
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const TileInfo ti = tile_info<TP>(a, t);
    float4 *tile_b = reinterpret_cast<float4 *>(a.bbuf + (size_t)t * TP * a.RP);
    __syncthreads();
    if constexpr (EM == 2) {
      for (int e = tid; e < TP * a.RP / 4; e += BT) {
        const int px = 4 * e / a.RP, k = 4 * e - px * a.RP;
        *reinterpret_cast<float4 *>(&bs[px * BS + k]) = tile_b[e];
      }
      __syncthreads();
    } else {
      stage_raw<TP, BT>(a, ti, raw, raw_mu(a, raw));
      __syncthreads();
      floatx4 acc[NT];
      float s2;
      tile_products<PREC, NT, true, true>(a, raw, tab_off, tab_nv, ct, acc, s2, ct_lo);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pxl = 16 * w + 4 * rq + i;
        const float n2 = __shfl(s2, 4 * rq + i, 64);  // lane 4 rq + i holds pixel 16w + 4 rq + i
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
          const int k = 16 * tt + col;
          const float d2 = fmaxf(n2 + cn2[k] - 2.0f * acc[tt][i], 0.0f);
          bs[pxl * BS + k] = k < a.r ? exp2f(-d2 * a.inv2s2 * 1.4426950408889634f) : 0.0f;
        }
      }
      __syncthreads();
      if constexpr (EM == 1) {
        // (bs is only 4-byte aligned here: scalar LDS reads)
        for (int e = tid; e < TP * a.RP / 4; e += BT) {
          const int px = 4 * e / a.RP, k = 4 * e - px * a.RP;
          const float *src = &bs[px * BS + k];
          tile_b[e] = make_float4(src[0], src[1], src[2], src[3]);
        }
        continue;
      }
    }
    // U[k'][px] = sum_j F[j][k'] b[px][j]: A = F^T, B = b^T (LDS).  The
    // wave's tile count is uniform and picks a loop of fixed length, so that
    // fa is only ever indexed by constants (a break out of the unrolled loop
    // left it indexed at run time, in scratch memory)
    auto mix = [&](auto mc) {
      constexpr int M = decltype(mc)::value;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const int t2 = w + NW * m;
#pragma unroll 1
        for (int gp = 0; gp < TP / 16; ++gp) {
          floatx4 o = {0.f, 0.f, 0.f, 0.f};
          const float *bcol = bs + (16 * gp + col) * BS + rq;
#pragma unroll
          for (int s = 0; s < KS; ++s) {
            float av;
            if constexpr (FREG)
              av = fa[m][s];
            else
              av = fval(m, s);
            o = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bcol[4 * s], o, 0, 0, 0);
          }
          // lane holds U[k' = 16 t2 + 4 rq + i][pixel 16 gp + col]
          const int pxl = 16 * gp + col;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int kp = 16 * t2 + 4 * rq + i;
            if (kp < a.r_eff && pxl < ti.nvalid) a.u[(int64_t)kp * a.N + ti.x0 + pxl] = o[i];
          }
        }
      }
    };
    if (nmix == MAXT2) {
      mix(std::integral_constant<int, MAXT2>{});
    } else if constexpr (MAXT2 > 1) {
      if (nmix == 1) {
        mix(std::integral_constant<int, 1>{});
      } else if constexpr (MAXT2 > 2) {
        if (nmix == 2)
          mix(std::integral_constant<int, 2>{});
        else if (nmix == 3)
          mix(std::integral_constant<int, 3>{});
      }
    }
  }
}

// ---- centring offsets -------------------------------------------------------
// mu[m] = mean over the pixels of guide column m (m < D; for patch guides
// m < C: a patch dimension takes its channel's mean).  Per-block FP64 partial
// sums over a contiguous pixel range (eight independent accumulators per
// thread keep eight loads in flight), then one block per dimension sums the
// partials in a fixed order, so the result is deterministic.
__global__ __launch_bounds__(256) void mean_partial_kernel(Guide g, int64_t N, int M, double *part) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int lanes = 256 / M;
  const int m = tid % M, ln = tid / M;
  const float *src = g.kind == GUIDE_EXPLICIT ? g.p : g.f;
  const int stride = g.kind == GUIDE_EXPLICIT ? g.D : g.C;
  const int64_t per = (N + gridDim.x - 1) / gridDim.x;
  const int64_t x0 = per * blockIdx.x, x1 = x0 + per < N ? x0 + per : N;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (ln < lanes) {
    int64_t x = x0 + ln;
    for (; x + 7 * lanes < x1; x += 8 * lanes) {
      float v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = src[(x + q * lanes) * stride + m];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += v[q];
    }
    for (; x < x1; x += lanes) acc[0] += src[x * stride + m];
  }
  red[tid] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (tid < M) {
    double t = 0.0;
    for (int q = 0; q < lanes; ++q) t += red[q * M + tid];
    part[(size_t)blockIdx.x * M + tid] = t;
  }
}

// grid: M blocks of 256 threads
__global__ __launch_bounds__(256) void mean_final_kernel(const double *part, int nb, int M, int64_t N, float *mu) {
  __shared__ double red[256];
  const int m = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int b = tid; b < nb; b += 256) s += part[(size_t)b * M + m];
  red[tid] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) mu[m] = (float)(red[0] / (double)N);
}

__global__ void f64_to_f32_kernel(const double *src, float *dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

MArgs make_args(const Guide &g, const float *c, int r, const float *mu, int TP) {
  MArgs a{};
  a.g = g;
  a.N = (int64_t)g.H * g.W;
  a.c = c;
  a.mu = mu;
  a.r = r;
  // landmark rows padded to the kernels' tile count NT = RP / 16 (4, 8 or 16)
  a.RP = r <= 64 ? 64 : (r <= 128 ? 128 : 256);
  if (g.kind == GUIDE_PATCH) {
    const int PW = 2 * g.pr + 1;
    a.NR = PW;
    a.RL = PW * g.C;
    a.pxstride = g.C;
    a.rowstride = (TP + 2 * g.pr) * g.C;
    a.muf = (g.C + 3) / 4 * 4;
    a.raw_floats = PW * a.rowstride + a.muf;
    a.tiles_x = (g.W + TP - 1) / TP;
    a.ntiles = (int)((int64_t)g.H * a.tiles_x);
  } else {
    a.NR = 1;
    a.RL = g.D;
    // row stride == 4 (mod 64) floats: the 16 rows read by one b128 phase
    // fall on distinct groups of four banks
    a.pxstride = (g.D + 63) / 64 * 64 + 4;
    a.rowstride = 0;
    a.muf = (g.D + 3) / 4 * 4;
    a.raw_floats = TP * a.pxstride + a.muf;
    a.tiles_x = 0;
    a.ntiles = (int)((a.N + TP - 1) / TP);
  }
  a.RLP = (a.RL + 7) / 8 * 8;
  a.Dp = (a.NR * a.RLP + 31) / 32 * 32;
  a.DS = a.Dp + 8;
  return a;
}

template <int PREC>
size_t ct_bytes(const MArgs &a) {
  return sizeof(typename Half<PREC>::T) * (size_t)a.RP * a.DS;
}

size_t lloyd_lds(const MArgs &a, int TP, size_t ctb, bool lds_acc, bool gemm_acc) {
  size_t b = ctb + sizeof(float) * ((size_t)a.raw_floats + 8 + a.RP) +
             sizeof(int) * (2 * kMaxChunks + TP + a.g.D + a.RP);
  if (lds_acc) b += sizeof(float) * (size_t)a.r * (a.g.D + 1);
  if (gemm_acc) b = ((b + 15) & ~(size_t)15) + (ctb / a.DS) * (TP + 8);  // one-hot [RP][TP + 8]
  return b;
}

size_t embed_lds(const MArgs &a, int TP, size_t ctb) {
  return ctb + sizeof(float) * ((size_t)a.raw_floats + 8 + (size_t)TP * (a.RP + 4) + a.RP) +
         sizeof(int) * 2 * kMaxChunks;
}

template <class K>
hipError_t set_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

// Block shape and accumulation of the k-means kernel, in order of preference:
// 8 waves with the sums on the matrix cores (mdt <= 2 dimension tiles per wave,
// NT * mdt <= 16 accumulator tiles), then LDS atomics with 8 or 4 waves, then
// FP64 atomics in global memory.
struct LloydPlan {
  int BT, mdt;
  bool lds_acc;
  size_t lds;
  bool ok;
};

template <int PREC>
LloydPlan plan_lloyd(const Guide &g, int r) {
  {
    const MArgs a = make_args(g, nullptr, r, nullptr, 128);
    if (a.Dp / 8 > kMaxChunks) return {0, 0, false, 0, false};
    const int ndt = (g.D + 15) / 16;
    const int mdt = (ndt + 7) / 8;
    const int NT = a.RP / 16;
    const size_t l = lloyd_lds(a, 128, ct_bytes<PREC>(a), false, true);
    if (mdt <= 2 && NT * mdt <= 16 && l <= kLdsMax) return {512, mdt, false, l, true};
  }
  for (int acc = 1; acc >= 0; --acc)
    for (int BT : {512, 256}) {
      const MArgs a = make_args(g, nullptr, r, nullptr, 16 * BT / 64);
      const size_t l = lloyd_lds(a, 16 * BT / 64, ct_bytes<PREC>(a), acc == 1, false);
      if (l <= kLdsMax) return {BT, 0, acc == 1, l, true};
    }
  return {0, 0, false, 0, false};
}

template <int PREC>
int plan_embed(const Guide &g, int r, size_t *lds) {
  for (int BT : {512, 256}) {
    const MArgs a = make_args(g, nullptr, r, nullptr, 16 * BT / 64);
    if (a.Dp / 8 > kMaxChunks) return 0;
    const size_t l = embed_lds(a, 16 * BT / 64, 2 * ct_bytes<PREC>(a));
    if (l <= kLdsMax) {
      *lds = l;
      return BT;
    }
  }
  return 0;
}

template <int PREC, int NT, int BT, int MDT, int PF>
hipError_t launch_lloyd_kp(const MArgs &a, size_t lds, hipStream_t s, int *nblocks) {
  hipError_t e = set_lds(lloyd_mfma_kernel<PREC, NT, BT, MDT, PF>, lds);
  if (e != hipSuccess) return e;
  int nb = a.ntiles < kMaxBlocks ? a.ntiles : kMaxBlocks;
  if (nb < 1) nb = 1;
  *nblocks = nb;
  hipLaunchKernelGGL((lloyd_mfma_kernel<PREC, NT, BT, MDT, PF>), dim3(nb), dim3(BT), lds, s, a);
  return hipGetLastError();
}

// The tile prefetch (registers) only for the 8-wave GEMM-sum kernels of wide
// explicit / self guides; patch guides stage their tiles directly.
template <int PREC, int NT, int BT, int MDT>
hipError_t launch_lloyd_k(const MArgs &a, size_t lds, hipStream_t s, int *nblocks) {
  constexpr int TP = 16 * BT / 64;
  if constexpr (BT == 512 && (MDT == 1 ? NT <= 8 : MDT == 2 && NT <= 4))  // these fit 256 VGPRs
    if (TilePrefetch<TP, BT>::usable(a)) return launch_lloyd_kp<PREC, NT, BT, MDT, 1>(a, lds, s, nblocks);
  if constexpr (BT == 512 && MDT > 0 && NT <= 8)
    if (PatchPrefetch<TP, BT>::usable(a)) return launch_lloyd_kp<PREC, NT, BT, MDT, 2>(a, lds, s, nblocks);
  return launch_lloyd_kp<PREC, NT, BT, MDT, 0>(a, lds, s, nblocks);
}

template <int PREC, int NT>
hipError_t launch_lloyd_nt(const MArgs &a, const LloydPlan &pl, hipStream_t s, int *nblocks) {
  if (pl.mdt == 0)
    return pl.BT == 512 ? launch_lloyd_k<PREC, NT, 512, 0>(a, pl.lds, s, nblocks)
                        : launch_lloyd_k<PREC, NT, 256, 0>(a, pl.lds, s, nblocks);
  if (pl.mdt == 1) return launch_lloyd_k<PREC, NT, 512, 1>(a, pl.lds, s, nblocks);
  if constexpr (NT <= 8)
    if (pl.mdt == 2) return launch_lloyd_k<PREC, NT, 512, 2>(a, pl.lds, s, nblocks);
  return hipErrorInvalidValue;
}

// The prepared landmarks live in the caller's scratch: [RP][DS] 16-bit values,
// [RP][DS] 16-bit remainders, then [RP] floats.
template <int PREC>
hipError_t prep_landmarks(MArgs &a, void *scratch, hipStream_t s) {
  using T = typename Half<PREC>::T;
  T *ctg = reinterpret_cast<T *>(scratch);
  T *ctg_lo = ctg + (size_t)a.RP * a.DS;
  float *cn2g = reinterpret_cast<float *>(ctg_lo + (size_t)a.RP * a.DS);
  a.ctg = ctg;
  a.ctg_lo = ctg_lo;
  a.cn2g = cn2g;
  hipLaunchKernelGGL(prep_landmarks_kernel<PREC>, dim3(a.RP), dim3(64), 0, s, a, ctg, ctg_lo, cn2g);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_lloyd_p(const Guide &g, const float *c, int r, const float *mu, double *partials, int *labels,
                          void *lm, hipStream_t s, int *nblocks) {
  const LloydPlan pl = plan_lloyd<PREC>(g, r);
  if (!pl.ok) return hipErrorInvalidValue;
  MArgs a = make_args(g, c, r, mu, 16 * pl.BT / 64);
  a.partials = partials;
  a.labels = labels;
  a.lds_acc = pl.lds_acc ? 1 : 0;
  hipError_t e = prep_landmarks<PREC>(a, lm, s);
  if (e != hipSuccess) return e;
  if (a.RP == 64) return launch_lloyd_nt<PREC, 4>(a, pl, s, nblocks);
  if (a.RP == 128) return launch_lloyd_nt<PREC, 8>(a, pl, s, nblocks);
  return launch_lloyd_nt<PREC, 16>(a, pl, s, nblocks);
}

template <int PREC, int NT, int BT, int EM>
hipError_t launch_embed_nt(const MArgs &a, size_t lds, hipStream_t s) {
  constexpr int NW = BT / 64;
  const int per_wave = (a.RE / 16 + NW - 1) / NW;
  hipError_t e;
  int nb = a.ntiles < kEmbedBlocks ? a.ntiles : kEmbedBlocks;
  if (nb < 1) nb = 1;
  if constexpr (EM == 1) {
    if ((e = set_lds(embed_mfma_kernel<PREC, NT, BT, 1, 1>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((embed_mfma_kernel<PREC, NT, BT, 1, 1>), dim3(nb), dim3(BT), lds, s, a);
    return hipGetLastError();
  }
#define NKF_EMBED_CASE(M)                                                                         \
  if (per_wave <= M) {                                                                            \
    if ((e = set_lds(embed_mfma_kernel<PREC, NT, BT, M, EM>, lds)) != hipSuccess) return e;       \
    hipLaunchKernelGGL((embed_mfma_kernel<PREC, NT, BT, M, EM>), dim3(nb), dim3(BT), lds, s, a); \
    return hipGetLastError();                                                                     \
  }
  NKF_EMBED_CASE(1)
  NKF_EMBED_CASE(2)
  NKF_EMBED_CASE(4)
#undef NKF_EMBED_CASE
  return hipErrorInvalidValue;
}

template <int PREC, int BT, int EM = 0>
hipError_t launch_embed_bt(const MArgs &a, size_t lds, hipStream_t s) {
  if (a.RP == 64) return launch_embed_nt<PREC, 4, BT, EM>(a, lds, s);
  if (a.RP == 128) return launch_embed_nt<PREC, 8, BT, EM>(a, lds, s);
  return launch_embed_nt<PREC, 16, BT, EM>(a, lds, s);
}

}  // namespace

bool mfma_path_supported(const Guide &g, int r, int prec) {
  size_t lds = 0;
  if (prec == 1) return plan_lloyd<1>(g, r).ok && plan_embed<1>(g, r, &lds) != 0;
  return plan_lloyd<2>(g, r).ok && plan_embed<2>(g, r, &lds) != 0;
}

bool assign_mfma32_supported(const Guide &g, int r) {
  // narrow guides stay on the VALU kernel (PCA guide, D = 25: 104 -> 138 us per
  // iteration on the matrix cores), as in the 16-bit forms
  if (g.D <= 32 || r < 1 || r > 256) return false;
  const MArgs a = make_args(g, nullptr, r, nullptr, 128);
  return a.Dp / 8 <= kMaxChunks && assign32_lds(a) <= kLdsMax;
}

size_t assign_mfma32_scratch_floats(const Guide &g, int r) {
  const MArgs a = make_args(g, nullptr, r, nullptr, 128);
  return (size_t)a.RP * a.DS + a.RP;
}

hipError_t launch_assign_mfma32(const Guide &g, const float *c, int r, int *labels, float *scratch,
                                hipStream_t s) {
  if (!assign_mfma32_supported(g, r)) return hipErrorInvalidValue;
  MArgs a = make_args(g, c, r, c, 128);  // centring offset: landmark 0
  a.labels = labels;
  float *ctg = scratch, *cn2g = scratch + (size_t)a.RP * a.DS;
  a.ctg = ctg;
  a.cn2g = cn2g;
  hipLaunchKernelGGL(prep_landmarks32_kernel, dim3(a.RP), dim3(64), 0, s, a, ctg, cn2g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = assign32_lds(a);
  if (a.RP == 64) return launch_assign32_nt<4>(a, lds, s);
  if (a.RP == 128) return launch_assign32_nt<8>(a, lds, s);
  return launch_assign32_nt<16>(a, lds, s);
}

size_t mfma_landmark_scratch_bytes(const Guide &g, int r) {
  const MArgs a = make_args(g, nullptr, r, nullptr, 16);
  return 2 * 2 * (size_t)a.RP * a.DS + sizeof(float) * a.RP;
}

size_t guide_mean_scratch_doubles(const Guide &g) {
  return (size_t)kMeanBlocks * (g.kind == GUIDE_PATCH ? g.C : g.D);
}

hipError_t launch_guide_mean(const Guide &g, float *mu, double *scratch, hipStream_t s) {
  const int M = g.kind == GUIDE_PATCH ? g.C : g.D;
  const int64_t N = (int64_t)g.H * g.W;
  hipLaunchKernelGGL(mean_partial_kernel, dim3(kMeanBlocks), dim3(256), 0, s, g, N, M, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mean_final_kernel, dim3(M), dim3(256), 0, s, scratch, kMeanBlocks, M, N, mu);
  return hipGetLastError();
}

hipError_t launch_lloyd_mfma(const Guide &g, const float *c, int r, const float *mu, int prec, double *partials,
                             int *labels, int *nparts, void *lm_scratch, hipStream_t s) {
  return prec == 1 ? launch_lloyd_p<1>(g, c, r, mu, partials, labels, lm_scratch, s, nparts)
                   : launch_lloyd_p<2>(g, c, r, mu, partials, labels, lm_scratch, s, nparts);
}

hipError_t launch_embed_mfma(const Guide &g, const float *c, int r, const float *mu, const double *F, float *F32,
                             int r_eff, double sigma_r, int prec, float *u, void *lm_scratch, hipStream_t s) {
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3((r * r_eff + 255) / 256), dim3(256), 0, s, F, F32, r * r_eff);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t lds = 0;
  const int BT = prec == 1 ? plan_embed<1>(g, r, &lds) : plan_embed<2>(g, r, &lds);
  if (BT == 0) return hipErrorInvalidValue;
  MArgs a = make_args(g, c, r, mu, 16 * BT / 64);
  a.F32 = F32;
  a.r_eff = r_eff;
  a.RE = (r_eff + 15) / 16 * 16;
  a.inv2s2 = isinf(sigma_r) ? 0.0f : (float)(1.0 / (2.0 * sigma_r * sigma_r));
  a.u = u;
  e = prec == 1 ? prep_landmarks<1>(a, lm_scratch, s) : prep_landmarks<2>(a, lm_scratch, s);
  if (e != hipSuccess) return e;
  if (prec == 1) return BT == 512 ? launch_embed_bt<1, 512>(a, lds, s) : launch_embed_bt<1, 256>(a, lds, s);
  return BT == 512 ? launch_embed_bt<2, 512>(a, lds, s) : launch_embed_bt<2, 256>(a, lds, s);
}

size_t embed_split_floats(const Guide &g, int r, int prec) {
  size_t lds = 0;
  const int BT = prec == 1 ? plan_embed<1>(g, r, &lds) : plan_embed<2>(g, r, &lds);
  if (BT == 0) return 0;
  const MArgs a = make_args(g, nullptr, r, nullptr, 16 * BT / 64);
  return (size_t)a.ntiles * (16 * BT / 64) * a.RP;
}

hipError_t launch_embed_mfma_b(const Guide &g, const float *c, int r, const float *mu, double sigma_r, int prec,
                               float *bbuf, void *lm_scratch, hipStream_t s) {
  size_t lds = 0;
  const int BT = prec == 1 ? plan_embed<1>(g, r, &lds) : plan_embed<2>(g, r, &lds);
  if (BT == 0) return hipErrorInvalidValue;
  MArgs a = make_args(g, c, r, mu, 16 * BT / 64);
  a.r_eff = 1;
  a.RE = 16;
  a.inv2s2 = isinf(sigma_r) ? 0.0f : (float)(1.0 / (2.0 * sigma_r * sigma_r));
  a.bbuf = bbuf;
  hipError_t e = prec == 1 ? prep_landmarks<1>(a, lm_scratch, s) : prep_landmarks<2>(a, lm_scratch, s);
  if (e != hipSuccess) return e;
  if (prec == 1) return BT == 512 ? launch_embed_bt<1, 512, 1>(a, lds, s) : launch_embed_bt<1, 256, 1>(a, lds, s);
  return BT == 512 ? launch_embed_bt<2, 512, 1>(a, lds, s) : launch_embed_bt<2, 256, 1>(a, lds, s);
}

hipError_t launch_embed_mfma_mix(const Guide &g, int r, const double *F, float *F32, int r_eff, int prec, float *u,
                                 const float *bbuf, hipStream_t s) {
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3((r * r_eff + 255) / 256), dim3(256), 0, s, F, F32, r * r_eff);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t lds_full = 0;
  const int BT = prec == 1 ? plan_embed<1>(g, r, &lds_full) : plan_embed<2>(g, r, &lds_full);
  if (BT == 0) return hipErrorInvalidValue;
  MArgs a = make_args(g, nullptr, r, nullptr, 16 * BT / 64);
  a.F32 = F32;
  a.r_eff = r_eff;
  a.RE = (r_eff + 15) / 16 * 16;
  a.u = u;
  a.bbuf = const_cast<float *>(bbuf);
  const size_t lds = sizeof(float) * (size_t)(16 * BT / 64) * (a.RP + 4);  // the b tile only
  if (prec == 1) return BT == 512 ? launch_embed_bt<1, 512, 2>(a, lds, s) : launch_embed_bt<1, 256, 2>(a, lds, s);
  return BT == 512 ? launch_embed_bt<2, 512, 2>(a, lds, s) : launch_embed_bt<2, 256, 2>(a, lds, s);
}

}  // namespace nkf
