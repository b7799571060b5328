// Distance step on the matrix cores for high-dimensional guides (hyperspectral
// bands, nonlocal-means patches): the cross kernel B(i, x) = k(c_i, p(x)) of
// Eq. (defB) and the k-means assignment (Section III) in GEMM form,
//     |p - c|^2 = |p~|^2 + |c~|^2 - 2 p~.c~,   p~ = p - mu, c~ = c - mu,
// with the centred guide and landmarks rounded to BF16 or FP16 for the MFMA
// product (FP32 accumulation), the squared norms taken in FP32 from the
// unrounded centred values, and the result clamped at zero.  mu is the mean
// guide value, which makes |p~| and |c~| small next to |p| and |c| and keeps
// the cancellation in the GEMM form within the 16-bit rounding.
//
// A block keeps the centred landmarks [r][D] in LDS and walks 64-pixel tiles;
// wave w computes the 16 x r tile of products for pixels 16w..16w+15 with
// v_mfma_f32_16x16x32_{bf16,f16}.  Assignment then takes the argmin of
// |c~|^2 - 2 p~.c~ (lowest index on ties); the embedding takes
// b = exp(-d^2 / (2 sigma_r^2)) and mixes it with the factor F (FP32 copy) on
// v_mfma_f32_16x16x4_f32, producing u^T tiles so that the planar stores of u
// are coalesced.
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>

#include "device_common.h"

namespace nkf {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int kBlock = 256;
constexpr int kTP = 64;  // pixels per tile (16 per wave)

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
  const float *c;    // [r][D] landmarks
  const float *mu;   // [D] centring offset
  int r, RP, Dp, DS; // RP = r rounded up to 16, Dp = D rounded up to 32, DS = Dp + 8 (LDS row stride)
  const float *F32;  // [r][r_eff] factor (embedding)
  int r_eff, RE;     // RE = r_eff rounded up to 16
  float inv2s2;
  float *u;          // [r_eff][N] (embedding)
  int *labels;       // [N] (assignment)
};

// Centred 16-bit guide rows of one 64-pixel tile into pt[64][DS], their FP32
// squared norms into np2[64].  Thread (px = tid & 63, q = tid >> 6) fills
// elements d = 8m + e for m = q, q + 4, ...
template <int PREC>
__device__ __forceinline__ void stage_pixels(const MArgs &a, int64_t base, typename Half<PREC>::T *pt, float *np2,
                                             float *red) {
  using T = typename Half<PREC>::T;
  const int tid = threadIdx.x, px = tid & (kTP - 1), q = tid >> 6;
  const int64_t x = base + px;
  const bool valid = x < a.N;
  const Guide &g = a.g;
  const int D = g.D;
  float s2 = 0.0f;
  if (g.kind == GUIDE_PATCH) {
    // element d = (dy T + dx) C + c of the patch around (y, xx), walked with
    // incremental (dy, dx, c) counters from the start of each 8-element chunk
    const int PW = 2 * g.pr + 1;  // patch width
    const int y = valid ? (int)(x / g.W) : 0, xx = valid ? (int)(x - (int64_t)y * g.W) : 0;
    for (int m = q; m < a.Dp / 8; m += 4) {
      int d = 8 * m;
      int c = d % g.C, qd = d / g.C;
      int dx = qd % PW, dy = qd / PW;
#pragma unroll
      for (int e = 0; e < 8; ++e, ++d) {
        float v = 0.0f;
        if (valid && d < D) {
          const int yy = sym_index(y + dy - g.pr, g.H), xs = sym_index(xx + dx - g.pr, g.W);
          v = g.f[((int64_t)yy * g.W + xs) * g.C + c] - a.mu[d];
        }
        s2 = fmaf(v, v, s2);
        pt[px * a.DS + d] = (T)v;
        if (++c == g.C) {
          c = 0;
          if (++dx == PW) {
            dx = 0;
            ++dy;
          }
        }
      }
    }
  } else {
    const float *src = g.kind == GUIDE_EXPLICIT ? g.p + x * D : g.f + x * g.C;
    for (int m = q; m < a.Dp / 8; m += 4) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int d = 8 * m + e;
        float v = 0.0f;
        if (valid && d < D) v = src[d] - a.mu[d];
        s2 = fmaf(v, v, s2);
        pt[px * a.DS + d] = (T)v;
      }
    }
  }
  red[q * kTP + px] = s2;
  __syncthreads();
  if (q == 0) np2[px] = (red[px] + red[kTP + px]) + (red[2 * kTP + px] + red[3 * kTP + px]);
}

// products acc[t] (t = cluster tile) of this wave's 16 pixels with all RP clusters
template <int PREC, int NT>
__device__ __forceinline__ void tile_products(const MArgs &a, const typename Half<PREC>::T *pt,
                                              const typename Half<PREC>::T *ct, floatx4 (&acc)[NT]) {
  using V = typename Half<PREC>::V;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int s = 0; s < a.Dp / 32; ++s) {
    const V av = *reinterpret_cast<const V *>(&pt[(16 * w + row) * a.DS + 32 * s + 8 * kq]);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (16 * t < a.RP) {
        const V bv = *reinterpret_cast<const V *>(&ct[(16 * t + row) * a.DS + 32 * s + 8 * kq]);
        acc[t] = Half<PREC>::mma(av, bv, acc[t]);
      }
    }
  }
}

template <int PREC>
__device__ __forceinline__ void stage_landmarks(const MArgs &a, typename Half<PREC>::T *ct, float *cn2) {
  using T = typename Half<PREC>::T;
  const int D = a.g.D;
  for (int e = threadIdx.x; e < a.RP * a.Dp; e += kBlock) {
    const int k = e / a.Dp, d = e - k * a.Dp;
    float v = 0.0f;
    if (k < a.r && d < D) v = a.c[k * D + d] - a.mu[d];
    ct[k * a.DS + d] = (T)v;
  }
  for (int k = threadIdx.x; k < a.RP; k += kBlock) {
    float s = 0.0f;
    if (k < a.r)
      for (int d = 0; d < D; ++d) {
        const float v = a.c[k * D + d] - a.mu[d];
        s = fmaf(v, v, s);
      }
    cn2[k] = k < a.r ? s : FLT_MAX;
  }
}

// ---- k-means assignment -----------------------------------------------------
template <int PREC, int NT>
__global__ __launch_bounds__(kBlock) void assign_mfma_kernel(MArgs a) {
  using T = typename Half<PREC>::T;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T *ct = reinterpret_cast<T *>(smem_raw);                                  // [RP][DS]
  T *pt = ct + (size_t)a.RP * a.DS;                                          // [64][DS]
  float *cn2 = reinterpret_cast<float *>(pt + (size_t)kTP * a.DS);           // [RP]
  float *np2 = cn2 + a.RP;                                                   // [64]
  float *red = np2 + kTP;                                                    // [4][64]
  stage_landmarks<PREC>(a, ct, cn2);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = lane & 15, rq = lane >> 4;
  for (int64_t base = (int64_t)blockIdx.x * kTP; base < a.N; base += (int64_t)gridDim.x * kTP) {
    __syncthreads();
    stage_pixels<PREC>(a, base, pt, np2, red);
    __syncthreads();
    floatx4 acc[NT];
    tile_products<PREC, NT>(a, pt, ct, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float best = FLT_MAX;
      int bi = 0x7fffffff;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (16 * t < a.RP) {
          const int k = 16 * t + col;
          const float v = cn2[k] - 2.0f * acc[t][i];
          if (k < a.r && v < best) {
            best = v;
            bi = k;
          }
        }
      }
      // argmin across the 16 lanes holding the same 4 pixels (lowest index on ties)
#pragma unroll
      for (int m = 1; m < 16; m <<= 1) {
        const float ob = __shfl_xor(best, m, 64);
        const int oi = __shfl_xor(bi, m, 64);
        if (ob < best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      const int64_t x = base + 16 * w + 4 * rq + i;
      if (col == 0 && x < a.N) a.labels[x] = bi;
    }
  }
}

// ---- embedding --------------------------------------------------------------
template <int PREC, int NT>
__global__ __launch_bounds__(kBlock) void embed_mfma_kernel(MArgs a) {
  using T = typename Half<PREC>::T;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T *ct = reinterpret_cast<T *>(smem_raw);                                  // [RP][DS]
  // pixel rows (16-bit) and the b tile (FP32) share one region
  unsigned char *region = reinterpret_cast<unsigned char *>(ct + (size_t)a.RP * a.DS);
  const size_t pt_bytes = sizeof(T) * (size_t)kTP * a.DS;
  const size_t bs_bytes = sizeof(float) * (size_t)kTP * (a.RP + 1);
  T *pt = reinterpret_cast<T *>(region);
  float *bs = reinterpret_cast<float *>(region);                             // [64][RP+1]
  float *cn2 = reinterpret_cast<float *>(region + (pt_bytes > bs_bytes ? pt_bytes : bs_bytes));
  float *np2 = cn2 + a.RP;
  float *red = np2 + kTP;
  stage_landmarks<PREC>(a, ct, cn2);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = lane & 15, rq = lane >> 4;
  const int BS = a.RP + 1;
  for (int64_t base = (int64_t)blockIdx.x * kTP; base < a.N; base += (int64_t)gridDim.x * kTP) {
    __syncthreads();
    stage_pixels<PREC>(a, base, pt, np2, red);
    __syncthreads();
    floatx4 acc[NT];
    tile_products<PREC, NT>(a, pt, ct, acc);
    __syncthreads();  // pt is overwritten by the b tile below
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int pxl = 16 * w + 4 * rq + i;
      const float n2 = np2[pxl];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (16 * t < a.RP) {
          const int k = 16 * t + col;
          const float d2 = fmaxf(n2 + cn2[k] - 2.0f * acc[t][i], 0.0f);
          bs[pxl * BS + k] = k < a.r ? exp2f(-d2 * a.inv2s2 * 1.4426950408889634f) : 0.0f;
        }
      }
    }
    __syncthreads();
    // u^T tile: U[k'][px] = sum_j F[j][k'] b[px][j]; A = F^T (k' x j), B = b^T (j x px)
    const int xs = 16 * w;  // this wave's pixels
    for (int t2 = 0; t2 < a.RE / 16; ++t2) {
      floatx4 o = {0.f, 0.f, 0.f, 0.f};
      const int kk = 16 * t2 + col;  // A row = output plane
      for (int s = 0; s < a.RP / 4; ++s) {
        const int j = 4 * s + rq;
        const float av = (kk < a.r_eff && j < a.r) ? a.F32[j * a.r_eff + kk] : 0.0f;
        const float bv = bs[(xs + col) * BS + j];
        o = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, o, 0, 0, 0);
      }
      // lane holds U[k' = 16 t2 + 4 rq + i][px = xs + col]
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int kp = 16 * t2 + 4 * rq + i;
        const int64_t x = base + xs + col;
        if (kp < a.r_eff && x < a.N) a.u[(int64_t)kp * a.N + x] = o[i];
      }
    }
  }
}

__global__ void mean_kernel(Guide g, int64_t N, float *mu) {
  // one block per guide dimension; FP64 sum in a fixed order
  __shared__ double red[256];
  const int d = blockIdx.x;
  double s = 0.0;
  if (g.kind == GUIDE_PATCH) {
    const int c = d % g.C;
    for (int64_t x = threadIdx.x; x < N; x += 256) s += g.f[x * g.C + c];
  } else {
    for (int64_t x = threadIdx.x; x < N; x += 256) s += guide_elem(g, x, d);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) mu[d] = (float)(red[0] / (double)N);
}

__global__ void f64_to_f32_kernel(const double *src, float *dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

MArgs make_args(const Guide &g, const float *c, int r, const float *mu) {
  MArgs a{};
  a.g = g;
  a.N = (int64_t)g.H * g.W;
  a.c = c;
  a.mu = mu;
  a.r = r;
  a.RP = (r + 15) / 16 * 16;
  a.Dp = (g.D + 31) / 32 * 32;
  a.DS = a.Dp + 8;
  return a;
}

template <int PREC, int NT>
hipError_t launch_assign_nt(const MArgs &a, hipStream_t s) {
  using T = typename Half<PREC>::T;
  const size_t sm = sizeof(T) * ((size_t)a.RP + kTP) * a.DS + sizeof(float) * (a.RP + kTP + 4 * kTP);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(assign_mfma_kernel<PREC, NT>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  int64_t blocks = (a.N + kTP - 1) / kTP;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL((assign_mfma_kernel<PREC, NT>), dim3((int)blocks), dim3(kBlock), sm, s, a);
  return hipGetLastError();
}

template <int PREC, int NT>
hipError_t launch_embed_nt(const MArgs &a, hipStream_t s) {
  using T = typename Half<PREC>::T;
  const size_t pt_bytes = sizeof(T) * (size_t)kTP * a.DS;
  const size_t bs_bytes = sizeof(float) * (size_t)kTP * (a.RP + 1);
  const size_t sm = sizeof(T) * (size_t)a.RP * a.DS + (pt_bytes > bs_bytes ? pt_bytes : bs_bytes) +
                    sizeof(float) * (a.RP + kTP + 4 * kTP);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(embed_mfma_kernel<PREC, NT>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  int64_t blocks = (a.N + kTP - 1) / kTP;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL((embed_mfma_kernel<PREC, NT>), dim3((int)blocks), dim3(kBlock), sm, s, a);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_assign_p(const MArgs &a, hipStream_t s) {
  if (a.RP <= 64) return launch_assign_nt<PREC, 4>(a, s);
  if (a.RP <= 128) return launch_assign_nt<PREC, 8>(a, s);
  return launch_assign_nt<PREC, 16>(a, s);
}
template <int PREC>
hipError_t launch_embed_p(const MArgs &a, hipStream_t s) {
  if (a.RP <= 64) return launch_embed_nt<PREC, 4>(a, s);
  if (a.RP <= 128) return launch_embed_nt<PREC, 8>(a, s);
  return launch_embed_nt<PREC, 16>(a, s);
}

}  // namespace

hipError_t launch_guide_mean(const Guide &g, float *mu, hipStream_t s) {
  hipLaunchKernelGGL(mean_kernel, dim3(g.D), dim3(256), 0, s, g, (int64_t)g.H * g.W, mu);
  return hipGetLastError();
}

hipError_t launch_assign_mfma(const Guide &g, const float *c, int r, const float *mu, int prec, int *labels,
                              hipStream_t s) {
  MArgs a = make_args(g, c, r, mu);
  a.labels = labels;
  return prec == 1 ? launch_assign_p<1>(a, s) : launch_assign_p<2>(a, s);
}

hipError_t launch_embed_mfma(const Guide &g, const float *c, int r, const float *mu, const double *F, float *F32,
                             int r_eff, double sigma_r, int prec, float *u, hipStream_t s) {
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3((r * r_eff + 255) / 256), dim3(256), 0, s, F, F32, r * r_eff);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  MArgs a = make_args(g, c, r, mu);
  a.F32 = F32;
  a.r_eff = r_eff;
  a.RE = (r_eff + 15) / 16 * 16;
  a.inv2s2 = isinf(sigma_r) ? 0.0f : (float)(1.0 / (2.0 * sigma_r * sigma_r));
  a.u = u;
  return prec == 1 ? launch_embed_p<1>(a, s) : launch_embed_p<2>(a, s);
}

}  // namespace nkf
