// k-means landmarks (Section III: landmarks are the centroids of a k-means
// partition of the guide values; Algorithm 1 clustering step).
//
// One Lloyd iteration = assignment (nearest centroid, ties to the lowest
// index) fused with the per-cluster sums, then the mean update.  Small guide
// dimensions (D <= 8, explicit or self guide) run one pixel per lane with the
// centroids in LDS; larger D (hyperspectral bands, NLM patches) use an LDS
// pixel tile and register-blocked distances, then a separate accumulation pass.
#include <hip/hip_runtime.h>
#include <float.h>

#include "device_common.h"

namespace nkf {

namespace {

constexpr int kBlock = 256;

__global__ void fill_f64_kernel(double *p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void gather_kernel(Guide g, const int64_t *__restrict__ idx, int r,
                              float *__restrict__ c) {
  const int n = r * g.D;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int i = e / g.D, d = e - i * g.D;
    c[e] = guide_elem(g, idx[i], d);
  }
}

// Adds the guide values (and a count of 1) of the lanes whose label is shared
// with the wave leader into acc[label][0..D], one distinct label at a time.
// All 64 lanes of the wave must call this together.
template <int D>
__device__ __forceinline__ void wave_accumulate_small(bool valid, int lab, const float (&pv)[D],
                                                      double *acc) {
  bool active = valid;
  while (true) {
    const uint64_t m = __ballot(active);
    if (m == 0) break;
    const int leader = __ffsll((unsigned long long)m) - 1;
    const int L = __shfl(lab, leader, kWave);
    const bool mine = active && lab == L;
    float s[D + 1];
#pragma unroll
    for (int j = 0; j < D; ++j) s[j] = wave_sum(mine ? pv[j] : 0.0f);
    s[D] = wave_sum(mine ? 1.0f : 0.0f);
    if (lane_id() == 0) {
#pragma unroll
      for (int j = 0; j <= D; ++j) atomicAdd(&acc[L * (D + 1) + j], (double)s[j]);
    }
    active = active && !mine;
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void assign_small_kernel(const float *__restrict__ P, int64_t N,
                                                              const float *__restrict__ c, int r,
                                                              double *__restrict__ sums,
                                                              int *__restrict__ labels) {
  __shared__ float sc[kMaxLandmarks * D];
  __shared__ double sacc[kMaxLandmarks * (D + 1)];
  const int tid = threadIdx.x;
  for (int i = tid; i < r * D; i += kBlock) sc[i] = c[i];
  for (int i = tid; i < r * (D + 1); i += kBlock) sacc[i] = 0.0;
  __syncthreads();
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < N; base += (int64_t)gridDim.x * kBlock) {
    const int64_t x = base + tid;
    const bool valid = x < N;
    float pv[D];
#pragma unroll
    for (int j = 0; j < D; ++j) pv[j] = valid ? P[x * D + j] : 0.0f;
    float best = FLT_MAX;
    int bi = 0;
    for (int k = 0; k < r; ++k) {
      float d2 = 0.0f;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const float t = pv[j] - sc[k * D + j];
        d2 = fmaf(t, t, d2);
      }
      if (d2 < best) {
        best = d2;
        bi = k;
      }
    }
    if (valid && labels) labels[x] = bi;
    wave_accumulate_small<D>(valid, bi, pv, sacc);
  }
  __syncthreads();
  for (int i = tid; i < r * (D + 1); i += kBlock)
    if (sacc[i] != 0.0) atomicAdd(&sums[i], sacc[i]);
}

// ---- generic D: labels from a pixel tile in LDS ----------------------------
constexpr int kTilePx = 64;

__global__ __launch_bounds__(kBlock) void assign_generic_kernel(Guide g, int64_t N,
                                                                const float *__restrict__ c, int r,
                                                                int *__restrict__ labels) {
  extern __shared__ float smem[];
  float *pt = smem;                              // [D][64]
  float *sbest = smem + (size_t)g.D * kTilePx;   // [4][64]
  int *sidx = reinterpret_cast<int *>(sbest + 4 * kTilePx);
  const int tid = threadIdx.x;
  const int px = tid & (kTilePx - 1);
  const int kg = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int D = g.D;
  for (int64_t base = (int64_t)blockIdx.x * kTilePx; base < N; base += (int64_t)gridDim.x * kTilePx) {
    __syncthreads();
    for (int e = tid; e < D * kTilePx; e += kBlock) {
      const int d = e / kTilePx, q = e - d * kTilePx;
      const int64_t x = base + q;
      pt[e] = x < N ? guide_elem(g, x, d) : 0.0f;
    }
    __syncthreads();
    float best = FLT_MAX;
    int bi = 0;
    // clusters k = kg + 4 * j, register-blocked four at a time
    for (int j0 = 0; kg + 4 * j0 < r; j0 += 4) {
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
      int kk[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = kg + 4 * (j0 + q);
        kk[q] = k < r ? k : r - 1;
      }
      for (int d = 0; d < D; ++d) {
        const float v = pt[d * kTilePx + px];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float t = v - c[kk[q] * D + d];
          acc[q] = fmaf(t, t, acc[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = kg + 4 * (j0 + q);
        if (k < r && acc[q] < best) {
          best = acc[q];
          bi = k;
        }
      }
    }
    sbest[kg * kTilePx + px] = best;
    sidx[kg * kTilePx + px] = bi;
    __syncthreads();
    if (kg == 0) {
      float b = sbest[px];
      int bk = sidx[px];
      for (int q = 1; q < 4; ++q) {
        const float o = sbest[q * kTilePx + px];
        const int ok = sidx[q * kTilePx + px];
        if (o < b || (o == b && ok < bk)) {
          b = o;
          bk = ok;
        }
      }
      const int64_t x = base + px;
      if (x < N) labels[x] = bk;
    }
  }
}

// Per-cluster sums of the guide values given labels.  acc in LDS when it fits,
// otherwise straight to the global FP64 sums.
__global__ __launch_bounds__(kBlock) void accumulate_generic_kernel(Guide g, int64_t N,
                                                                    const int *__restrict__ labels,
                                                                    int r, double *__restrict__ sums,
                                                                    int use_lds) {
  extern __shared__ float sacc[];  // [r][D+1] when use_lds
  const int tid = threadIdx.x;
  const int D = g.D;
  const int stride = D + 1;
  if (use_lds) {
    for (int i = tid; i < r * stride; i += kBlock) sacc[i] = 0.0f;
    __syncthreads();
  }
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < N; base += (int64_t)gridDim.x * kBlock) {
    const int64_t x = base + tid;
    const bool valid = x < N;
    const int lab = valid ? labels[x] : 0;
    bool active = valid;
    while (true) {
      const uint64_t m = __ballot(active);
      if (m == 0) break;
      const int leader = __ffsll((unsigned long long)m) - 1;
      const int L = __shfl(lab, leader, kWave);
      const bool mine = active && lab == L;
      for (int d = 0; d < D; ++d) {
        const float s = wave_sum(mine ? guide_elem(g, x, d) : 0.0f);
        if (lane_id() == 0) {
          if (use_lds)
            atomicAdd(&sacc[L * stride + d], s);
          else
            atomicAdd(&sums[L * stride + d], (double)s);
        }
      }
      const float cnt = wave_sum(mine ? 1.0f : 0.0f);
      if (lane_id() == 0) {
        if (use_lds)
          atomicAdd(&sacc[L * stride + D], cnt);
        else
          atomicAdd(&sums[L * stride + D], (double)cnt);
      }
      active = active && !mine;
    }
  }
  if (use_lds) {
    __syncthreads();
    for (int i = tid; i < r * stride; i += kBlock)
      if (sacc[i] != 0.0f) atomicAdd(&sums[i], (double)sacc[i]);
  }
}

__global__ void update_kernel(const double *__restrict__ sums, int r, int D, float *__restrict__ c) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * D) return;
  const int k = e / D, d = e - k * D;
  const double cnt = sums[k * (D + 1) + D];
  if (cnt > 0.0) c[e] = (float)(sums[k * (D + 1) + d] / cnt);
}

int grid_for(int64_t n, int per_block, int cap) {
  int64_t b = (n + per_block - 1) / per_block;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

template <int D>
hipError_t launch_small(const Guide &g, const float *c, int r, double *sums, int *labels, hipStream_t s) {
  const int64_t N = (int64_t)g.H * g.W;
  const float *P = g.kind == GUIDE_EXPLICIT ? g.p : g.f;
  hipLaunchKernelGGL(assign_small_kernel<D>, dim3(grid_for(N, kBlock * 4, 2048)), dim3(kBlock), 0, s,
                     P, N, c, r, sums, labels);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n, kBlock, 1024)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_gather_landmarks(const Guide &g, const int64_t *idx, int r, float *c, hipStream_t s) {
  hipLaunchKernelGGL(gather_kernel, dim3(grid_for((int64_t)r * g.D, kBlock, 256)), dim3(kBlock), 0, s, g,
                     idx, r, c);
  return hipGetLastError();
}

hipError_t launch_kmeans_assign(const Guide &g, const float *c, int r, double *sums, int *labels,
                                int *label_scratch, hipStream_t s) {
  const bool contiguous = g.kind != GUIDE_PATCH || g.pr == 0;
  if (contiguous) {
    switch (g.D) {
      case 1: return launch_small<1>(g, c, r, sums, labels, s);
      case 2: return launch_small<2>(g, c, r, sums, labels, s);
      case 3: return launch_small<3>(g, c, r, sums, labels, s);
      case 4: return launch_small<4>(g, c, r, sums, labels, s);
      default: break;
    }
  }
  const int64_t N = (int64_t)g.H * g.W;
  int *lab = labels ? labels : label_scratch;
  const size_t sm1 = sizeof(float) * ((size_t)g.D * kTilePx + 4 * kTilePx) + sizeof(int) * 4 * kTilePx;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(assign_generic_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(assign_generic_kernel, dim3(grid_for(N, kTilePx, 8192)), dim3(kBlock), sm1, s, g, N,
                     c, r, lab);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t acc_bytes = sizeof(float) * (size_t)r * (g.D + 1);
  const int use_lds = acc_bytes <= 96 * 1024;
  if (use_lds) {
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(accumulate_generic_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)acc_bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(accumulate_generic_kernel, dim3(grid_for(N, kBlock * 16, 1024)), dim3(kBlock),
                     use_lds ? acc_bytes : 0, s, g, N, lab, r, sums, use_lds);
  return hipGetLastError();
}

hipError_t launch_kmeans_update(const double *sums, int r, int D, float *c, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel, dim3((r * D + kBlock - 1) / kBlock), dim3(kBlock), 0, s, sums, r, D, c);
  return hipGetLastError();
}

}  // namespace nkf
