// Principal-component patch guide of PCA-NLM (Section IV): the patch vectors
// p(x) ((2pr+1)^2 C values in (dy, dx, channel) order, symmetric padding) of
// a sample of pixels give the mean and the mean-centred covariance in FP64;
// the host eigensolver picks the basis V [D][dim]; every pixel's patch is then
// projected, g(x)_k = sum_d (p(x)_d - mean_d) V[d][k], in FP64 and stored as
// float32 [N][dim], an explicit guide for the filter.
//
// Sums over the sample run in a fixed order (per-block partials added in
// block order), so the basis does not depend on timing.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace nkf {

namespace {

constexpr int kBlock = 256;
constexpr int kCovTile = 16;     // output tile of the covariance (16 x 16 entries)
constexpr int kCovBatch = 64;    // samples staged per pass
constexpr int kProjMaxDim = 32;  // dim bound (registers of the projection)

__device__ __forceinline__ int64_t sample_pixel(const int64_t *idx, int s) { return idx ? idx[s] : (int64_t)s; }

// partials[b][d] = sum of p(x)_d over block b's share of the sample
__global__ __launch_bounds__(kBlock) void pca_mean_kernel(Guide g, const int64_t *__restrict__ idx, int ns,
                                                          int chunk, double *__restrict__ partials) {
  const int s0 = blockIdx.x * chunk, s1 = min(ns, s0 + chunk);
  for (int d = threadIdx.x; d < g.D; d += kBlock) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int s = s0;
    for (; s + 4 <= s1; s += 4)
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] += (double)guide_elem(g, sample_pixel(idx, s + q), d);
    for (; s < s1; ++s) a[0] += (double)guide_elem(g, sample_pixel(idx, s), d);
    partials[(size_t)blockIdx.x * g.D + d] = (a[0] + a[1]) + (a[2] + a[3]);
  }
}

__global__ void pca_mean_final_kernel(const double *__restrict__ partials, int nb, int D, int ns,
                                      double *__restrict__ mu) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partials[(size_t)b * D + d];
  mu[d] = s / ns;
}

// One 16 x 16 tile (ti <= tj) of sum_s (p_s - mu)(p_s - mu)^T over one chunk
// of the sample: thread (a, b) owns entry (16 ti + a, 16 tj + b); the centred
// values of 64 samples for both tiles' dimensions are staged in LDS per pass.
// cpart[chunk][i][j] for the entries of tiles with ti <= tj.
__global__ __launch_bounds__(kBlock) void pca_cov_kernel(Guide g, const int64_t *__restrict__ idx, int ns,
                                                         const double *__restrict__ mu, int chunk,
                                                         double *__restrict__ cpart) {
  __shared__ double xi[kCovBatch][kCovTile], xj[kCovBatch][kCovTile + 1];
  const int D = g.D;
  const int nt = (D + kCovTile - 1) / kCovTile;
  // pair index -> (ti, tj), ti <= tj, row-major over the upper triangle
  int pidx = blockIdx.x, ti = 0;
  while (pidx >= nt - ti) {
    pidx -= nt - ti;
    ++ti;
  }
  const int tj = ti + pidx;
  const int a = threadIdx.x / kCovTile, b = threadIdx.x % kCovTile;
  const int s0 = blockIdx.y * chunk, s1 = min(ns, s0 + chunk);
  double acc = 0.0;
  for (int sb = s0; sb < s1; sb += kCovBatch) {
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * kCovBatch * kCovTile; e += kBlock) {
      const int which = e / (kCovBatch * kCovTile);
      const int r = e % (kCovBatch * kCovTile);
      const int s = r / kCovTile, k = r % kCovTile;
      const int d = (which ? tj : ti) * kCovTile + k;
      double v = 0.0;
      if (sb + s < s1 && d < D) v = (double)guide_elem(g, sample_pixel(idx, sb + s), d) - mu[d];
      if (which)
        xj[s][k] = v;
      else
        xi[s][k] = v;
    }
    __syncthreads();
#pragma unroll 8
    for (int s = 0; s < kCovBatch; ++s) acc = fma(xi[s][a], xj[s][b], acc);
  }
  const int i = ti * kCovTile + a, j = tj * kCovTile + b;
  if (i < D && j < D) cpart[((size_t)blockIdx.y * D + i) * D + j] = acc;
}

// cov[i][j] = (sum over chunks, in order) / ns, from the computed triangle
__global__ void pca_cov_final_kernel(const double *__restrict__ cpart, int nchunks, int D, int ns,
                                     double *__restrict__ cov) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D * D) return;
  int i = e / D, j = e % D;
  if (i / kCovTile > j / kCovTile) {
    const int t = i;
    i = j;
    j = t;
  }
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += cpart[((size_t)c * D + i) * D + j];
  cov[e] = s / ns;
}

// g(x) = (p(x) - mu) V for one pixel per thread; V and mu in LDS.
__global__ __launch_bounds__(kBlock) void pca_project_kernel(Guide g, int64_t N, const double *__restrict__ mu,
                                                             const double *__restrict__ V, int dim,
                                                             float *__restrict__ out) {
  extern __shared__ double sm[];
  const int D = g.D;
  double *Vs = sm;              // [D][dim]
  double *ms = sm + D * dim;    // [D]
  for (int e = threadIdx.x; e < D * dim; e += kBlock) Vs[e] = V[e];
  for (int e = threadIdx.x; e < D; e += kBlock) ms[e] = mu[e];
  __syncthreads();
  const int T = 2 * g.pr + 1, C = g.C;
  for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < N; x += (int64_t)gridDim.x * kBlock) {
    double acc[kProjMaxDim];
#pragma unroll
    for (int k = 0; k < kProjMaxDim; ++k) acc[k] = 0.0;
    const int y = (int)(x / g.W), xx = (int)(x - (int64_t)y * g.W);
    int d = 0;
    for (int dy = 0; dy < T; ++dy) {
      const int yy = sym_index(y + dy - g.pr, g.H);
      const float *row = g.f + (int64_t)yy * g.W * C;
      for (int dx = 0; dx < T; ++dx) {
        const float *px = row + (int64_t)sym_index(xx + dx - g.pr, g.W) * C;
        for (int c = 0; c < C; ++c, ++d) {
          const double v = (double)px[c] - ms[d];
          const double *vr = Vs + d * dim;
#pragma unroll
          for (int k = 0; k < kProjMaxDim; ++k)
            if (k < dim) acc[k] = fma(v, vr[k], acc[k]);
        }
      }
    }
    float *o = out + x * dim;
#pragma unroll
    for (int k = 0; k < kProjMaxDim; ++k)
      if (k < dim) o[k] = (float)acc[k];
  }
}

}  // namespace

int pca_max_dim() { return kProjMaxDim; }

hipError_t launch_pca_moments(const Guide &g, const int64_t *idx, int ns, int mean_blocks, int cov_chunks,
                              double *partials, double *mu, double *cpart, double *cov, hipStream_t s) {
  const int chunk_m = (ns + mean_blocks - 1) / mean_blocks;
  hipLaunchKernelGGL(pca_mean_kernel, dim3(mean_blocks), dim3(kBlock), 0, s, g, idx, ns, chunk_m, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pca_mean_final_kernel, dim3((g.D + 255) / 256), dim3(256), 0, s, partials, mean_blocks, g.D,
                     ns, mu);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nt = (g.D + kCovTile - 1) / kCovTile;
  const int npairs = nt * (nt + 1) / 2;
  const int chunk_c = (ns + cov_chunks - 1) / cov_chunks;
  hipLaunchKernelGGL(pca_cov_kernel, dim3(npairs, cov_chunks), dim3(kBlock), 0, s, g, idx, ns, mu, chunk_c, cpart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(pca_cov_final_kernel, dim3((g.D * g.D + 255) / 256), dim3(256), 0, s, cpart, cov_chunks, g.D,
                     ns, cov);
  return hipGetLastError();
}

hipError_t launch_pca_project(const Guide &g, const double *mu, const double *V, int dim, float *out,
                              hipStream_t s) {
  const int64_t N = (int64_t)g.H * g.W;
  const size_t sm = sizeof(double) * ((size_t)g.D * dim + g.D);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(pca_project_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  int64_t blocks = (N + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(pca_project_kernel, dim3((int)blocks), dim3(kBlock), sm, s, g, N, mu, V, dim, out);
  return hipGetLastError();
}

}  // namespace nkf
