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

// S[s][d] = p(x_s)_d: the sample's patches gathered once, row-major
__global__ __launch_bounds__(kBlock) void pca_gather_kernel(Guide g, const int64_t *__restrict__ idx, int ns,
                                                            float *__restrict__ S) {
  const int64_t total = (int64_t)ns * g.D;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
    const int s = (int)(e / g.D), d = (int)(e - (int64_t)s * g.D);
    S[e] = guide_elem(g, sample_pixel(idx, s), d);
  }
}

// partials[b][d] = sum of S[s][d] over block b's share of the sample
__global__ __launch_bounds__(kBlock) void pca_mean_kernel(const float *__restrict__ S, int ns, int D, int chunk,
                                                          double *__restrict__ partials) {
  const int s0 = blockIdx.x * chunk, s1 = min(ns, s0 + chunk);
  for (int d = threadIdx.x; d < D; d += kBlock) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int s = s0;
    for (; s + 4 <= s1; s += 4)
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] += (double)S[(size_t)(s + q) * D + d];
    for (; s < s1; ++s) a[0] += (double)S[(size_t)s * D + d];
    partials[(size_t)blockIdx.x * D + d] = (a[0] + a[1]) + (a[2] + a[3]);
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

// One 16 x 16 tile (ti <= tj) of sum_s (S_s - mu)(S_s - mu)^T over one chunk
// of the sample: thread (a, b) owns entry (16 ti + a, 16 tj + b); the centred
// values of 64 samples for both tiles' dimensions are staged in LDS per pass,
// and each pass feeds four accumulators (samples s mod 4), added in that
// order at the end.  cpart[chunk][i][j] for the entries of tiles with ti <= tj.
__global__ __launch_bounds__(kBlock) void pca_cov_kernel(const float *__restrict__ S, int ns, int D,
                                                         const double *__restrict__ mu, int chunk,
                                                         double *__restrict__ cpart) {
  __shared__ double xi[kCovBatch][kCovTile], xj[kCovBatch][kCovTile + 1];
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
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int sb = s0; sb < s1; sb += kCovBatch) {
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * kCovBatch * kCovTile; e += kBlock) {
      const int which = e / (kCovBatch * kCovTile);
      const int r = e % (kCovBatch * kCovTile);
      const int s = r / kCovTile, k = r % kCovTile;
      const int d = (which ? tj : ti) * kCovTile + k;
      double v = 0.0;
      if (sb + s < s1 && d < D) v = (double)S[(size_t)(sb + s) * D + d] - mu[d];
      if (which)
        xj[s][k] = v;
      else
        xi[s][k] = v;
    }
    __syncthreads();
#pragma unroll 8
    for (int s = 0; s < kCovBatch; ++s) acc[s & 3] = fma(xi[s][a], xj[s][b], acc[s & 3]);
  }
  const int i = ti * kCovTile + a, j = tj * kCovTile + b;
  if (i < D && j < D) cpart[((size_t)blockIdx.y * D + i) * D + j] = ((acc[0] + acc[1]) + acc[2]) + acc[3];
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

// g(x) = (p(x) - mu) V for one pixel per thread.  The patch dimension d is
// the same in every lane, so row d of V and mu[d] are scalar loads (through
// the scalar cache, each FMA takes its V entry from an SGPR pair); a patch
// row of T C values is walked with its mirrored column offsets fixed per lane.
template <int DIM>
__global__ __launch_bounds__(kBlock) void pca_project_kernel(Guide g, int64_t N, const double *__restrict__ mu,
                                                             const double *__restrict__ V,
                                                             float *__restrict__ out) {
  const int T = 2 * g.pr + 1, C = g.C;
  for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < N; x += (int64_t)gridDim.x * kBlock) {
    double acc[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) acc[k] = 0.0;
    const int y = (int)(x / g.W), xx = (int)(x - (int64_t)y * g.W);
    const double *vr = V;
    const double *mr = mu;
    for (int dy = 0; dy < T; ++dy) {
      const int yy = sym_index(y + dy - g.pr, g.H);
      const float *row = g.f + (int64_t)yy * g.W * C;
      for (int dx = 0; dx < T; ++dx) {
        const float *px = row + (int64_t)sym_index(xx + dx - g.pr, g.W) * C;
        for (int c = 0; c < C; ++c, vr += DIM, ++mr) {
          const double v = (double)px[c] - *mr;
#pragma unroll
          for (int k = 0; k < DIM; ++k) acc[k] = fma(v, vr[k], acc[k]);
        }
      }
    }
    float *o = out + x * DIM;
#pragma unroll
    for (int k = 0; k < DIM; ++k) o[k] = (float)acc[k];
  }
}

template <int DIM>
hipError_t launch_project_dim(const Guide &g, const double *mu, const double *V, float *out, hipStream_t s) {
  const int64_t N = (int64_t)g.H * g.W;
  int64_t blocks = (N + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(pca_project_kernel<DIM>, dim3((int)blocks), dim3(kBlock), 0, s, g, N, mu, V, out);
  return hipGetLastError();
}

}  // namespace

int pca_max_dim() { return kProjMaxDim; }

size_t pca_sample_floats(int D, int ns) { return (size_t)ns * D; }

hipError_t launch_pca_moments(const Guide &g, const int64_t *idx, int ns, int mean_blocks, int cov_chunks,
                              float *S, double *partials, double *mu, double *cpart, double *cov, hipStream_t s) {
  const int D = g.D;
  int64_t gb = ((int64_t)ns * D + kBlock - 1) / kBlock;
  if (gb > 16384) gb = 16384;
  hipLaunchKernelGGL(pca_gather_kernel, dim3((int)gb), dim3(kBlock), 0, s, g, idx, ns, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int chunk_m = (ns + mean_blocks - 1) / mean_blocks;
  hipLaunchKernelGGL(pca_mean_kernel, dim3(mean_blocks), dim3(kBlock), 0, s, S, ns, D, chunk_m, partials);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(pca_mean_final_kernel, dim3((D + 255) / 256), dim3(256), 0, s, partials, mean_blocks, D, ns, mu);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nt = (D + kCovTile - 1) / kCovTile;
  const int npairs = nt * (nt + 1) / 2;
  const int chunk_c = (ns + cov_chunks - 1) / cov_chunks;
  hipLaunchKernelGGL(pca_cov_kernel, dim3(npairs, cov_chunks), dim3(kBlock), 0, s, S, ns, D, mu, chunk_c, cpart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(pca_cov_final_kernel, dim3((D * D + 255) / 256), dim3(256), 0, s, cpart, cov_chunks, D, ns, cov);
  return hipGetLastError();
}

hipError_t launch_pca_project(const Guide &g, const double *mu, const double *V, int dim, float *out,
                              hipStream_t s) {
  switch (dim) {
#define NKF_DIM(n) \
  case n:          \
    return launch_project_dim<n>(g, mu, V, out, s);
    NKF_DIM(1) NKF_DIM(2) NKF_DIM(3) NKF_DIM(4) NKF_DIM(5) NKF_DIM(6) NKF_DIM(7) NKF_DIM(8)
    NKF_DIM(9) NKF_DIM(10) NKF_DIM(11) NKF_DIM(12) NKF_DIM(13) NKF_DIM(14) NKF_DIM(15) NKF_DIM(16)
    NKF_DIM(17) NKF_DIM(18) NKF_DIM(19) NKF_DIM(20) NKF_DIM(21) NKF_DIM(22) NKF_DIM(23) NKF_DIM(24)
    NKF_DIM(25) NKF_DIM(26) NKF_DIM(27) NKF_DIM(28) NKF_DIM(29) NKF_DIM(30) NKF_DIM(31) NKF_DIM(32)
#undef NKF_DIM
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace nkf
