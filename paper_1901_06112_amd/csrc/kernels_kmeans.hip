// k-means landmarks (Section III: landmarks are the centroids of a k-means
// partition of the guide values; Algorithm 1 clustering step).
//
// One Lloyd iteration = assignment (nearest centroid, ties to the lowest
// index) fused with the per-cluster sums, then the mean update.  Small guide
// dimensions (D <= 4, explicit or self guide) run one pixel per lane with the
// centroids in LDS; larger D use a labels pass, then a separate accumulation
// pass: for D > 32 (hyperspectral bands, NLM patches) the labels come from
// FP32 products on the matrix cores (kernels_mfma.hip), else from an LDS pixel
// tile with register-blocked distances on the VALU (below).  The 16-bit
// precision forms' k-means is in kernels_mfma.hip.
#include <hip/hip_runtime.h>
#include <float.h>

#include "device_common.h"

namespace nkf {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxPartials = 1024;        // blocks of the small-D assignment
constexpr int kMaxPartialsGeneric = 256;  // blocks of the generic accumulation
constexpr int kMaxPartialsOwned = 1024;   // blocks of the owned-dimension accumulation

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

// Block b writes its per-cluster sums to partials[b][r][D+1] (every entry,
// zeros included); the update kernel reduces the partials in block order.
// Distances in the GEMM form |c|^2 - 2 p.c (|p|^2 is common to all clusters
// and drops out of the argmin); each lane adds its pixel to one of ncopy
// FP64 accumulator sets in LDS (thread % ncopy) with native LDS atomics:
// neighbouring pixels mostly share a cluster, and one set would serialise a
// wave's atomics on the same words.  The sets (stride padded by one double so
// that they start on different banks) are summed in a fixed order at the end.
constexpr int kSmallCopiesMax = 32;
constexpr int kSmallPx = 4;  // pixels per thread and pass of the small-D assignment
constexpr size_t kSmallCopiesLds = 64 * 1024;

template <int D>
__global__ __launch_bounds__(kBlock) void assign_small_kernel(const float *__restrict__ P, int64_t N,
                                                              const float *__restrict__ c, int r,
                                                              double *__restrict__ partials,
                                                              int *__restrict__ labels, int ncopy) {
  constexpr int DS = D + 1;  // stored per cluster: -2 c (D values), |c|^2
  __shared__ __attribute__((aligned(16))) float sc[kMaxLandmarks * DS];
  extern __shared__ double sacc_all[];  // [ncopy][r (D+1) + 1]
  const int tid = threadIdx.x;
  const int cstride = r * (D + 1) + 1;
  double *sacc = sacc_all + (tid % ncopy) * cstride;
  for (int k = tid; k < r; k += kBlock) {
    float n2 = 0.0f;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const float v = c[k * D + j];
      sc[k * DS + j] = -2.0f * v;
      n2 = fmaf(v, v, n2);
    }
    sc[k * DS + D] = n2;
  }
  for (int i = tid; i < ncopy * cstride; i += kBlock) sacc_all[i] = 0.0;
  __syncthreads();
  // kSmallPx pixels per thread per pass share each centroid read and
  // interleave independent distance chains
  constexpr int PX = kSmallPx;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t xb = (int64_t)blockIdx.x * kBlock + tid; xb < N; xb += PX * stride) {
    float pv[PX][D];
    bool vv[PX];
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      const int64_t x = xb + q * stride;
      vv[q] = x < N;
#pragma unroll
      for (int j = 0; j < D; ++j) pv[q][j] = vv[q] ? P[x * D + j] : 0.0f;
    }
    float b[PX];
    int bi[PX];
#pragma unroll
    for (int q = 0; q < PX; ++q) b[q] = FLT_MAX, bi[q] = 0;
    for (int k = 0; k < r; ++k) {
      float d[PX];
#pragma unroll
      for (int q = 0; q < PX; ++q) d[q] = sc[k * DS + D];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const float cj = sc[k * DS + j];
#pragma unroll
        for (int q = 0; q < PX; ++q) d[q] = fmaf(pv[q][j], cj, d[q]);
      }
#pragma unroll
      for (int q = 0; q < PX; ++q)
        if (d[q] < b[q]) {
          b[q] = d[q];
          bi[q] = k;
        }
    }
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      if (!vv[q]) continue;
      if (labels) labels[xb + q * stride] = bi[q];
#pragma unroll
      for (int j = 0; j < D; ++j) atomicAdd(&sacc[bi[q] * (D + 1) + j], (double)pv[q][j]);
      atomicAdd(&sacc[bi[q] * (D + 1) + D], 1.0);
    }
  }
  __syncthreads();
  double *dst = partials + (size_t)blockIdx.x * r * (D + 1);
  for (int i = tid; i < r * (D + 1); i += kBlock) {
    double s = 0.0;
    for (int q = 0; q < ncopy; ++q) s += sacc_all[q * cstride + i];
    dst[i] = s;
  }
}

// ---- generic D: labels from a pixel tile in LDS ----------------------------
constexpr int kTilePx = 64;

// Register block of the generic assignment: clusters per distance pass.
constexpr int kAssignRB = 8;

// ct[d][k] = c[k][d] with rows padded to RP = r rounded up to kAssignRB
// (zeros past r)
__global__ void transpose_centroids_kernel(const float *__restrict__ c, int r, int D, int RP,
                                           float *__restrict__ ct) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D * RP) return;
  const int d = e / RP, k = e - d * RP;
  ct[e] = k < r ? c[k * D + d] : 0.0f;
}

// Nearest landmark of every pixel for any D (Algorithm 1, assignment; used for
// D <= 32 and when the matrix-core form's landmark tile does not fit LDS): a
// 64-pixel tile staged in LDS as [D][64]; wave kg scans the contiguous
// cluster range [kg CW, (kg + 1) CW) (CW a multiple of kAssignRB) with the
// landmarks transposed, so the clusters of a register block are 16-byte
// scalar loads per dimension; the four waves' minima merge with the lower
// index winning ties.  For a patch guide every thread stages dimensions
// d = kg, kg + 4, ... of its own pixel, the patch offset of d read from a
// per-block table.
__global__ __launch_bounds__(kBlock) void assign_generic_kernel(Guide g, int64_t N, const float *__restrict__ ct,
                                                                int RP, int r, int *__restrict__ labels) {
  extern __shared__ float smem[];
  float *pt = smem;                              // [D][64]
  float *sbest = smem + (size_t)g.D * kTilePx;   // [4][64]
  int *sidx = reinterpret_cast<int *>(sbest + 4 * kTilePx);
  int *ptab = sidx + 4 * kTilePx;                // [D] channel | dx << 8 | dy << 16
  const int tid = threadIdx.x;
  const int px = tid & (kTilePx - 1);
  const int kg = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int D = g.D;
  const bool patch = g.kind == GUIDE_PATCH;
  if (patch) {
    const int T = 2 * g.pr + 1;
    for (int d = tid; d < D; d += kBlock) {
      const int q = d / g.C;
      ptab[d] = (d - q * g.C) | ((q % T) << 8) | ((q / T) << 16);
    }
  }
  const int CW = ((r + 3) / 4 + kAssignRB - 1) / kAssignRB * kAssignRB;
  const int k0 = kg * CW, k1 = min(r, k0 + CW);
  for (int64_t base = (int64_t)blockIdx.x * kTilePx; base < N; base += (int64_t)gridDim.x * kTilePx) {
    __syncthreads();
    if (patch) {
      const int64_t x = base + px;
      const int64_t xs = x < N ? x : N - 1;
      const int y = (int)(xs / g.W), xx = (int)(xs - (int64_t)y * g.W);
      for (int d = kg; d < D; d += 4) {
        const int t = ptab[d];
        const int yy = sym_index(y + (t >> 16) - g.pr, g.H);
        const int xq = sym_index(xx + ((t >> 8) & 255) - g.pr, g.W);
        const float v = g.f[((int64_t)yy * g.W + xq) * g.C + (t & 255)];
        pt[d * kTilePx + px] = x < N ? v : 0.0f;
      }
    } else {
      for (int e = tid; e < D * kTilePx; e += kBlock) {
        const int d = e / kTilePx, q = e - d * kTilePx;
        const int64_t x = base + q;
        pt[e] = x < N ? guide_elem(g, x, d) : 0.0f;
      }
    }
    __syncthreads();
    float best = FLT_MAX;
    int bi = 0;
    for (int j0 = k0; j0 < k1; j0 += kAssignRB) {
      float acc[kAssignRB];
#pragma unroll
      for (int q = 0; q < kAssignRB; ++q) acc[q] = 0.f;
      // unrolled so that the scalar landmark loads of four steps are in flight together
#pragma unroll 4
      for (int d = 0; d < D; ++d) {
        const float v = pt[d * kTilePx + px];
        const float4 *crow = reinterpret_cast<const float4 *>(ct + (size_t)d * RP + j0);
#pragma unroll
        for (int h = 0; h < kAssignRB / 4; ++h) {
          const float4 cq = crow[h];
          const float t0 = v - cq.x, t1 = v - cq.y, t2 = v - cq.z, t3 = v - cq.w;
          acc[4 * h] = fmaf(t0, t0, acc[4 * h]);
          acc[4 * h + 1] = fmaf(t1, t1, acc[4 * h + 1]);
          acc[4 * h + 2] = fmaf(t2, t2, acc[4 * h + 2]);
          acc[4 * h + 3] = fmaf(t3, t3, acc[4 * h + 3]);
        }
      }
#pragma unroll
      for (int q = 0; q < kAssignRB; ++q) {
        if (j0 + q < k1 && acc[q] < best) {
          best = acc[q];
          bi = j0 + q;
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

// Per-cluster sums without contention (D + 1 <= kBlock): thread t owns
// dimension d = t % (D+1) (d = D is the count) of pixel stripe s = t / (D+1)
// (ns = kBlock / (D+1) stripes, each a contiguous share of the block's
// pixels).  It keeps a running FP32 sum while consecutive pixels of its
// stripe share a label and adds it to its own LDS word sacc[s][L][d] when the
// label changes (no other thread touches that word, so the sum and its order
// are fixed; a plain read and write, which measured faster than LDS atomics).
// The stripes' rows are added in stripe order, so the sums do not depend on
// timing.  Labels and values are read kOwnedBatch pixels at a time, ahead of
// the sequential scan, with every address in bounds: a slot past the stripe
// repeats the last label with value 0.  PATCH: the thread's (dy, dx, channel)
// is fixed and the pixel coordinates advance one column at a time; otherwise
// the value is p[x D + d] (an explicit guide, or the image itself, D = C).
constexpr int kOwnedBatch = 16;

template <bool PATCH>
__global__ __launch_bounds__(kBlock) void accumulate_owned_kernel(Guide g, int64_t N, int64_t per_block,
                                                                  const int *__restrict__ labels, int r,
                                                                  double *__restrict__ partials) {
  extern __shared__ float sacc[];  // [ns][r][D+1]
  const int tid = threadIdx.x;
  const int D = g.D, Dp = D + 1;
  const int ns = kBlock / Dp;
  const int rows = r * Dp;
  for (int i = tid; i < ns * rows; i += kBlock) sacc[i] = 0.0f;
  __syncthreads();
  const int s = tid / Dp, d = tid - s * Dp;
  if (s < ns) {
    const int64_t x0 = (int64_t)blockIdx.x * per_block;
    const int64_t x1 = x0 + per_block < N ? x0 + per_block : N;
    const int64_t sp = (x1 - x0 + ns - 1) / ns;
    const int64_t xs0 = x0 + s * sp;
    const int64_t xs1 = xs0 + sp < x1 ? xs0 + sp : x1;
    if (xs0 < xs1) {
      float *row = sacc + (size_t)s * rows + d;
      const bool cnt = d == D;
      const int dd = cnt ? 0 : d;
      int pdy = 0, pdx = 0, pc = 0;
      if (PATCH) {
        const int T = 2 * g.pr + 1, q = dd / g.C;
        pc = dd - q * g.C;
        pdx = q % T - g.pr;
        pdy = q / T - g.pr;
      }
      const float *src = g.kind == GUIDE_EXPLICIT ? g.p : g.f;
      int cy = (int)(xs0 / g.W), cx = (int)(xs0 - (int64_t)cy * g.W);
      float run = 0.0f;
      int L = labels[xs0];
      for (int64_t xb = xs0; xb < xs1; xb += kOwnedBatch) {
        int lb[kOwnedBatch];
        float vb[kOwnedBatch];
        int lprev = L;
#pragma unroll
        for (int q = 0; q < kOwnedBatch; ++q) {
          const int64_t x = xb + q;
          const bool in = x < xs1;
          const int64_t xa = in ? x : xs1 - 1;
          const int lab = labels[xa];
          float v;
          if (PATCH) {
            // cy passes H - 1 only after the image's last pixel; clamp it for the address
            const int yy = sym_index(min(cy, g.H - 1) + pdy, g.H), xq = sym_index(cx + pdx, g.W);
            v = g.f[((int64_t)yy * g.W + xq) * g.C + pc];
            const int cx1 = cx + 1;
            const bool wrap = cx1 == g.W;
            cx = wrap ? 0 : cx1;
            cy = wrap ? cy + 1 : cy;
          } else {
            v = src[xa * D + dd];
          }
          lb[q] = in ? lab : lprev;
          lprev = lb[q];
          vb[q] = in ? (cnt ? 1.0f : v) : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < kOwnedBatch; ++q) {
          if (lb[q] != L) {
            row[(size_t)L * Dp] += run;
            run = 0.0f;
            L = lb[q];
          }
          run += vb[q];
        }
      }
      row[(size_t)L * Dp] += run;
    }
  }
  __syncthreads();
  double *sums = partials + (size_t)blockIdx.x * rows;
  for (int i = tid; i < rows; i += kBlock) {
    double t = 0.0;
    for (int q = 0; q < ns; ++q) t += (double)sacc[(size_t)q * rows + i];
    sums[i] = t;
  }
}

// Per-cluster sums of the guide values given labels, into this block's slot
// partials[b][r][D+1]: accumulated in FP32 LDS when it fits (each block sums
// at most a few thousand pixels), otherwise in FP64 directly in the slot
// (which is zeroed first).
__global__ __launch_bounds__(kBlock) void accumulate_generic_kernel(Guide g, int64_t N,
                                                                    const int *__restrict__ labels,
                                                                    int r, double *__restrict__ partials,
                                                                    int use_lds) {
  extern __shared__ float sacc[];  // [r][D+1] when use_lds
  const int tid = threadIdx.x;
  const int D = g.D;
  const int stride = D + 1;
  double *sums = partials + (size_t)blockIdx.x * r * stride;
  if (use_lds) {
    for (int i = tid; i < r * stride; i += kBlock) sacc[i] = 0.0f;
  } else {
    for (int i = tid; i < r * stride; i += kBlock) sums[i] = 0.0;
  }
  __syncthreads();
  // Each lane adds its pixel's guide vector to its cluster's row: lanes of a
  // wave that share a label hit the same LDS word and are serialised by the
  // LDS unit, which is still far cheaper than reducing across the wave once
  // per distinct label.
  auto add = [&](int L, int d, float v) {
    if (use_lds)
      atomicAdd(&sacc[L * stride + d], v);
    else
      atomicAdd(&sums[L * stride + d], (double)v);
  };
  for (int64_t x = (int64_t)blockIdx.x * kBlock + tid; x < N; x += (int64_t)gridDim.x * kBlock) {
    const int L = labels[x];
    if (g.kind == GUIDE_PATCH) {
      // walk the patch as (dy, dx, c) with incremental addressing
      const int T = 2 * g.pr + 1;
      const int y = (int)(x / g.W), xx = (int)(x - (int64_t)y * g.W);
      int d = 0;
      for (int dy = 0; dy < T; ++dy) {
        const int yy = sym_index(y + dy - g.pr, g.H);
        const float *row = g.f + (int64_t)yy * g.W * g.C;
        for (int dx = 0; dx < T; ++dx) {
          const float *px = row + (int64_t)sym_index(xx + dx - g.pr, g.W) * g.C;
          for (int c = 0; c < g.C; ++c, ++d) add(L, d, px[c]);
        }
      }
    } else {
      const float *px = g.kind == GUIDE_EXPLICIT ? g.p + x * D : g.f + x * g.C;
      for (int d = 0; d < D; ++d) add(L, d, px[d]);
    }
    add(L, D, 1.0f);
  }
  if (use_lds) {
    __syncthreads();
    for (int i = tid; i < r * stride; i += kBlock) sums[i] = (double)sacc[i];
  }
}

// c_k[d] = mu(d) + S_k[d] / n_k from the per-block partial sums (S of the
// centred values when mu is given, of the raw values otherwise; mu_mod > 0
// indexes mu by d % mu_mod).  An empty cluster keeps its centroid.  One block
// per cluster of UB threads (1024 when D + 1 > 64, so that wide rows still get
// several lanes per column; 256 otherwise, where the lane sums' ordered combine
// would dominate); the D sums and the count (column D) are formed in groups
// of up to UB columns, each column summed by G lanes (partial b on lane
// b mod G, loads issued eight at a time) and the G lane sums added in lane
// order: a fixed order, so the result does not depend on timing.
template <int UB>
__global__ __launch_bounds__(UB) void update_kernel(const double *__restrict__ partials, int nparts, int r, int D,
                                                    const float *__restrict__ mu, int mu_mod,
                                                    float *__restrict__ c) {
  constexpr int kUpdBlock = UB;
  __shared__ double red[kUpdBlock];
  __shared__ double tot[kMaxGuideDim + 1];
  const int k = blockIdx.x, tid = threadIdx.x;
  const int DA = D + 1;
  const size_t stride = (size_t)r * DA;
  const double *base = partials + (size_t)k * DA;
  for (int m0 = 0; m0 < DA; m0 += kUpdBlock) {
    const int M = DA - m0 < kUpdBlock ? DA - m0 : kUpdBlock;
    const int G = kUpdBlock / M;
    const int m = tid % M, gl = tid / M;
    double s = 0.0;
    if (gl < G) {
      int b = gl;
      for (; b + 7 * G < nparts; b += 8 * G) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = base[(size_t)(b + j * G) * stride + m0 + m];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j];
      }
      for (; b < nparts; b += G) s += base[(size_t)b * stride + m0 + m];
    }
    red[tid] = s;
    __syncthreads();
    if (tid < M) {
      double t = 0.0;
      for (int q = 0; q < G; ++q) t += red[q * M + tid];
      tot[m0 + tid] = t;
    }
    __syncthreads();
  }
  const double n = tot[D];
  if (!(n > 0.0)) return;
  for (int d = tid; d < D; d += kUpdBlock) {
    const double off = mu ? (double)mu[mu_mod > 0 ? d % mu_mod : d] : 0.0;
    c[k * D + d] = (float)(off + tot[d] / n);
  }
}

// the owned-dimension accumulation: D + 1 threads per stripe, and the
// stripes' FP32 rows fit in 96 KB of LDS
bool owned_applies(int r, int D) {
  return D + 1 <= kBlock && sizeof(float) * (size_t)r * (D + 1) * (kBlock / (D + 1)) <= 96 * 1024;
}

int grid_for(int64_t n, int per_block, int cap) {
  int64_t b = (n + per_block - 1) / per_block;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

template <int D>
hipError_t launch_small(const Guide &g, const float *c, int r, double *partials, int *labels, int *nparts,
                        hipStream_t s) {
  const int64_t N = (int64_t)g.H * g.W;
  const float *P = g.kind == GUIDE_EXPLICIT ? g.p : g.f;
  *nparts = grid_for(N, kBlock * 8, kMaxPartials);
  const size_t set_bytes = sizeof(double) * ((size_t)r * (D + 1) + 1);
  int ncopy = (int)(kSmallCopiesLds / set_bytes);
  ncopy = ncopy < 1 ? 1 : (ncopy > kSmallCopiesMax ? kSmallCopiesMax : ncopy);
  const size_t sm = set_bytes * ncopy;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(assign_small_kernel<D>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(assign_small_kernel<D>, dim3(*nparts), dim3(kBlock), sm, s, P, N, c, r, partials, labels,
                     ncopy);
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

static hipError_t assign_accumulate(const Guide &g, const float *c, int r, double *partials, int *labels,
                                    int *label_scratch, float *ct, int *nparts, hipStream_t s) {
  const bool contiguous = g.kind != GUIDE_PATCH || g.pr == 0;
  if (contiguous) {
    switch (g.D) {
      case 1: return launch_small<1>(g, c, r, partials, labels, nparts, s);
      case 2: return launch_small<2>(g, c, r, partials, labels, nparts, s);
      case 3: return launch_small<3>(g, c, r, partials, labels, nparts, s);
      case 4: return launch_small<4>(g, c, r, partials, labels, nparts, s);
      default: break;
    }
  }
  const int64_t N = (int64_t)g.H * g.W;
  int *lab = labels ? labels : label_scratch;
  hipError_t e;
  if (assign_mfma32_supported(g, r)) {
    // the FP32 products on the matrix cores
    e = launch_assign_mfma32(g, c, r, lab, ct, s);
    if (e != hipSuccess) return e;
  } else {
    const size_t sm1 = sizeof(float) * ((size_t)g.D * kTilePx + 4 * kTilePx) + sizeof(int) * (4 * kTilePx + g.D);
    const int RP = (r + kAssignRB - 1) / kAssignRB * kAssignRB;
    hipLaunchKernelGGL(transpose_centroids_kernel, dim3((g.D * RP + 255) / 256), dim3(256), 0, s, c, r, g.D, RP,
                       ct);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(assign_generic_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm1);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(assign_generic_kernel, dim3(grid_for(N, kTilePx, 8192)), dim3(kBlock), sm1, s, g, N, ct,
                       RP, r, lab);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const size_t acc_bytes = sizeof(float) * (size_t)r * (g.D + 1);
  const int use_lds = acc_bytes <= 96 * 1024;
  if (owned_applies(r, g.D)) {
    const size_t own_bytes = acc_bytes * (kBlock / (g.D + 1));
    // about 1024 pixels per block: several blocks per CU even with one stripe
    // at least 256 pixels per block: up to kMaxPartialsOwned blocks, so that a
    // 512 x 512 image still fills every CU several times
    *nparts = grid_for(N, 256, kMaxPartialsOwned);
    const int64_t per_block = (N + *nparts - 1) / *nparts;
    auto *kern = g.kind == GUIDE_PATCH ? accumulate_owned_kernel<true> : accumulate_owned_kernel<false>;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)own_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(*nparts), dim3(kBlock), own_bytes, s, g, N, per_block, lab, r, partials);
    return hipGetLastError();
  }
  if (use_lds) {
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(accumulate_generic_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)acc_bytes);
    if (e != hipSuccess) return e;
  }
  *nparts = grid_for(N, kBlock * 16, kMaxPartialsGeneric);
  hipLaunchKernelGGL(accumulate_generic_kernel, dim3(*nparts), dim3(kBlock), use_lds ? acc_bytes : 0, s, g, N,
                     lab, r, partials, use_lds);
  return hipGetLastError();
}

size_t kmeans_transposed_floats(const Guide &g, int r) {
  const size_t t = (size_t)g.D * (size_t)((r + kAssignRB - 1) / kAssignRB * kAssignRB);
  const size_t m = assign_mfma32_supported(g, r) ? assign_mfma32_scratch_floats(g, r) : 0;
  return t > m ? t : m;
}

size_t kmeans_partials_doubles(int r, int D) {
  // (the MFMA path: at most 256 blocks)
  const int parts = D <= 4 ? kMaxPartials : (owned_applies(r, D) ? kMaxPartialsOwned : kMaxPartialsGeneric);
  return (size_t)parts * r * (D + 1);
}

static hipError_t launch_update(const double *partials, int nparts, int r, int D, const float *mu, int mu_mod,
                                float *c, hipStream_t s) {
  if (D + 1 > 64)
    hipLaunchKernelGGL(update_kernel<1024>, dim3(r), dim3(1024), 0, s, partials, nparts, r, D, mu, mu_mod, c);
  else
    hipLaunchKernelGGL(update_kernel<256>, dim3(r), dim3(256), 0, s, partials, nparts, r, D, mu, mu_mod, c);
  return hipGetLastError();
}

hipError_t launch_kmeans_step_mfma(const Guide &g, float *c, int r, const float *mu, int prec, double *partials,
                                   int *labels, void *lm_scratch, hipStream_t s) {
  int nparts = 0;
  hipError_t e = launch_lloyd_mfma(g, c, r, mu, prec, partials, labels, &nparts, lm_scratch, s);
  if (e != hipSuccess) return e;
  return launch_update(partials, nparts, r, g.D, mu, g.kind == GUIDE_PATCH ? g.C : 0, c, s);
}

hipError_t launch_kmeans_step(const Guide &g, float *c, int r, double *partials, int *labels, int *label_scratch,
                              float *ct, hipStream_t s) {
  int nparts = 0;
  hipError_t e = assign_accumulate(g, c, r, partials, labels, label_scratch, ct, &nparts, s);
  if (e != hipSuccess) return e;
  return launch_update(partials, nparts, r, g.D, nullptr, 0, c, s);
}

}  // namespace nkf
