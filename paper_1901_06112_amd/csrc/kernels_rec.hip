// Recursive-Gaussian convolutions + contraction + normalisation (Section III,
// Eqs. (finalnum), (finalden), with the spatial Gaussian evaluated by Young and
// van Vliet's O(1) recursive filter as in Section IV) for images with up to
// three channels.
//
// The 1-D filter is the forward-backward cascade of Young and van Vliet's
// third-order recursion; its impulse response h is symmetric.  With the image
// extended by zeros (numerator and denominator alike, as for the truncated
// window), the filtered line is h convolved with the line.  It is evaluated
// here in parallel form, h = h+ + h-, with h+ the causal half (h+[0] = h[0]/2,
// h+[n] = h[n] for n > 0) and h- its mirror image.  For n > 0, h[n] is a sum
// of the cascade's three causal geometric modes, so h+ is the response of
// N(z) / A(z), A(z) = 1 - a1 z^-1 - a2 z^-2 - a3 z^-3 (the cascade's poles)
// and N(z) = n0 + n1 z^-1 + n2 z^-2 + n3 z^-3 fitted to h[0]/2, h[1], h[2],
// h[3].  It runs as the all-pole recursion followed by the numerator:
//   w[n] = x[n] + a1 w[n-1] + a2 w[n-2] + a3 w[n-3],
//   y+[n] = n0 w[n] + n1 w[n-1] + n2 w[n-2] + n3 w[n-3],
// so (w[n-1], w[n-2], w[n-3]) is the whole state.  y- runs the same from the
// other end.  Both start from rest at the line ends, which is exactly the
// zero extension.
//
// Each line is one thread's, in two phases: phase A runs the all-pole
// recursion along the whole line and keeps only its state at the start of
// every chunk of the line; phase C walks the chunks from the far end, reloads
// each chunk's inputs into registers, restarts the causal half from the kept
// state (the same FP64 values as one full sweep), runs the anticausal half
// back over the chunk, carried from the previous chunk, and stores y+ + y-
// once.  Per line and pass: the input read twice, the output written once,
// three doubles per chunk.
//
// For embedding plane u_k, the planes are u_k f~_c (f~ = f - f0) and u_k
// itself (plane 0); every recursion runs in FP64, the filtered planes are
// stored as FP32 between passes.
//   columns   block (64 columns, two k), wave = (k, plane): each lane owns a
//             column, chunks of 24 rows, the plane's input formed from u_k
//             and f on the fly (f copied to channel planes first, so a wave
//             reads only its channel, and both k of a block read it from the
//             same cache lines); output V_kp = column-filtered planes;
//   rows      block (64 rows, k), wave = plane: each lane owns a row of V_kp,
//             chunks of 32 columns (eight 16-byte loads); the output Z_kp
//             overwrites V_kp chunk by chunk (each chunk is read before it
//             is written, by the same thread);
//   contract  thread per pixel: eta = sum_k u_k Z_k0 and zeta_c =
//             sum_k u_k Z_k(c+1) in FP64, g = zeta / eta + f0 (f where eta
//             <= 0 or not finite).
// Rows of V are padded to Wp = W rounded up to 64 columns; the padding
// columns hold zeros (the zero extension) before the row pass and are never
// read after it.  The row stride is Wp + 32 floats: with a power-of-two
// stride the row pass's 64 lanes (64 rows) fall on fewer memory channels
// (measured 4% slower).  Every sweep prefetches its next chunk while it computes the
// current one.
#include <hip/hip_runtime.h>
#include <math.h>

#include <vector>

#include "device_common.h"
#include "nkf_internal.h"

namespace nkf {

namespace {

constexpr int kRL = 24;   // rows per chunk of the column pass
constexpr int kCL = 32;   // columns per chunk of the row pass (eight float4)

struct RecArgs {
  int H, W, Wp, ld, C, r_eff;  // ld: row stride of the planes
  int64_t N, plane;        // pixels; floats per stored plane (H * Wp)
  const float *f, *f0, *u;
  float *fpl;              // forward: f as channel planes [C][N]; backward: (beta, a_c) planes [C + 1][N]
  float *V;                // the filtered planes, [r_eff][C + 1][H][Wp]
  double *carry;           // causal states at chunk starts
  float *out, *eta_out;
  RecCoef k;
  // backward (bwd = 1): the planes' inputs are beta u_k and a_c u_k
  int bwd;
  const float *G, *eta, *ab;  // dL/dg [N][C], the forward's eta_hat [N], (beta, a_c) [N][4]
  float *dud, *du, *df;       // du_dir and du [r_eff][N], df [N][C]
};

// One half of the filter; w1..w3 hold the all-pole recursion's last three
// values.
struct Rec {
  double w1 = 0, w2 = 0, w3 = 0;
  __device__ double advance(const RecCoef &c, double x) {
    const double w = fma(c.a1, w1, fma(c.a2, w2, fma(c.a3, w3, x)));
    w3 = w2;
    w2 = w1;
    w1 = w;
    return w;
  }
  __device__ double step(const RecCoef &c, double x) {
    const double p1 = w1, p2 = w2, p3 = w3;
    const double w = advance(c, x);
    return fma(c.n0, w, fma(c.n1, p1, fma(c.n2, p2, c.n3 * p3)));
  }
};

constexpr int kColK = 2;  // embedding planes per block of the column pass

__global__ __launch_bounds__(512) void planar_kernel(RecArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.N * a.C;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pix = i / a.C;
    const int c = (int)(i - pix * a.C);
    a.fpl[c * a.N + pix] = a.f[i];
  }
}

__global__ __launch_bounds__(512) void planar_ab_kernel(RecArgs a) {
  const int P = a.C + 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.N * P;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pix = i / P;
    const int c = (int)(i - pix * P);
    a.fpl[c * a.N + pix] = a.ab[pix * 4 + c];
  }
}

__global__ __launch_bounds__(64 * kColK * 4) void rec_cols_kernel(RecArgs a) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int P = a.C + 1;
  const int p = w % P;  // 0: u_k, c + 1: u_k f~_c
  const int k = blockIdx.y * kColK + w / P;
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  if (k >= a.r_eff || x >= a.Wp) return;
  const bool valid = x < a.W;
  const int xc = valid ? x : a.W - 1;  // in-bounds address; the value is dropped when !valid
  // wave-uniform 64-bit bases, the lane's column as a 32-bit offset
  const float *__restrict__ ub = a.u + (int64_t)k * a.N;
  const float *__restrict__ fb = a.fpl + (int64_t)(a.bwd ? p : (p > 0 ? p - 1 : 0)) * a.N;
  const unsigned xo = (unsigned)xc, xs = (unsigned)x;
  const double f0 = p > 0 ? (double)a.f0[p - 1] : 0.0;
  const int H = a.H, Wp = a.Wp, ld = a.ld;
  const int64_t line = (int64_t)k * (a.C + 1) + p;
  float *__restrict__ vb = a.V + line * a.plane;
  const int nch = (H + kRL - 1) / kRL, nfull = H / kRL;
  double *__restrict__ cs = a.carry + line * nch * 3 * Wp + x;  // [chunk][3][Wp]
  const int64_t us = a.W, fs = a.W;
  // forward: plane 0 is u_k, plane c + 1 is u_k (f_c - f0_c); backward: u_k
  // times the plane's per-pixel coefficient (beta, a_c)
  const bool scaled = a.bwd || p > 0;
  const double off = a.bwd ? 0.0 : f0;
  auto input = [&](float uv, float fv) -> double {
    const double uu = valid ? (double)uv : 0.0;
    return scaled ? uu * ((double)fv - off) : uu;
  };
  auto load = [&](int y0, float (&U)[kRL], float (&F)[kRL]) {
#pragma unroll
    for (int j = 0; j < kRL; ++j) {
      U[j] = (ub + (int64_t)(y0 + j) * us)[xo];
      F[j] = (fb + (int64_t)(y0 + j) * fs)[xo];  // plane 0 loads channel 0 and ignores it: no branch
    }
  };
  auto keep = [&](int c, const Rec &r) {
    cs[(int64_t)(3 * c + 0) * Wp] = r.w1;
    cs[(int64_t)(3 * c + 1) * Wp] = r.w2;
    cs[(int64_t)(3 * c + 2) * Wp] = r.w3;
  };
  auto restart = [&](int c) {
    Rec r;
    r.w1 = cs[(int64_t)(3 * c + 0) * Wp];
    r.w2 = cs[(int64_t)(3 * c + 1) * Wp];
    r.w3 = cs[(int64_t)(3 * c + 2) * Wp];
    return r;
  };
  float cu[kRL], cf[kRL], nu[kRL], nf[kRL];
  // ---- phase A: causal states at the chunk starts
  {
    Rec r;
    if (nfull > 0) load(0, cu, cf);
    for (int c = 0; c < nfull; ++c) {
      // unconditional prefetch (the last chunk is loaded again at the end): a
      // load under a branch makes the compiler's wait at the join cover the
      // newer loads as well
      load((c + 1 < nfull ? c + 1 : c) * kRL, nu, nf);
      keep(c, r);
#pragma unroll
      for (int j = 0; j < kRL; ++j) r.advance(a.k, input(cu[j], cf[j]));
#pragma unroll
      for (int j = 0; j < kRL; ++j) {
        cu[j] = nu[j];
        cf[j] = nf[j];
      }
    }
    if (nfull < nch) keep(nfull, r);  // the short last chunk needs only its start
  }
  // ---- phase C: chunks from the bottom; causal restarted from the kept
  // state, anticausal carried, V = y+ + y-
  Rec ra;
  double yp[kRL];
  if (nfull < nch) {  // the short last chunk: the same steps, predicated
    const int y0 = nfull * kRL, len = H - y0;
#pragma unroll
    for (int j = 0; j < kRL; ++j) {
      const int64_t yy = y0 + (j < len ? j : len - 1);
      cu[j] = (ub + yy * us)[xo];
      cf[j] = (fb + yy * fs)[xo];
    }
    Rec rc = restart(nfull);
#pragma unroll
    for (int j = 0; j < kRL; ++j)
      if (j < len) yp[j] = rc.step(a.k, input(cu[j], cf[j]));
#pragma unroll
    for (int j = kRL - 1; j >= 0; --j)
      if (j < len) (vb + (int64_t)(y0 + j) * ld)[xs] = (float)(yp[j] + ra.step(a.k, input(cu[j], cf[j])));
  }
  // the kept state of the next chunk is loaded with its inputs, one chunk
  // ahead (a load issued after the prefetch and used at once would make the
  // wait cover the prefetch as well)
  Rec rc_next;
  if (nfull > 0) {
    rc_next = restart(nfull - 1);
    load((nfull - 1) * kRL, cu, cf);
  }
  for (int c = nfull - 1; c >= 0; --c) {
    Rec rc = rc_next;
    rc_next = restart(c > 0 ? c - 1 : 0);
    load((c > 0 ? c - 1 : 0) * kRL, nu, nf);
#pragma unroll
    for (int j = 0; j < kRL; ++j) yp[j] = rc.step(a.k, input(cu[j], cf[j]));
#pragma unroll
    for (int j = kRL - 1; j >= 0; --j)
      (vb + (int64_t)(c * kRL + j) * ld)[xs] = (float)(yp[j] + ra.step(a.k, input(cu[j], cf[j])));
#pragma unroll
    for (int j = 0; j < kRL; ++j) {
      cu[j] = nu[j];
      cf[j] = nf[j];
    }
  }
}

__global__ __launch_bounds__(256) void rec_rows_kernel(RecArgs a) {
  const int p = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int k = blockIdx.y;
  const int y = blockIdx.x * 64 + (threadIdx.x & 63);
  if (y >= a.H) return;
  const int64_t line = (int64_t)k * (a.C + 1) + p;
  // wave-uniform base of the plane, the lane's row as a 32-bit offset
  float4 *__restrict__ vb4 = reinterpret_cast<float4 *>(a.V + line * a.plane);
  const unsigned yo = (unsigned)y * (unsigned)(a.ld / 4);
  constexpr int Q = kCL / 4;
  const int nch = a.Wp / kCL;
  double *__restrict__ cs = a.carry + line * nch * 3 * a.H + y;  // [chunk][3][H]
  // Chunks go in pairs with the two register sets swapping roles (a copy of
  // the prefetched set would wait for it; nch is even), and prefetches are
  // unconditional, as in the column pass.
  float4 b0[Q], b1[Q];
  auto fetch = [&](int c, float4 (&B)[Q]) {
#pragma unroll
    for (int q = 0; q < Q; ++q) B[q] = (vb4 + c * Q + q)[yo];
  };
  // ---- phase A: causal states at the chunk starts
  {
    Rec r;
    auto step_a = [&](int c, const float4 (&B)[Q], float4 (&NB)[Q]) {
      fetch(c + 1 < nch ? c + 1 : c, NB);
      cs[(int64_t)(3 * c + 0) * a.H] = r.w1;
      cs[(int64_t)(3 * c + 1) * a.H] = r.w2;
      cs[(int64_t)(3 * c + 2) * a.H] = r.w3;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        r.advance(a.k, (double)B[q].x);
        r.advance(a.k, (double)B[q].y);
        r.advance(a.k, (double)B[q].z);
        r.advance(a.k, (double)B[q].w);
      }
    };
    fetch(0, b0);
    for (int c = 0; c < nch; c += 2) {
      step_a(c, b0, b1);
      step_a(c + 1, b1, b0);
    }
  }
  // ---- phase C: chunks from the right end, Z = y+ + y- over V in place; the
  // kept state of the next chunk is loaded with its inputs, one chunk ahead
  Rec ra;
  double yp[kCL];
  auto restart = [&](int c) {
    Rec r;
    r.w1 = cs[(int64_t)(3 * c + 0) * a.H];
    r.w2 = cs[(int64_t)(3 * c + 1) * a.H];
    r.w3 = cs[(int64_t)(3 * c + 2) * a.H];
    return r;
  };
  auto step_c = [&](int c, const Rec &rc0, const float4 (&B)[Q], Rec &rcn, float4 (&NB)[Q]) {
    const int cn = c > 0 ? c - 1 : 0;
    rcn = restart(cn);
    fetch(cn, NB);
    Rec rc = rc0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      yp[4 * q + 0] = rc.step(a.k, (double)B[q].x);
      yp[4 * q + 1] = rc.step(a.k, (double)B[q].y);
      yp[4 * q + 2] = rc.step(a.k, (double)B[q].z);
      yp[4 * q + 3] = rc.step(a.k, (double)B[q].w);
    }
#pragma unroll
    for (int q = Q - 1; q >= 0; --q) {
      float4 o;
      o.w = (float)(yp[4 * q + 3] + ra.step(a.k, (double)B[q].w));
      o.z = (float)(yp[4 * q + 2] + ra.step(a.k, (double)B[q].z));
      o.y = (float)(yp[4 * q + 1] + ra.step(a.k, (double)B[q].y));
      o.x = (float)(yp[4 * q + 0] + ra.step(a.k, (double)B[q].x));
      (vb4 + c * Q + q)[yo] = o;
    }
  };
  Rec r0 = restart(nch - 1), r1;
  fetch(nch - 1, b0);
  for (int c = nch - 1; c >= 1; c -= 2) {
    step_c(c, r0, b0, r1, b1);
    step_c(c - 1, r1, b1, r0, b0);
  }
}

template <int C>
__global__ __launch_bounds__(256) void rec_contract_kernel(RecArgs a) {
  constexpr int P = C + 1;
  for (int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pix < a.N;
       pix += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(pix / a.W), x = (int)(pix - (int64_t)y * a.W);
    const float *__restrict__ zp = a.V + (int64_t)y * a.ld + x;
    const float *__restrict__ up = a.u + pix;
    double e = 0.0, z[C];
#pragma unroll
    for (int c = 0; c < C; ++c) z[c] = 0.0;
    for (int k = 0; k < a.r_eff; ++k) {
      const double uk = (double)up[(int64_t)k * a.N];
      const float *zk = zp + (int64_t)k * P * a.plane;
      e = fma(uk, (double)zk[0], e);
#pragma unroll
      for (int c = 0; c < C; ++c) z[c] = fma(uk, (double)zk[(int64_t)(c + 1) * a.plane], z[c]);
    }
    const bool ok = e > 0.0 && isfinite(e);
#pragma unroll
    for (int c = 0; c < C; ++c)
      a.out[pix * C + c] = ok ? (float)(z[c] / e + (double)a.f0[c]) : a.f[pix * C + c];
    if (a.eta_out) a.eta_out[pix] = (float)e;
  }
}

// Backward, from the forward's filtered planes Z_kp (E_k = Z_k0):
// du_dir_k = beta E_k + sum_c a_c Z_k(c+1).
template <int C>
__global__ __launch_bounds__(256) void rec_dudir_kernel(RecArgs a) {
  constexpr int P = C + 1;
  for (int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pix < a.N;
       pix += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(pix / a.W), x = (int)(pix - (int64_t)y * a.W);
    const float *__restrict__ zp = a.V + (int64_t)y * a.ld + x;
    const float4 co = reinterpret_cast<const float4 *>(a.ab)[pix];
    const double cf[4] = {co.x, co.y, co.z, co.w};
    for (int k = 0; k < a.r_eff; ++k) {
      const float *zk = zp + (int64_t)k * P * a.plane;
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < P; ++q) v = fma(cf[q], (double)zk[(int64_t)q * a.plane], v);
      a.dud[(int64_t)k * a.N + pix] = (float)v;
    }
  }
}

// Backward, from the planes Y_kp filtered again with inputs beta u_k and a_c u_k:
// du_k = du_dir_k + Y_k0 + sum_c f~_c Y_k(c+1),  df_c = sum_k u_k Y_k(c+1)
// (plus dL/dg itself where the forward took the eta <= 0 guard).
template <int C>
__global__ __launch_bounds__(256) void rec_bwd_contract_kernel(RecArgs a) {
  constexpr int P = C + 1;
  for (int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pix < a.N;
       pix += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(pix / a.W), x = (int)(pix - (int64_t)y * a.W);
    const float *__restrict__ zp = a.V + (int64_t)y * a.ld + x;
    double ft[C], d[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      ft[c] = (double)a.f[pix * C + c] - (double)a.f0[c];
      d[c] = 0.0;
    }
    for (int k = 0; k < a.r_eff; ++k) {
      const float *zk = zp + (int64_t)k * P * a.plane;
      const double uk = (double)a.u[(int64_t)k * a.N + pix];
      double v = (double)a.dud[(int64_t)k * a.N + pix] + (double)zk[0];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const double yc = (double)zk[(int64_t)(c + 1) * a.plane];
        v = fma(ft[c], yc, v);
        d[c] = fma(uk, yc, d[c]);
      }
      a.du[(int64_t)k * a.N + pix] = (float)v;
    }
    const float e = a.eta[pix];
    const bool guard = !(e > 0.0f && isfinite(e));
#pragma unroll
    for (int c = 0; c < C; ++c) a.df[pix * C + c] = (float)d[c] + (guard ? a.G[pix * C + c] : 0.0f);
  }
}

// a whole number of chunk pairs per row
int padded_width(int W) { return (W + 2 * kCL - 1) / (2 * kCL) * (2 * kCL); }

size_t plane_floats(int H, int W, int C, int r_eff) { return (size_t)r_eff * (C + 1) * H * (padded_width(W) + 32); }

size_t carry_doubles(int H, int W, int C, int r_eff) {
  const size_t lines_c = (size_t)r_eff * (C + 1) * padded_width(W), lines_r = (size_t)r_eff * (C + 1) * H;
  const size_t nc = 3 * lines_c * ((H + kRL - 1) / kRL), nr = 3 * lines_r * (padded_width(W) / kCL);
  return nc > nr ? nc : nr;
}

}  // namespace

bool rec_coefficients(double sigma_s, RecCoef *c) {
  if (!(sigma_s >= kRecSigmaMin && sigma_s <= kRecSigmaMax)) return false;
  // Young and van Vliet's scale q for sigma and their b0..b3 polynomials
  const double q = sigma_s >= 2.5 ? 0.98711 * sigma_s - 0.96330
                                  : 3.97156 - 4.14554 * sqrt(1.0 - 0.26891 * sigma_s);
  const double b0 = 1.57825 + q * (2.44413 + q * (1.4281 + q * 0.422205));
  const double b1 = q * (2.44413 + q * (2.85619 + q * 1.26661));
  const double b2 = -q * q * (1.4281 + q * 1.26661);
  const double b3 = 0.422205 * q * q * q;
  const double a1 = b1 / b0, a2 = b2 / b0, a3 = b3 / b0, B = 1.0 - a1 - a2 - a3;
  // h[0..3] of the cascade: forward then backward over an impulse in the
  // middle of a zero line long enough for the response to vanish in FP64
  // (the slowest mode decays by at least exp(-1 / sigma) per sample)
  const int L = 64 + (int)ceil(60.0 * sigma_s);
  const int n = 2 * L + 1;
  std::vector<double> w(n + 3, 0.0), y(n + 3, 0.0);
  for (int i = 0; i < n; ++i) {
    const double xi = i == L ? 1.0 : 0.0;
    w[i + 3] = B * xi + a1 * w[i + 2] + a2 * w[i + 1] + a3 * w[i];
  }
  for (int i = n - 1; i >= 0; --i) y[i] = B * w[i + 3] + a1 * y[i + 1] + a2 * y[i + 2] + a3 * y[i + 3];
  const double h0 = y[L], h1 = y[L + 1], h2 = y[L + 2], h3 = y[L + 3];
  c->a1 = a1;
  c->a2 = a2;
  c->a3 = a3;
  c->n0 = 0.5 * h0;
  c->n1 = h1 - a1 * c->n0;
  c->n2 = h2 - a1 * h1 - a2 * c->n0;
  c->n3 = h3 - a1 * h2 - a2 * h1 - a3 * c->n0;
  return true;
}

size_t rec_plane_floats(int H, int W, int C, int r_eff) {
  // the planes, the carries, f as channel planes (each 256-byte aligned)
  const size_t pf = (plane_floats(H, W, C, r_eff) + 63) / 64 * 64;
  const size_t cf = (2 * carry_doubles(H, W, C, r_eff) + 63) / 64 * 64;
  return pf + cf + (size_t)(C + 1) * H * W;  // the backward's C + 1 coefficient planes
}

namespace {

RecArgs rec_args(const RecProblem &pb) {
  RecArgs a{};
  a.H = pb.H;
  a.W = pb.W;
  a.Wp = padded_width(pb.W);
  a.C = pb.C;
  a.r_eff = pb.r_eff;
  a.N = (int64_t)pb.H * pb.W;
  a.ld = a.Wp + 32;
  a.plane = (int64_t)pb.H * a.ld;
  a.f = pb.f;
  a.f0 = pb.f0;
  a.u = pb.u;
  a.V = pb.planes;
  const size_t pf = (plane_floats(pb.H, pb.W, pb.C, pb.r_eff) + 63) / 64 * 64;
  const size_t cf = (2 * carry_doubles(pb.H, pb.W, pb.C, pb.r_eff) + 63) / 64 * 64;
  a.carry = reinterpret_cast<double *>(pb.planes + pf);
  a.fpl = pb.planes + pf + cf;
  a.out = pb.out;
  a.eta_out = pb.eta_out;
  a.k = pb.coef;
  a.G = pb.G;
  a.eta = pb.eta;
  a.ab = pb.ab;
  a.dud = pb.dud;
  a.du = pb.du;
  a.df = pb.df;
  return a;
}

unsigned grid_of(int64_t n, int64_t per_block, int64_t cap) {
  const int64_t b = (n + per_block - 1) / per_block;
  return (unsigned)(b < cap ? b : cap);
}

// the column and row passes over the planes whose inputs the column pass forms
void rec_filter(const RecArgs &a, hipStream_t s) {
  const int P = a.C + 1;
  hipLaunchKernelGGL(rec_cols_kernel, dim3((a.Wp + 63) / 64, (a.r_eff + kColK - 1) / kColK), dim3(64 * P * kColK),
                     0, s, a);
  hipLaunchKernelGGL(rec_rows_kernel, dim3((a.H + 63) / 64, a.r_eff), dim3(64 * P), 0, s, a);
}

}  // namespace

hipError_t launch_rec(const RecProblem &pb, hipStream_t s) {
  if (pb.C < 1 || pb.C > 3 || pb.r_eff < 1) return hipErrorInvalidValue;
  RecArgs a = rec_args(pb);
  hipLaunchKernelGGL(planar_kernel, dim3(grid_of(a.N * pb.C, 512, 4096)), dim3(512), 0, s, a);
  rec_filter(a, s);
  const dim3 g(grid_of(a.N, 256, 8192));
  switch (pb.C) {
    case 1: hipLaunchKernelGGL(rec_contract_kernel<1>, g, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(rec_contract_kernel<2>, g, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(rec_contract_kernel<3>, g, dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_rec_bwd(const RecProblem &pb, hipStream_t s) {
  if (pb.C < 1 || pb.C > 3 || pb.r_eff < 1 || !pb.G || !pb.eta || !pb.ab || !pb.dud || !pb.du || !pb.df)
    return hipErrorInvalidValue;
  RecArgs a = rec_args(pb);
  const dim3 g(grid_of(a.N, 256, 8192));
  // du_dir from the forward's planes, still in the plane buffer
  switch (pb.C) {
    case 1: hipLaunchKernelGGL(rec_dudir_kernel<1>, g, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(rec_dudir_kernel<2>, g, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(rec_dudir_kernel<3>, g, dim3(256), 0, s, a); break;
  }
  // the filter is symmetric (zero-extended convolution with an even
  // response), so the adjoint's planes go through the same passes
  a.bwd = 1;
  hipLaunchKernelGGL(planar_ab_kernel, dim3(grid_of(a.N * (pb.C + 1), 512, 4096)), dim3(512), 0, s, a);
  rec_filter(a, s);
  switch (pb.C) {
    case 1: hipLaunchKernelGGL(rec_bwd_contract_kernel<1>, g, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(rec_bwd_contract_kernel<2>, g, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(rec_bwd_contract_kernel<3>, g, dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace nkf
