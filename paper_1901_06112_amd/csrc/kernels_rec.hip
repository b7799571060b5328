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
//   y+[n] = n0 x[n] + n1 x[n-1] + n2 x[n-2] + n3 x[n-3]
//           + a1 y+[n-1] + a2 y+[n-2] + a3 y+[n-3]
// with n0..n3 fitted to h[0]/2, h[1], h[2], h[3]; y- runs the same recursion
// from the other end.  Both start from rest at the line ends, which is exactly
// the zero extension.  Each sweep reads only the input: a pass stores the
// first sweep's result and the second sweep adds its own.
//
// For embedding plane u_k, the planes are u_k f~_c (f~ = f - f0) and u_k
// itself (plane 0); every recursion runs in FP64, the filtered planes are
// stored as FP32 between passes.
//   columns   block (64 columns, k), wave = plane: each lane sweeps down and
//             then up its column, forming the plane's input from u_k and f
//             on the fly; V_kp = column-filtered planes;
//   rows      block (64 rows, k), wave = plane: each lane sweeps right and
//             then left along its row of V_kp, 16 columns per batch of four
//             16-byte loads; Z_kp = filtered planes;
//   contract  thread per pixel: eta = sum_k u_k Z_k0 and zeta_c =
//             sum_k u_k Z_k(c+1) in FP64, g = zeta / eta + f0 (f where eta
//             <= 0 or not finite).
// Rows of V and Z are padded to Wp = W rounded up to 16 columns; the padding
// columns of V hold zeros (the zero extension), those of Z are never read.
// Every sweep prefetches its next batch of rows or columns while it computes
// the current one.
#include <hip/hip_runtime.h>
#include <math.h>

#include <vector>

#include "device_common.h"
#include "nkf_internal.h"

namespace nkf {

namespace {

constexpr int kRB = 16;   // rows per batch of the column sweeps
constexpr int kCB = 16;   // columns per batch of the row sweeps (four float4)

struct RecArgs {
  int H, W, Wp, C, r_eff;
  int64_t N, plane;        // pixels; floats per stored plane (H * Wp)
  const float *f, *f0, *u;
  float *V, *Z;
  float *out, *eta_out;
  RecCoef k;
};

// One step of the causal recursion; x1..x3 and y1..y3 hold the last three
// inputs and outputs.
struct Rec {
  double x1 = 0, x2 = 0, x3 = 0, y1 = 0, y2 = 0, y3 = 0;
  __device__ double step(const RecCoef &c, double x) {
    const double part = fma(c.n0, x, fma(c.n1, x1, fma(c.n2, x2, fma(c.n3, x3, fma(c.a3, y3, c.a2 * y2)))));
    const double y = fma(c.a1, y1, part);
    x3 = x2;
    x2 = x1;
    x1 = x;
    y3 = y2;
    y2 = y1;
    y1 = y;
    return y;
  }
};

__global__ __launch_bounds__(256) void rec_cols_kernel(RecArgs a) {
  const int p = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // 0: u_k, c + 1: u_k f~_c
  const int k = blockIdx.y;
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  if (x >= a.Wp) return;
  const bool valid = x < a.W;
  const int xc = valid ? x : a.W - 1;  // in-bounds address; the value is dropped when !valid
  const float *__restrict__ up = a.u + (int64_t)k * a.N + xc;
  const float *__restrict__ fp = a.f + (int64_t)xc * a.C + (p > 0 ? p - 1 : 0);
  const double f0 = p > 0 ? (double)a.f0[p - 1] : 0.0;
  float *__restrict__ vp = a.V + ((int64_t)k * (a.C + 1) + p) * a.plane + x;
  const int H = a.H, Wp = a.Wp;
  const int64_t us = a.W, fs = (int64_t)a.W * a.C;
  auto input = [&](float uv, float fv) -> double {
    const double uu = valid ? (double)uv : 0.0;
    return p > 0 ? uu * ((double)fv - f0) : uu;
  };
  const int nb = H / kRB;
  float cu[kRB], cf[kRB], nu[kRB], nf[kRB], cv[kRB], nv[kRB];
  // ---- down: y+ stored in V
  {
    auto load = [&](int y0, float (&U)[kRB], float (&F)[kRB]) {
#pragma unroll
      for (int j = 0; j < kRB; ++j) {
        U[j] = up[(int64_t)(y0 + j) * us];
        F[j] = p > 0 ? fp[(int64_t)(y0 + j) * fs] : 0.0f;
      }
    };
    Rec r;
    if (nb > 0) load(0, cu, cf);
    for (int b = 0; b < nb; ++b) {
      if (b + 1 < nb) load((b + 1) * kRB, nu, nf);
#pragma unroll
      for (int j = 0; j < kRB; ++j) vp[(int64_t)(b * kRB + j) * Wp] = (float)r.step(a.k, input(cu[j], cf[j]));
#pragma unroll
      for (int j = 0; j < kRB; ++j) {
        cu[j] = nu[j];
        cf[j] = nf[j];
      }
    }
    for (int y = nb * kRB; y < H; ++y)
      vp[(int64_t)y * Wp] = (float)r.step(a.k, input(up[(int64_t)y * us], p > 0 ? fp[(int64_t)y * fs] : 0.0f));
  }
  // ---- up: V = y+ + y-
  {
    auto load = [&](int i0, float (&U)[kRB], float (&F)[kRB], float (&Vv)[kRB]) {
#pragma unroll
      for (int j = 0; j < kRB; ++j) {
        const int64_t y = H - 1 - (i0 + j);
        U[j] = up[y * us];
        F[j] = p > 0 ? fp[y * fs] : 0.0f;
        Vv[j] = vp[y * Wp];
      }
    };
    Rec r;
    if (nb > 0) load(0, cu, cf, cv);
    for (int b = 0; b < nb; ++b) {
      if (b + 1 < nb) load((b + 1) * kRB, nu, nf, nv);
#pragma unroll
      for (int j = 0; j < kRB; ++j) {
        const int64_t y = H - 1 - (b * kRB + j);
        vp[y * Wp] = (float)((double)cv[j] + r.step(a.k, input(cu[j], cf[j])));
      }
#pragma unroll
      for (int j = 0; j < kRB; ++j) {
        cu[j] = nu[j];
        cf[j] = nf[j];
        cv[j] = nv[j];
      }
    }
    for (int i = nb * kRB; i < H; ++i) {
      const int64_t y = H - 1 - i;
      const double yv = r.step(a.k, input(up[y * us], p > 0 ? fp[y * fs] : 0.0f));
      vp[y * Wp] = (float)((double)vp[y * Wp] + yv);
    }
  }
}

__global__ __launch_bounds__(256) void rec_rows_kernel(RecArgs a) {
  const int p = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int k = blockIdx.y;
  const int y = blockIdx.x * 64 + (threadIdx.x & 63);
  if (y >= a.H) return;
  const int64_t row = ((int64_t)k * (a.C + 1) + p) * a.plane + (int64_t)y * a.Wp;
  const float4 *__restrict__ vr = reinterpret_cast<const float4 *>(a.V + row);
  float4 *__restrict__ zr = reinterpret_cast<float4 *>(a.Z + row);
  constexpr int Q = kCB / 4;
  const int nb = a.Wp / kCB;
  float4 cur[Q], nxt[Q], cz[Q], nz[Q];
  // ---- right: y+ stored in Z
  {
    Rec r;
#pragma unroll
    for (int q = 0; q < Q; ++q) cur[q] = vr[q];
    for (int b = 0; b < nb; ++b) {
      if (b + 1 < nb) {
#pragma unroll
        for (int q = 0; q < Q; ++q) nxt[q] = vr[(b + 1) * Q + q];
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        float4 o;
        o.x = (float)r.step(a.k, (double)cur[q].x);
        o.y = (float)r.step(a.k, (double)cur[q].y);
        o.z = (float)r.step(a.k, (double)cur[q].z);
        o.w = (float)r.step(a.k, (double)cur[q].w);
        zr[b * Q + q] = o;
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) cur[q] = nxt[q];
    }
  }
  // ---- left: Z = y+ + y-
  {
    Rec r;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      cur[q] = vr[(nb - 1) * Q + q];
      cz[q] = zr[(nb - 1) * Q + q];
    }
    for (int b = nb - 1; b >= 0; --b) {
      if (b > 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          nxt[q] = vr[(b - 1) * Q + q];
          nz[q] = zr[(b - 1) * Q + q];
        }
      }
#pragma unroll
      for (int q = Q - 1; q >= 0; --q) {
        float4 o;
        o.w = (float)((double)cz[q].w + r.step(a.k, (double)cur[q].w));
        o.z = (float)((double)cz[q].z + r.step(a.k, (double)cur[q].z));
        o.y = (float)((double)cz[q].y + r.step(a.k, (double)cur[q].y));
        o.x = (float)((double)cz[q].x + r.step(a.k, (double)cur[q].x));
        zr[b * Q + q] = o;
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        cur[q] = nxt[q];
        cz[q] = nz[q];
      }
    }
  }
}

template <int C>
__global__ __launch_bounds__(256) void rec_contract_kernel(RecArgs a) {
  constexpr int P = C + 1;
  for (int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pix < a.N;
       pix += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(pix / a.W), x = (int)(pix - (int64_t)y * a.W);
    const float *__restrict__ zp = a.Z + (int64_t)y * a.Wp + x;
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

int padded_width(int W) { return (W + kCB - 1) / kCB * kCB; }

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
  return 2 * (size_t)r_eff * (C + 1) * H * padded_width(W);
}

hipError_t launch_rec(const RecProblem &pb, hipStream_t s) {
  if (pb.C < 1 || pb.C > 3 || pb.r_eff < 1) return hipErrorInvalidValue;
  RecArgs a{};
  a.H = pb.H;
  a.W = pb.W;
  a.Wp = padded_width(pb.W);
  a.C = pb.C;
  a.r_eff = pb.r_eff;
  a.N = (int64_t)pb.H * pb.W;
  a.plane = (int64_t)pb.H * a.Wp;
  a.f = pb.f;
  a.f0 = pb.f0;
  a.u = pb.u;
  a.V = pb.planes;
  a.Z = pb.planes + (size_t)pb.r_eff * (pb.C + 1) * a.plane;
  a.out = pb.out;
  a.eta_out = pb.eta_out;
  a.k = pb.coef;
  const int P = pb.C + 1;
  hipLaunchKernelGGL(rec_cols_kernel, dim3((a.Wp + 63) / 64, pb.r_eff), dim3(64 * P), 0, s, a);
  hipLaunchKernelGGL(rec_rows_kernel, dim3((pb.H + 63) / 64, pb.r_eff), dim3(64 * P), 0, s, a);
  const int64_t nblk = (a.N + 255) / 256;
  const dim3 g((unsigned)(nblk < 8192 ? nblk : 8192));
  switch (pb.C) {
    case 1: hipLaunchKernelGGL(rec_contract_kernel<1>, g, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(rec_contract_kernel<2>, g, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(rec_contract_kernel<3>, g, dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace nkf
