// Host FP64 symmetric eigensolver for the landmark Gram matrix A (Eq. (eigA)).
//
// Method (Golub & Van Loan, "Matrix Computations", Sections 8.3.1-8.3.3):
// Householder reduction A = Q T Q^T to tridiagonal form (updating the lower
// triangle only, the reflectors kept), then implicit symmetric QR steps with
// the Wilkinson shift on the unreduced blocks of T (kept as its diagonal and
// off-diagonal), the rotations recorded; the eigenvectors are the reflections
// and rotations applied to the identity, by column blocks on up to 8 threads
// (the columns are independent).  Cost O(n^3) with a small constant, n <= 256.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <thread>
#include <utility>
#include <vector>

namespace nkf {

namespace {

inline double sgn(double x) { return x < 0.0 ? -1.0 : 1.0; }

// a . b over n entries in four partial sums (a single running sum is a chain
// of dependent FMAs, bound by their latency)
inline double dot4(const double *a, const double *b, int n) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int i = 0;
  for (; i + 4 <= n; i += 4)
    for (int u = 0; u < 4; ++u) s[u] += a[i + u] * b[i + u];
  for (; i < n; ++i) s[0] += a[i] * b[i];
  return (s[0] + s[1]) + (s[2] + s[3]);
}

}  // namespace

namespace {

// Threads for the eigenvector stage: from n = 96 on, up to 8, one column
// block of at least 16 columns each (below, thread start-up costs more than
// the work).
int vec_threads(int n) {
  if (n < 96) return 1;
  const unsigned hc = std::thread::hardware_concurrency();
  int t = std::min(8, n / 16);
  if (hc > 0) t = std::min(t, (int)hc);
  return std::max(1, t);
}

int sym_eig_impl(int n, const double *A, double *w, double *V) {
  std::vector<double> T(A, A + (size_t)n * n);
  // symmetrise (guards against a caller's round-off asymmetry)
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double m = 0.5 * (T[i * n + j] + T[j * n + i]);
      T[i * n + j] = T[j * n + i] = m;
    }

  // ---- Householder tridiagonalisation (lower triangle) ---------------------
  // reflector k acts on entries k+1 .. n-1: H_k = I - beta_k v v^T, v kept in
  // R[k][0 .. n-k-2]; Q = H_0 H_1 ... H_{n-3} is not formed here
  std::vector<double> R((size_t)n * n, 0.0), betas(n, 0.0);
  std::vector<double> p(n), q(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of x = T[k+1:, k]
    double *v = &R[(size_t)k * n];
    double sigma = 0.0;
    for (int i = 1; i < m; ++i) sigma += T[(k + 1 + i) * n + k] * T[(k + 1 + i) * n + k];
    const double x0 = T[(k + 1) * n + k];
    if (sigma == 0.0) continue;  // already tridiagonal in this column
    const double mu = sqrt(x0 * x0 + sigma);
    // v = x + sign(x0) |x| e1, beta = 2 / v^T v; H x = -sign(x0) |x| e1
    v[0] = x0 + sgn(x0) * mu;
    for (int i = 1; i < m; ++i) v[i] = T[(k + 1 + i) * n + k];
    const double beta = 2.0 / (v[0] * v[0] + sigma);
    betas[k] = beta;
    // p = beta * T' v on the trailing block T' = T[k+1:, k+1:], of which only
    // the lower triangle is kept (rows j <= i and their transposes)
    for (int i = 0; i < m; ++i) p[i] = 0.0;
    for (int i = 0; i < m; ++i) {
      const double *row = &T[(k + 1 + i) * n + (k + 1)];
      const double vi = v[i];
      double a4[4] = {0.0, 0.0, 0.0, 0.0};  // the row's dot product in four partial sums (dot4)
      int j = 0;
      for (; j + 4 <= i; j += 4)
        for (int u = 0; u < 4; ++u) {
          a4[u] += row[j + u] * v[j + u];
          p[j + u] += row[j + u] * vi;
        }
      for (; j < i; ++j) {
        a4[0] += row[j] * v[j];
        p[j] += row[j] * vi;
      }
      p[i] += ((a4[0] + a4[1]) + (a4[2] + a4[3])) + row[i] * vi;
    }
    for (int i = 0; i < m; ++i) p[i] *= beta;
    double ptv = 0.0;
    for (int i = 0; i < m; ++i) ptv += p[i] * v[i];
    const double kk = 0.5 * beta * ptv;
    for (int i = 0; i < m; ++i) q[i] = p[i] - kk * v[i];
    for (int i = 0; i < m; ++i) {
      double *row = &T[(k + 1 + i) * n + (k + 1)];
      const double vi = v[i], qi = q[i];
      for (int j = 0; j <= i; ++j) row[j] -= vi * q[j] + qi * v[j];
    }
    T[(k + 1) * n + k] = -sgn(x0) * mu;
    for (int i = 1; i < m; ++i) T[(k + 1 + i) * n + k] = 0.0;
  }

  // ---- implicit symmetric QR with Wilkinson shift on the band -------------
  // d: diagonal, e[i]: entry (i+1, i).  The rotations act on (d, e) here and
  // are recorded; the eigenvector estimates, the rows of Z = G ... G Q^T, are
  // formed below.
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) {
    d[i] = T[i * n + i];
    if (i + 1 < n) e[i] = T[(i + 1) * n + i];
  }
  struct Rot {
    int k;
    double c, s;
  };
  std::vector<Rot> rots;
  rots.reserve((size_t)2 * n * n);
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int iter = 0;
  const int max_iter = 60 * n + 100;
  while (hi > 0) {
    // deflate negligible off-diagonals of the active part
    for (int i = 0; i < hi; ++i)
      if (fabs(e[i]) <= eps * (fabs(d[i]) + fabs(d[i + 1])) || fabs(e[i]) < 1e-300) e[i] = 0.0;
    if (e[hi - 1] == 0.0) {
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    if (++iter > max_iter) return -1;
    // Wilkinson shift: eigenvalue of the trailing 2x2 closer to d[hi]
    const double dd = 0.5 * (d[hi - 1] - d[hi]), b2 = e[hi - 1];
    const double shift = d[hi] - b2 * b2 / (dd + sgn(dd) * hypot(dd, b2));
    double x = d[lo] - shift, z = e[lo];
    double bulge = 0.0;
    for (int k = lo; k < hi; ++k) {
      // rotation G = [[c, s], [-s, c]] in the (k, k+1) plane with G (x, z)^T = (r, 0)^T
      const double s2 = x * x + z * z;
      const double rr = s2 > 1e-290 && s2 < 1e290 ? sqrt(s2) : hypot(x, z);
      double c = 1.0, s = 0.0;
      if (rr != 0.0) {
        c = x / rr;
        s = z / rr;
      }
      if (k > lo) e[k - 1] = rr;  // the bulge at (k-1, k+1) is chased out
      // T <- G T G^T on the 2x2 block and its neighbours
      const double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = c * c * dk + 2.0 * c * s * ek + s * s * dk1;
      d[k + 1] = s * s * dk - 2.0 * c * s * ek + c * c * dk1;
      e[k] = c * s * (dk1 - dk) + (c * c - s * s) * ek;
      if (k + 1 < hi) {
        bulge = s * e[k + 1];  // new entry (k, k+2)
        e[k + 1] *= c;
      }
      rots.push_back(Rot{k, c, s});
      if (k + 1 < hi) {
        x = e[k];
        z = bulge;
      }
    }
  }

  // ---- eigenvectors: Z = G_last ... G_1 H_{n-3} ... H_0 I ------------------
  // The columns of Z are independent, so each thread takes a block of them
  // (row-major n x JB in its own buffer, in L1/L2 throughout), applies the
  // reflectors in order and then the recorded rotations.
  std::vector<double> Z((size_t)n * n);
  auto vec_block = [&](int j0, int j1) {
    const int JB = j1 - j0;
    std::vector<double> B((size_t)n * JB, 0.0), acc(JB);
    for (int j = 0; j < JB; ++j) B[(size_t)(j0 + j) * JB + j] = 1.0;
    for (int k = 0; k + 2 < n; ++k) {
      const double beta = betas[k];
      if (beta == 0.0) continue;
      const int m = n - k - 1;
      const double *v = &R[(size_t)k * n];
      for (int j = 0; j < JB; ++j) acc[j] = 0.0;
      for (int i = 0; i < m; ++i) {
        const double *row = &B[(size_t)(k + 1 + i) * JB];
        const double vi = v[i];
        for (int j = 0; j < JB; ++j) acc[j] += vi * row[j];
      }
      for (int j = 0; j < JB; ++j) acc[j] *= beta;
      for (int i = 0; i < m; ++i) {
        double *row = &B[(size_t)(k + 1 + i) * JB];
        const double vi = v[i];
        for (int j = 0; j < JB; ++j) row[j] -= vi * acc[j];
      }
    }
    for (const Rot &g : rots) {
      double *zk = &B[(size_t)g.k * JB], *zk1 = &B[(size_t)(g.k + 1) * JB];
      for (int j = 0; j < JB; ++j) {
        const double a = zk[j], bb = zk1[j];
        zk[j] = g.c * a + g.s * bb;
        zk1[j] = -g.s * a + g.c * bb;
      }
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < JB; ++j) Z[(size_t)i * n + j0 + j] = B[(size_t)i * JB + j];
  };
  const int nt = vec_threads(n);
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(vec_block, t * n / nt, (t + 1) * n / nt);
  vec_block(0, n / nt);
  for (auto &th : pool) th.join();

  // ---- sort ascending -------------------------------------------------------
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int i, int j) { return d[i] < d[j]; });
  for (int j = 0; j < n; ++j) {
    w[j] = d[ord[j]];
    for (int i = 0; i < n; ++i) V[i * n + j] = Z[(size_t)ord[j] * n + i];
  }
  return 0;
}

}  // namespace

// A: n x n row-major symmetric.  On success w[0..n) ascending and V (row-major
// n x n) holds the matching eigenvectors as columns.  Returns 0, or -1 if the
// QR iteration did not converge.
int sym_eig(int n, const double *A, double *w, double *V) { return sym_eig_impl(n, A, w, V); }

// The k largest eigenpairs only (Golub & Van Loan, Sections 8.3 and 8.2.2):
// the same Householder reduction on the lower triangle, keeping the
// reflectors instead of forming Q; all eigenvalues of T by the same implicit
// QR steps without rotating vectors (rotation lengths by sqrt away from
// overflow and underflow); the k eigenvectors of T by inverse
// iteration (tridiagonal LU with partial pivoting, three steps from a fixed
// start vector, each orthogonalised against the vectors already found for
// eigenvalues within 1e-3 |T|_1, nearly equal shifts separated by 10 eps |lambda|);
// then the k vectors carried back through the reflectors.  Cost about
// 2/3 n^3 + O(n^2 k) instead of about 6 n^3.  w[0..k) ascending, V row-major
// n x k with the matching columns.  Returns 0, or -1 if the QR iteration did
// not converge.
int sym_eig_top(int n, const double *A, int k, double *w, double *V) {
  if (k < 1 || k > n) return -1;
  std::vector<double> T(A, A + (size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double m = 0.5 * (T[i * n + j] + T[j * n + i]);
      T[i * n + j] = T[j * n + i] = m;
    }
  // reflector kk acts on entries kk+1 .. n-1: H = I - beta v v^T, v stored in
  // R[kk][0 .. n-kk-2]
  std::vector<double> R((size_t)n * n, 0.0), betas(n, 0.0);
  std::vector<double> p(n), q(n);
  for (int kk = 0; kk + 2 < n; ++kk) {
    const int m = n - kk - 1;
    double *v = &R[(size_t)kk * n];
    double sigma = 0.0;
    for (int i = 1; i < m; ++i) sigma += T[(kk + 1 + i) * n + kk] * T[(kk + 1 + i) * n + kk];
    const double x0 = T[(kk + 1) * n + kk];
    if (sigma == 0.0) continue;
    const double mu = sqrt(x0 * x0 + sigma);
    v[0] = x0 + sgn(x0) * mu;
    for (int i = 1; i < m; ++i) v[i] = T[(kk + 1 + i) * n + kk];
    const double beta = 2.0 / (v[0] * v[0] + sigma);
    betas[kk] = beta;
    // only the lower triangle of the trailing block is kept: p = T' v by
    // rows (j <= i) and their transposes
    for (int i = 0; i < m; ++i) p[i] = 0.0;
    for (int i = 0; i < m; ++i) {
      const double *row = &T[(kk + 1 + i) * n + (kk + 1)];
      const double vi = v[i];
      double a4[4] = {0.0, 0.0, 0.0, 0.0};  // the row's dot product in four partial sums (dot4)
      int j = 0;
      for (; j + 4 <= i; j += 4)
        for (int u = 0; u < 4; ++u) {
          a4[u] += row[j + u] * v[j + u];
          p[j + u] += row[j + u] * vi;
        }
      for (; j < i; ++j) {
        a4[0] += row[j] * v[j];
        p[j] += row[j] * vi;
      }
      p[i] += ((a4[0] + a4[1]) + (a4[2] + a4[3])) + row[i] * vi;
    }
    for (int i = 0; i < m; ++i) p[i] *= beta;
    double ptv = 0.0;
    for (int i = 0; i < m; ++i) ptv += p[i] * v[i];
    const double hk = 0.5 * beta * ptv;
    for (int i = 0; i < m; ++i) q[i] = p[i] - hk * v[i];
    for (int i = 0; i < m; ++i) {
      double *row = &T[(kk + 1 + i) * n + (kk + 1)];
      const double vi = v[i], qi = q[i];
      for (int j = 0; j <= i; ++j) row[j] -= vi * q[j] + qi * v[j];
    }
    T[(kk + 1) * n + kk] = -sgn(x0) * mu;
    for (int i = 1; i < m; ++i) T[(kk + 1 + i) * n + kk] = 0.0;
  }
  std::vector<double> d0(n), e0(n, 0.0);
  for (int i = 0; i < n; ++i) {
    d0[i] = T[i * n + i];
    if (i + 1 < n) e0[i] = T[(i + 1) * n + i];
  }
  // eigenvalues: the implicit QR steps of sym_eig on (d, e) alone
  std::vector<double> d(d0), e(e0);
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, iter = 0;
  const int max_iter = 60 * n + 100;
  while (hi > 0) {
    for (int i = 0; i < hi; ++i)
      if (fabs(e[i]) <= eps * (fabs(d[i]) + fabs(d[i + 1])) || fabs(e[i]) < 1e-300) e[i] = 0.0;
    if (e[hi - 1] == 0.0) {
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    if (++iter > max_iter) return -1;
    const double dd = 0.5 * (d[hi - 1] - d[hi]), b2 = e[hi - 1];
    const double shift = d[hi] - b2 * b2 / (dd + sgn(dd) * hypot(dd, b2));
    double x = d[lo] - shift, z = e[lo];
    double bulge = 0.0;
    for (int j = lo; j < hi; ++j) {
      const double s2 = x * x + z * z;
      const double rr = s2 > 1e-290 && s2 < 1e290 ? sqrt(s2) : hypot(x, z);
      double c = 1.0, s = 0.0;
      if (rr != 0.0) {
        c = x / rr;
        s = z / rr;
      }
      if (j > lo) e[j - 1] = rr;
      const double dk = d[j], dk1 = d[j + 1], ek = e[j];
      d[j] = c * c * dk + 2.0 * c * s * ek + s * s * dk1;
      d[j + 1] = s * s * dk - 2.0 * c * s * ek + c * c * dk1;
      e[j] = c * s * (dk1 - dk) + (c * c - s * s) * ek;
      if (j + 1 < hi) {
        bulge = s * e[j + 1];
        e[j + 1] *= c;
        x = e[j];
        z = bulge;
      }
    }
  }
  std::sort(d.begin(), d.end());
  // |T|_1 of the tridiagonal form
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i) {
    double cs = fabs(d0[i]);
    if (i > 0) cs += fabs(e0[i - 1]);
    if (i + 1 < n) cs += fabs(e0[i]);
    tnorm = std::max(tnorm, cs);
  }
  if (tnorm == 0.0) tnorm = 1.0;
  const double ortol = 1e-3 * tnorm, tiny = eps * tnorm;
  std::vector<double> X((size_t)k * n);  // eigenvectors of T, descending eigenvalue order
  std::vector<double> u0(n), u1(n), u2(n), l(n), y(n);
  std::vector<char> piv(n);
  double prev_shift = 0.0;
  int cluster_start = 0;
  for (int j = 0; j < k; ++j) {
    const double lam = d[n - 1 - j];
    double sh = lam;
    if (j > 0) {
      if (fabs(d[n - j] - lam) > ortol) cluster_start = j;
      const double pertol = 10.0 * fabs(lam) * eps;
      if (prev_shift - sh < pertol) sh = prev_shift - pertol;
    }
    prev_shift = sh;
    // LU of T - sh I with partial pivoting: rows of U hold (u0, u1, u2)
    double ca = d0[0] - sh, cb = n > 1 ? e0[0] : 0.0;
    for (int i = 0; i + 1 < n; ++i) {
      const double sub = e0[i], a1 = d0[i + 1] - sh, b1 = i + 2 < n ? e0[i + 1] : 0.0;
      if (fabs(ca) >= fabs(sub)) {
        piv[i] = 0;
        if (ca == 0.0) ca = tiny;
        l[i] = sub / ca;
        u0[i] = ca;
        u1[i] = cb;
        u2[i] = 0.0;
        ca = a1 - l[i] * cb;
        cb = b1;
      } else {
        piv[i] = 1;
        l[i] = ca / sub;
        u0[i] = sub;
        u1[i] = a1;
        u2[i] = b1;
        ca = cb - l[i] * a1;
        cb = -l[i] * b1;
      }
    }
    u0[n - 1] = ca == 0.0 ? tiny : ca;
    double *xv = &X[(size_t)j * n];
    // fixed start vector with entries in (-1, 1)
    uint64_t st = 0x9E3779B97F4A7C15ull * (uint64_t)(j + 1);
    for (int i = 0; i < n; ++i) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      xv[i] = (double)(int64_t)(st >> 11) / 4503599627370496.0 - 1.0;
    }
    for (int it = 0; it < 3; ++it) {
      for (int i = 0; i < n; ++i) y[i] = xv[i];
      for (int i = 0; i + 1 < n; ++i) {
        if (piv[i]) std::swap(y[i], y[i + 1]);
        y[i + 1] -= l[i] * y[i];
      }
      for (int i = n - 1; i >= 0; --i) {
        double t = y[i];
        if (i + 1 < n) t -= u1[i] * xv[i + 1];
        if (i + 2 < n) t -= u2[i] * xv[i + 2];
        xv[i] = t / u0[i];
      }
      // against the vectors of the same cluster, then unit length
      for (int jj = cluster_start; jj < j; ++jj) {
        const double *o = &X[(size_t)jj * n];
        double dot = 0.0;
        for (int i = 0; i < n; ++i) dot += o[i] * xv[i];
        for (int i = 0; i < n; ++i) xv[i] -= dot * o[i];
      }
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += xv[i] * xv[i];
      nrm = sqrt(nrm);
      if (!(nrm > 0.0) || !std::isfinite(nrm)) return -1;
      for (int i = 0; i < n; ++i) xv[i] /= nrm;
    }
  }
  // back through the reflectors (A = Q T Q^T with Q = H_0 H_1 ... H_{n-3}),
  // then ascending order
  for (int j = 0; j < k; ++j) {
    double *xv = &X[(size_t)j * n];
    for (int kk = n - 3; kk >= 0; --kk) {
      if (betas[kk] == 0.0) continue;
      const int m = n - kk - 1;
      const double *v = &R[(size_t)kk * n];
      double dot = dot4(v, xv + kk + 1, m) * betas[kk];
      for (int i = 0; i < m; ++i) xv[kk + 1 + i] -= dot * v[i];
    }
    const int col = k - 1 - j;
    w[col] = d[n - 1 - j];
    for (int i = 0; i < n; ++i) V[(size_t)i * k + col] = xv[i];
  }
  return 0;
}

}  // namespace nkf
