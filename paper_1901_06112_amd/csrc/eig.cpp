// Host FP64 symmetric eigensolver for the landmark Gram matrix A (Eq. (eigA)).
//
// Method (Golub & Van Loan, "Matrix Computations", Sections 8.3.1-8.3.3):
// Householder reduction A = Q T Q^T to tridiagonal form, then implicit
// symmetric QR steps with the Wilkinson shift on the unreduced blocks of T
// (kept as its diagonal and off-diagonal), accumulating every reflection and
// rotation into Q.  Cost O(n^3) with a small constant, n <= 256.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

namespace nkf {

namespace {

inline double sgn(double x) { return x < 0.0 ? -1.0 : 1.0; }

}  // namespace

namespace {

int sym_eig_impl(int n, const double *A, double *w, double *V) {
  std::vector<double> T(A, A + (size_t)n * n), Q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  // symmetrise (guards against a caller's round-off asymmetry)
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double m = 0.5 * (T[i * n + j] + T[j * n + i]);
      T[i * n + j] = T[j * n + i] = m;
    }

  // ---- Householder tridiagonalisation -------------------------------------
  std::vector<double> v(n), p(n), q(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of x = T[k+1:, k]
    double sigma = 0.0;
    for (int i = 1; i < m; ++i) sigma += T[(k + 1 + i) * n + k] * T[(k + 1 + i) * n + k];
    const double x0 = T[(k + 1) * n + k];
    if (sigma == 0.0) continue;  // already tridiagonal in this column
    const double mu = sqrt(x0 * x0 + sigma);
    // v = x + sign(x0) |x| e1, beta = 2 / v^T v; H x = -sign(x0) |x| e1
    v[0] = x0 + sgn(x0) * mu;
    for (int i = 1; i < m; ++i) v[i] = T[(k + 1 + i) * n + k];
    double vtv = v[0] * v[0] + sigma;
    const double beta = 2.0 / vtv;
    // p = beta * T' v on the trailing block T' = T[k+1:, k+1:]
    for (int i = 0; i < m; ++i) {
      double acc = 0.0;
      const double *row = &T[(k + 1 + i) * n + (k + 1)];
      for (int j = 0; j < m; ++j) acc += row[j] * v[j];
      p[i] = beta * acc;
    }
    double ptv = 0.0;
    for (int i = 0; i < m; ++i) ptv += p[i] * v[i];
    const double kk = 0.5 * beta * ptv;
    for (int i = 0; i < m; ++i) q[i] = p[i] - kk * v[i];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j)
        T[(k + 1 + i) * n + (k + 1 + j)] -= v[i] * q[j] + q[i] * v[j];
    const double newx = -sgn(x0) * mu;
    T[(k + 1) * n + k] = T[k * n + k + 1] = newx;
    for (int i = 1; i < m; ++i) T[(k + 1 + i) * n + k] = T[k * n + k + 1 + i] = 0.0;
    // Q <- Q H on columns k+1..n-1
    for (int i = 0; i < n; ++i) {
      double acc = 0.0;
      const double *row = &Q[i * n + (k + 1)];
      for (int j = 0; j < m; ++j) acc += row[j] * v[j];
      acc *= beta;
      double *roww = &Q[i * n + (k + 1)];
      for (int j = 0; j < m; ++j) roww[j] -= acc * v[j];
    }
  }
  // ---- implicit symmetric QR with Wilkinson shift on the band -------------
  // d: diagonal, e[i]: entry (i+1, i); the eigenvector estimates are the rows
  // of Z = Q^T, so that a rotation in the (k, k+1) plane updates two
  // contiguous rows.
  std::vector<double> d(n), e(n, 0.0), Z((size_t)n * n);
  for (int i = 0; i < n; ++i) {
    d[i] = T[i * n + i];
    if (i + 1 < n) e[i] = T[(i + 1) * n + i];
    for (int j = 0; j < n; ++j) Z[(size_t)i * n + j] = Q[(size_t)j * n + i];
  }
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
      const double rr = hypot(x, z);
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
      // Q <- Q G^T, i.e. rows k, k+1 of Z
      double *zk = &Z[(size_t)k * n], *zk1 = &Z[(size_t)(k + 1) * n];
      for (int i = 0; i < n; ++i) {
        const double a = zk[i], bb = zk1[i];
        zk[i] = c * a + s * bb;
        zk1[i] = -s * a + c * bb;
      }
      if (k + 1 < hi) {
        x = e[k];
        z = bulge;
      }
    }
  }

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

}  // namespace nkf
