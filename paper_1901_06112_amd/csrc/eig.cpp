// Host FP64 symmetric eigensolver for the landmark Gram matrix A (Eq. (eigA)).
//
// Method (Golub & Van Loan, "Matrix Computations", Sections 8.3.1-8.3.3):
// Householder reduction A = Q T Q^T to tridiagonal form, then implicit
// symmetric QR steps with the Wilkinson shift on the unreduced blocks of T,
// accumulating every reflection and rotation into Q.  Cost O(n^3) with a small
// constant, n <= 256.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

namespace nkf {

namespace {

inline double sgn(double x) { return x < 0.0 ? -1.0 : 1.0; }

// Rotation in the (k, k+1) plane, G = [[c, s], [-s, c]]: T <- G T G^T on the
// band rows/columns [lo, hi), Q <- Q G^T on all rows.
void rotate(int n, std::vector<double> &T, std::vector<double> &Q, int k, double c, double s) {
  const int lo = std::max(0, k - 1), hi = std::min(n, k + 3);
  for (int j = lo; j < hi; ++j) {  // rows k, k+1
    const double a = T[k * n + j], b = T[(k + 1) * n + j];
    T[k * n + j] = c * a + s * b;
    T[(k + 1) * n + j] = -s * a + c * b;
  }
  for (int i = lo; i < hi; ++i) {  // columns k, k+1
    const double a = T[i * n + k], b = T[i * n + k + 1];
    T[i * n + k] = c * a + s * b;
    T[i * n + k + 1] = -s * a + c * b;
  }
  for (int i = 0; i < n; ++i) {
    const double a = Q[i * n + k], b = Q[i * n + k + 1];
    Q[i * n + k] = c * a + s * b;
    Q[i * n + k + 1] = -s * a + c * b;
  }
}

}  // namespace

// A: n x n row-major symmetric.  On success w[0..n) ascending and V (row-major
// n x n) holds the matching eigenvectors as columns.  Returns 0, or -1 if the
// QR iteration did not converge.
int sym_eig(int n, const double *A, double *w, double *V) {
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
  // exact zeros outside the band
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (j < i - 1 || j > i + 1) T[i * n + j] = 0.0;

  // ---- implicit symmetric QR with Wilkinson shift -------------------------
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int iter = 0;
  const int max_iter = 60 * n + 100;
  while (hi > 0) {
    // deflate negligible off-diagonals
    for (int i = 1; i <= hi; ++i) {
      const double off = fabs(T[i * n + i - 1]);
      if (off <= eps * (fabs(T[i * n + i]) + fabs(T[(i - 1) * n + i - 1])) || off < 1e-300)
        T[i * n + i - 1] = T[(i - 1) * n + i] = 0.0;
    }
    if (T[hi * n + hi - 1] == 0.0) {
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && T[lo * n + lo - 1] != 0.0) --lo;
    if (++iter > max_iter) return -1;
    // Wilkinson shift from the trailing 2x2 of the block
    const double a = T[(hi - 1) * n + hi - 1], b = T[hi * n + hi - 1], c = T[hi * n + hi];
    const double d = 0.5 * (a - c);
    const double shift = c - b * b / (d + sgn(d) * hypot(d, b));
    double x = T[lo * n + lo] - shift;
    double z = T[(lo + 1) * n + lo];
    for (int k = lo; k < hi; ++k) {
      const double rr = hypot(x, z);
      double cs = 1.0, sn = 0.0;
      if (rr != 0.0) {
        cs = x / rr;
        sn = z / rr;
      }
      rotate(n, T, Q, k, cs, sn);
      if (k > lo) T[(k + 1) * n + k - 1] = T[(k - 1) * n + k + 1] = 0.0;  // bulge chased out
      if (k + 1 < hi) {
        x = T[(k + 1) * n + k];
        z = T[(k + 2) * n + k];
      }
    }
  }

  // ---- sort ascending -------------------------------------------------------
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int i, int j) { return T[i * n + i] < T[j * n + j]; });
  for (int j = 0; j < n; ++j) {
    w[j] = T[ord[j] * n + ord[j]];
    for (int i = 0; i < n; ++i) V[i * n + j] = Q[i * n + ord[j]];
  }
  return 0;
}

}  // namespace nkf
