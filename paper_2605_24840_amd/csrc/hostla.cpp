// Small dense linear algebra on the host for the k x k and block-Lanczos
// problems of the driver (never larger than a few hundred): symmetric
// eigen-decomposition by Householder reduction to tridiagonal form followed
// by the implicit QL iteration with shifts, and a Cholesky factorisation.
#include "hostla.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace refl {

int sym_eig_small(int n, const double* A_in, double* w, double* Q_out) {
  if (n <= 0) return 0;
  std::vector<double> A(A_in, A_in + (size_t)n * n);
  // Symmetrise (callers pass matrices that are symmetric up to rounding).
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double v = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
      A[(size_t)i * n + j] = A[(size_t)j * n + i] = v;
    }
  std::vector<double> Q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;

  // Householder: for column c, reflect rows c+1..n-1 so that A[c+2.., c] = 0.
  std::vector<double> v(n), p(n), q(n);
  for (int c = 0; c + 2 < n; ++c) {
    double alpha = 0.0;
    for (int i = c + 1; i < n; ++i) alpha += A[(size_t)i * n + c] * A[(size_t)i * n + c];
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    const double x0 = A[(size_t)(c + 1) * n + c];
    const double beta = (x0 >= 0.0) ? -alpha : alpha;  // new subdiagonal entry
    std::fill(v.begin(), v.end(), 0.0);
    for (int i = c + 1; i < n; ++i) v[i] = A[(size_t)i * n + c];
    v[c + 1] -= beta;
    double vv = 0.0;
    for (int i = c + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double tau = 2.0 / vv;  // P = I - tau v v^T
    // A <- P A P: p = tau A v, K = tau/2 v.p, q = p - K v, A -= v q^T + q v^T.
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = c + 1; j < n; ++j) s += A[(size_t)i * n + j] * v[j];
      p[i] = tau * s;
    }
    double vp = 0.0;
    for (int i = c + 1; i < n; ++i) vp += v[i] * p[i];
    const double K = 0.5 * tau * vp;
    for (int i = 0; i < n; ++i) q[i] = p[i] - K * v[i];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) A[(size_t)i * n + j] -= v[i] * q[j] + q[i] * v[j];
    // Q <- Q P
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = c + 1; j < n; ++j) s += Q[(size_t)i * n + j] * v[j];
      s *= tau;
      for (int j = c + 1; j < n; ++j) Q[(size_t)i * n + j] -= s * v[j];
    }
  }
  std::vector<double> dg(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) dg[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];  // couples i and i+1

  // Implicit QL with a shift from the trailing 2 x 2 of the active block.
  const double eps = 2.220446049250313e-16;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    while (true) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(dg[m]) + std::fabs(dg[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      if (++iter > 200) return -1;
      double g = (dg[l + 1] - dg[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = dg[m] - dg[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, pacc = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          dg[i + 1] -= pacc;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = dg[i + 1] - pacc;
        r = (dg[i] - g) * s + 2.0 * c * b;
        pacc = s * r;
        dg[i + 1] = g + pacc;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {
          const double t = Q[(size_t)k * n + i + 1];
          Q[(size_t)k * n + i + 1] = s * Q[(size_t)k * n + i] + c * t;
          Q[(size_t)k * n + i] = c * Q[(size_t)k * n + i] - s * t;
        }
      }
      if (deflated) continue;
      dg[l] -= pacc;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  // Sort ascending.
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return dg[a] < dg[b]; });
  for (int j = 0; j < n; ++j) {
    w[j] = dg[idx[j]];
    if (Q_out)
      for (int i = 0; i < n; ++i) Q_out[(size_t)i * n + j] = Q[(size_t)i * n + idx[j]];
  }
  return 0;
}

int cholesky_small(int n, const double* G, double* L) {
  for (int i = 0; i < n * n; ++i) L[i] = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = G[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0.0)) return -1;
    const double ljj = std::sqrt(s);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = G[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / ljj;
    }
  }
  return 0;
}

void inv_lower_transpose(int n, const double* L, double* C) {
  // C = L^{-T} (upper triangular), column-major n x n (C[i + n*j]).
  std::vector<double> Li((size_t)n * n, 0.0);  // L^{-1}, row-major
  for (int j = 0; j < n; ++j) {
    Li[(size_t)j * n + j] = 1.0 / L[(size_t)j * n + j];
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[(size_t)i * n + k] * Li[(size_t)k * n + j];
      Li[(size_t)i * n + j] = -s / L[(size_t)i * n + i];
    }
  }
  // (L^{-T})_{ij} = (L^{-1})_{ji}
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C[i + (size_t)n * j] = Li[(size_t)j * n + i];
}

}  // namespace refl
