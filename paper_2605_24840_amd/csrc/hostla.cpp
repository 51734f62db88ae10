// Small dense linear algebra on the host for the k x k problems of the
// driver: symmetric eigen-decomposition by Householder reduction to
// tridiagonal form followed by the implicit QL iteration with shifts, and a
// Cholesky factorisation.  The QL stage is the published procedure of
// Bowdler, Martin, Reinsch and Wilkinson ("The QR and QL algorithms for
// symmetric matrices", Numer. Math. 11, 1968, 293-306; EISPACK tql2): a
// shift from the leading 2 x 2 block of the unreduced part, a chase of
// plane rotations from the bottom of that part to its top, accumulated into
// Q; its recurrence variables (g, r, s, c, p, f, b) keep the roles they
// have there.  For the block tridiagonal matrices of the
// Lanczos run (order up to d, half-bandwidth b <= 32): reduction of a band
// matrix to tridiagonal form by plane rotations that chase the bulge down the
// band (Schwarz, Numer. Math. 12, 1968), Sturm-sequence bisection for single
// eigenvalues (Kahan's LDL^T count), and inverse iteration with banded LU.
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

void band_tridiag(int n, int bw, const double* Lb, double* diag, double* sub) {
  // Working storage with one extra diagonal for the bulge:
  // A[i][j] (i >= j, i - j <= bw + 1) at S[i * ws + (i - j)], ws = bw + 2.
  const int ws = bw + 2;
  std::vector<double> S((size_t)n * ws, 0.0);
  for (int i = 0; i < n; ++i)
    for (int t = 0; t <= bw && t <= i; ++t) S[(size_t)i * ws + t] = Lb[(size_t)i * (bw + 1) + t];
  double* A = S.data();
  // Rotation in the plane (p, q = p + 1) that zeroes A[q][col] (col < p):
  // rows p and q of the lower band (columns m < p) are contiguous, and for
  // m > q the pair (A[m][q], A[m][p]) is adjacent in row m.
  auto rotate = [&](int p, int col) {
    const int q = p + 1;
    double* rp = A + (size_t)p * ws;  // rp[t] = A[p][p - t]
    double* rq = A + (size_t)q * ws;  // rq[t] = A[q][q - t]
    const double a = rp[p - col], e = rq[q - col];
    if (e == 0.0) return;
    const double r = std::hypot(a, e), c = a / r, s = e / r;
    const int lo = std::max(0, q - bw - 1);
    for (int m = lo; m < p; ++m) {
      const double x = rp[p - m], y = rq[q - m];
      rp[p - m] = c * x + s * y;
      rq[q - m] = -s * x + c * y;
    }
    const int hi = std::min(n - 1, p + bw + 1);
    for (int m = q + 1; m <= hi; ++m) {
      double* rm = A + (size_t)m * ws;
      const double x = rm[m - p], y = rm[m - q];
      rm[m - p] = c * x + s * y;
      rm[m - q] = -s * x + c * y;
    }
    const double app = rp[0], aqq = rq[0], apq = rq[1];
    rp[0] = c * c * app + 2.0 * c * s * apq + s * s * aqq;
    rq[0] = s * s * app - 2.0 * c * s * apq + c * c * aqq;
    rq[1] = c * s * (aqq - app) + (c * c - s * s) * apq;
    rq[q - col] = 0.0;
  };
  if (bw > 1) {
    for (int k = 0; k + 2 < n; ++k) {
      for (int r = std::min(bw, n - 1 - k); r >= 2; --r) {
        int i = k + r, col = k;
        rotate(i - 1, col);
        while (i + bw < n) {  // bulge at (i + bw, i - 1)
          col = i - 1;
          i += bw;
          rotate(i - 1, col);
        }
      }
    }
  }
  for (int i = 0; i < n; ++i) diag[i] = A[(size_t)i * ws];
  for (int i = 0; i + 1 < n; ++i) sub[i] = (bw >= 1) ? A[(size_t)(i + 1) * ws + 1] : 0.0;
}

int tridiag_count_below(int n, const double* diag, const double* sub, double x) {
  // Number of negative pivots of the LDL^T factorisation of T - xI.
  const double tiny = 1e-300;
  int cnt = 0;
  double q = diag[0] - x;
  if (q == 0.0) q = -tiny;
  if (q < 0.0) ++cnt;
  for (int i = 1; i < n; ++i) {
    q = (diag[i] - x) - sub[i - 1] * sub[i - 1] / q;
    if (q == 0.0) q = -tiny;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

double tridiag_eigval(int n, const double* diag, const double* sub, int m) {
  // Gershgorin interval, then bisection on the Sturm count.
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(sub[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(sub[i]) : 0.0);
    lo = std::min(lo, diag[i] - r);
    hi = std::max(hi, diag[i] + r);
  }
  const double scale = std::max(std::fabs(lo), std::fabs(hi));
  lo -= 1e-14 * scale + 1e-300;
  hi += 1e-14 * scale + 1e-300;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (hi - lo <= 4.0 * 2.220446049250313e-16 * std::max(std::fabs(lo), std::fabs(hi))) break;
    if (tridiag_count_below(n, diag, sub, mid) > m)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

int band_count_below(int n, int bw, const double* Lb, double x, double* work, double* lmax) {
  // T - xI = L D L^T without pivoting; L (unit lower, band) row i at
  // work[i * bw + (i - j - 1)], j = i - bw .. i - 1; 1 / D at work[n * bw + i].
  // Row i is a forward substitution with the rows of L above it: with
  // v[j] = L[i][j] D[j],
  //   v[j] = T[i][j] - sum_{i - bw <= m < j} v[m] L[j][m],  L[i][j] = v[j] / D[j],
  //   D[i] = T[i][i] - x - sum_j L[i][j] v[j];
  // it is done column by column (each finished v[m] updates all later
  // entries at once), which keeps the dependent chain b long, not b^2 / 2.
  // Returns the number of negative pivots, or -1 if a multiplier exceeds
  // 1e8 in size (element growth: the count is not trusted).
  double* L = work;
  double* Di = work + (size_t)n * bw;
  const double tiny = 1e-300;
  double big = 0.0;
  double pbuf[64];
  std::vector<double> pvec;
  double* p = pbuf;
  if (bw > 64) {
    pvec.resize(bw);
    p = pvec.data();
  }
  int cnt = 0;
  for (int i = 0; i < n; ++i) {
    const int j0 = std::max(0, i - bw), w = i - j0;
    const double* ai = Lb + (size_t)i * (bw + 1);  // ai[t] = T[i][i - t]
    double* li = L + (size_t)i * bw;                // li[t - 1] = L[i][i - t]
    for (int q = 0; q < w; ++q) p[q] = ai[i - j0 - q];   // p[q] for column j0 + q
    double di = ai[0] - x;
    for (int q = 0; q < w; ++q) {
      const int j = j0 + q;
      const double u = p[q];                   // v[j], final
      const double l = u * Di[j];
      if (!(std::fabs(l) < 1e8)) return -1;
      big = std::max(big, std::fabs(l));
      li[i - j - 1] = l;
      di -= l * u;
      // Later columns jj > j of this row: p[jj] -= v[j] L[jj][j].
      for (int qq = q + 1; qq < w; ++qq) {
        const int jj = j0 + qq;
        p[qq] -= u * L[(size_t)jj * bw + (jj - j - 1)];
      }
    }
    if (di == 0.0) di = -tiny;
    Di[i] = 1.0 / di;
    if (di < 0.0) ++cnt;
  }
  if (lmax) *lmax = big;
  return cnt;
}

void band_ldl_solve(int n, int bw, const double* work, double* y) {
  const double* L = work;
  const double* Di = work + (size_t)n * bw;
  for (int i = 0; i < n; ++i) {                  // L z = y
    const double* li = L + (size_t)i * bw;
    double s = y[i];
    for (int t = 1; t <= bw && t <= i; ++t) s -= li[t - 1] * y[i - t];
    y[i] = s;
  }
  for (int i = 0; i < n; ++i) y[i] *= Di[i];     // D w = z
  for (int i = n - 1; i >= 0; --i) {             // L^T y = w
    double s = y[i];
    for (int t = 1; t <= bw && i + t < n; ++t) s -= L[(size_t)(i + t) * bw + (t - 1)] * y[i + t];
    y[i] = s;
  }
}

double band_inverse_iteration(int n, int bw, const double* Lb, double sigma, int iters,
                              double* y, const double* Q, int nq, bool use_start) {
  // LU with partial pivoting of B = T - sigma I (band, half-bandwidth bw).
  // Row i is held for columns i - bw .. i + 2 bw at U[i * uw + (c - i + bw)].
  const int uw = 3 * bw + 1;
  auto tij = [&](int i, int j) -> double {
    const int t = i >= j ? i - j : j - i;
    if (t > bw) return 0.0;
    return i >= j ? Lb[(size_t)i * (bw + 1) + t] : Lb[(size_t)j * (bw + 1) + t];
  };
  std::vector<double> U((size_t)n * uw, 0.0), Lm((size_t)n * (bw + 1), 0.0);
  std::vector<int> piv(n);
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i) {
    double rs = 0.0;
    for (int j = std::max(0, i - bw); j <= std::min(n - 1, i + bw); ++j) {
      const double v = tij(i, j) - (i == j ? sigma : 0.0);
      U[(size_t)i * uw + (j - i + bw)] = v;
      rs += std::fabs(tij(i, j));
    }
    tnorm = std::max(tnorm, rs);
  }
  const double tiny = 2.220446049250313e-16 * std::max(tnorm, 1e-300);
  auto u = [&](int i, int c) -> double& { return U[(size_t)i * uw + (c - i + bw)]; };
  for (int j = 0; j < n; ++j) {
    const int last = std::min(n - 1, j + bw);
    int p = j;
    for (int i = j + 1; i <= last; ++i)
      if (std::fabs(u(i, j)) > std::fabs(u(p, j))) p = i;
    piv[j] = p;
    const int cend = std::min(n - 1, j + 2 * bw);
    if (p != j)
      for (int c = j; c <= cend; ++c) std::swap(u(j, c), u(p, c));
    if (std::fabs(u(j, j)) < tiny) u(j, j) = (u(j, j) < 0.0 ? -tiny : tiny);
    for (int i = j + 1; i <= last; ++i) {
      const double m = u(i, j) / u(j, j);
      Lm[(size_t)i * (bw + 1) + (i - j)] = m;
      u(i, j) = 0.0;
      if (m != 0.0)
        for (int c = j + 1; c <= cend; ++c) u(i, c) -= m * u(j, c);
    }
  }
  // Start vector: the caller's, or a fixed, non-special sequence.
  if (!use_start)
    for (int i = 0; i < n; ++i) y[i] = 1.0 + 0.5 * std::sin(1.0 + 0.7 * i);
  // Components along the columns of Q (n x nq, orthonormal) are removed
  // after every solve (two passes of modified Gram-Schmidt).
  auto deflate = [&]() {
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 0; q < nq; ++q) {
        const double* qc = Q + (size_t)q * n;
        double c = 0.0;
        for (int i = 0; i < n; ++i) c += qc[i] * y[i];
        for (int i = 0; i < n; ++i) y[i] -= c * qc[i];
      }
  };
  deflate();
  for (int it = 0; it < iters; ++it) {
    // Forward: apply the row swaps and unit-lower multipliers in order.
    for (int j = 0; j < n; ++j) {
      if (piv[j] != j) std::swap(y[j], y[piv[j]]);
      const int last = std::min(n - 1, j + bw);
      for (int i = j + 1; i <= last; ++i) y[i] -= Lm[(size_t)i * (bw + 1) + (i - j)] * y[j];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      const int cend = std::min(n - 1, i + 2 * bw);
      for (int c = i + 1; c <= cend; ++c) s -= u(i, c) * y[c];
      y[i] = s / u(i, i);
    }
    deflate();
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) nrm += y[i] * y[i];
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return INFINITY;
    for (int i = 0; i < n; ++i) y[i] /= nrm;
  }
  double r2 = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = -sigma * y[i];
    for (int j = std::max(0, i - bw); j <= std::min(n - 1, i + bw); ++j) s += tij(i, j) * y[j];
    r2 += s * s;
  }
  return std::sqrt(r2);
}

// ------------------------------------------------ Ritz test of block Lanczos


// Lower band (half-bandwidth b) of the block tridiagonal T_j with diagonal
// blocks A_i (symmetrised) and sub-diagonal blocks B_i (upper triangular).
static std::vector<double> lower_band_of(int j, int b, const double* TA, const double* TB) {
  const int n = j * b;
  std::vector<double> Lb((size_t)n * (b + 1), 0.0);
  for (int i = 0; i < n; ++i) {
    const int I = i / b, r = i % b;
    const double* A = TA + (size_t)I * b * b;
    for (int c = 0; c <= r; ++c) Lb[(size_t)i * (b + 1) + (r - c)] = 0.5 * (A[r + c * b] + A[c + r * b]);
    if (I > 0) {
      const double* B = TB + (size_t)(I - 1) * b * b;  // T[I b + r][(I-1) b + c] = B[r][c], r <= c
      for (int c = r; c < b; ++c) Lb[(size_t)i * (b + 1) + (b + r - c)] = B[r + c * b];
    }
  }
  return Lb;
}

// Ritz pairs of the block tridiagonal T_j for the eigenvalue indices ms[q]
// (0-based, q < nm): theta[q], the residual radius res[q], and with Y != null
// the unit Ritz vector of T_j in column q of Y (n x nm, column-major).  With
// t0/r0 (an earlier step's Ritz values and radii for the same indices; NaN
// for none) the bisection starts from a bracket near the earlier value: T_i
// is a leading principal submatrix of T_j, so by interlacing each Ritz value
// can only have moved down; the bracket is confirmed by two inertia counts
// and widened until it holds, so the result does not depend on the guess.
static void ritz_pairs(int j, int b, const double* TA, const double* TB, int nm, const int* ms,
                       const double* t0, const double* r0, double* theta_out, double* res_out,
                       double* Y) {
  const int n = j * b;
  const std::vector<double> Lb = lower_band_of(j, b, TA, TB);
  // Gershgorin bounds.
  double glo = INFINITY, ghi = -INFINITY;
  {
    std::vector<double> rad(n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int t = 1; t <= b && t <= i; ++t) {
        const double v = std::fabs(Lb[(size_t)i * (b + 1) + t]);
        rad[i] += v;
        rad[i - t] += v;
      }
    for (int i = 0; i < n; ++i) {
      glo = std::min(glo, Lb[(size_t)i * (b + 1)] - rad[i]);
      ghi = std::max(ghi, Lb[(size_t)i * (b + 1)] + rad[i]);
    }
  }
  const double scale = std::max({std::fabs(glo), std::fabs(ghi), 1e-300});
  std::vector<double> work((size_t)n * (b + 1)), diag, sub;
  bool reduced = false;
  // Bracket the m-th smallest eigenvalue (0-based) to width 1e-9 * scale by
  // bisection on the inertia of T - xI; if the factorisation declines, use
  // the band-to-tridiagonal reduction and its Sturm count instead.
  auto count = [&](double x) {
    if (!reduced) {
      const int c = band_count_below(n, b, Lb.data(), x, work.data());
      if (c >= 0) return c;
      diag.resize(n);
      sub.resize(std::max(n - 1, 1));
      band_tridiag(n, b, Lb.data(), diag.data(), sub.data());
      reduced = true;
    }
    return tridiag_count_below(n, diag.data(), sub.data(), x);
  };
  // Bisection to `width`, then (in pair) inverse iteration from the
  // midpoint; if the Rayleigh quotient leaves the bracket (a neighbour was
  // closer to the midpoint) the bracket is narrowed further and the
  // iteration repeated.
  struct Bracket {
    double lo, hi;
  };
  auto bracket = [&](int m, double width, Bracket* b0) {
    Bracket b = b0 ? *b0 : Bracket{glo - 1e-12 * scale, ghi + 1e-12 * scale};
    while (b.hi - b.lo > width) {
      const double mid = 0.5 * (b.lo + b.hi);
      if (mid <= b.lo || mid >= b.hi) break;
      if (count(mid) > m) b.hi = mid; else b.lo = mid;
    }
    return b;
  };
  std::vector<double> y(n), ty(n), fwork((size_t)n * (b + 1));
  const double* Bj = TB + (size_t)(j - 1) * b * b;
  // For the unit vector y: theta = y^T T y, rT = ||(T - theta) y|| and the
  // residual radius of the Ritz pair,
  // ||H x - theta x||^2 = ||(T - theta) y||^2 + ||B_j y(last block)||^2.
  auto rayleigh = [&](double& theta, double& rT, double& res) {
    double q = 0.0;
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int t = 0; t <= b; ++t) {
        if (i - t >= 0) s += Lb[(size_t)i * (b + 1) + t] * y[i - t];
        if (t > 0 && i + t < n) s += Lb[(size_t)(i + t) * (b + 1) + t] * y[i + t];
      }
      ty[i] = s;
      q += s * y[i];
    }
    theta = q;
    double r1 = 0.0;
    for (int i = 0; i < n; ++i) r1 += (ty[i] - q * y[i]) * (ty[i] - q * y[i]);
    double r2 = 0.0;
    for (int r = 0; r < b; ++r) {
      double s = 0.0;
      for (int c = r; c < b; ++c) s += Bj[r + c * b] * y[n - b + c];
      r2 += s * s;
    }
    rT = std::sqrt(r1);
    res = std::sqrt(r1 + r2);
  };
  // `solves` steps of inverse iteration on y with the L D L^T factors that
  // band_count_below left in fwork; false if y lost its norm.
  auto ldl_steps = [&](int solves) {
    for (int it = 0; it < solves; ++it) {
      band_ldl_solve(n, b, fwork.data(), y.data());
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += y[i] * y[i];
      nrm = std::sqrt(nrm);
      if (!(nrm > 0.0) || !std::isfinite(nrm)) return false;
      for (int i = 0; i < n; ++i) y[i] /= nrm;
    }
    return true;
  };
  auto start_vector = [&]() {
    for (int i = 0; i < n; ++i) y[i] = 1.0 + 0.5 * std::sin(1.0 + 0.7 * i);
  };
  // Inverse iteration from the L D L^T factors of T - sigma I when they
  // came without growth (multipliers below 1e3), else from the pivoted LU.
  // Either way theta and res are the Rayleigh quotient and the true
  // residual radius of the vector returned.
  auto pair = [&](double sigma, double& theta, double& res) {
    double lmax = 0.0, rT;
    bool done = false;
    if (band_count_below(n, b, Lb.data(), sigma, fwork.data(), &lmax) >= 0 && lmax < 1e3) {
      start_vector();
      done = ldl_steps(3);
    }
    if (!done) band_inverse_iteration(n, b, Lb.data(), sigma, 3, y.data());
    rayleigh(theta, rT, res);
  };
  // A bracket [lo, hi] of the m-th eigenvalue near an earlier Ritz value
  // t0 with residual radius r0, confirmed by counts (false if none found
  // before the Gershgorin bounds).
  auto warm = [&](int m, double t0, double r0, Bracket& out_b) {
    if (!std::isfinite(t0) || !std::isfinite(r0)) return false;
    double dlo = std::max(4.0 * r0, 1e-6 * scale), dhi = 1e-9 * scale;
    for (int tries = 0; tries < 60; ++tries) {
      const double lo = std::max(t0 - dlo, glo - 1e-12 * scale);
      const double hi = std::min(t0 + dhi, ghi + 1e-12 * scale);
      const bool lo_ok = lo <= glo - 1e-12 * scale || count(lo) <= m;
      const bool hi_ok = hi >= ghi + 1e-12 * scale || count(hi) > m;
      if (lo_ok && hi_ok) {
        out_b = Bracket{lo, hi};
        return true;
      }
      if (!lo_ok) dlo *= 8.0;
      if (!hi_ok) dhi = std::max(8.0 * dhi, 1e-6 * scale);
      if (lo <= glo - 1e-12 * scale && hi >= ghi + 1e-12 * scale) break;
    }
    return false;
  };
  // Two shifted inverse iterations from an earlier Ritz value t0 with
  // residual radius r0, instead of a bisection: two solves at
  // t0 - max(r0, w) (w = 1e-6 scale; not at t0 itself, an eigenvalue of a
  // leading block of T, where the factorisation without pivoting grows),
  // then four at w / 4 below their Rayleigh quotient (above, for the
  // largest eigenvalue).  The result is accepted
  // only if two inertia counts show that [theta - delta, theta + delta],
  // delta >= 4 ||(T - theta) y||, holds exactly one eigenvalue and that it
  // is the m-th: the eigenvalue within ||(T - theta) y|| of theta is then
  // that one.
  auto rqi = [&](int m, double t0, double r0, double& theta, double& res) {
    if (!std::isfinite(t0) || !std::isfinite(r0)) return false;
    const double w = 1e-6 * scale;
    // Interlacing: Ritz values counted from the bottom only move down as
    // the basis grows, the largest only up.
    const double dir = (m == n - 1 && n > 1) ? 1.0 : -1.0;
    double sigma = t0 + dir * std::max(r0, w), rT = INFINITY;
    start_vector();
    for (int it = 0; it < 2; ++it) {
      double lmax = 0.0;
      if (band_count_below(n, b, Lb.data(), sigma, fwork.data(), &lmax) < 0 || !(lmax < 1e3)) return false;
      if (!ldl_steps(it == 0 ? 2 : 4)) return false;
      rayleigh(theta, rT, res);
      if (!std::isfinite(theta) || !std::isfinite(res)) return false;
      sigma = theta + dir * 0.25 * w;
    }
    const double delta = std::max(4.0 * rT, 2.0 * w);
    return count(theta - delta) == m && count(theta + delta) == m + 1;
  };
  // The smallest (m = 0) or largest (m = n - 1) eigenvalue by inverse
  // iteration with shifts outside the spectrum, where T - sigma I is
  // definite and its factorisation without pivoting is stable: from the
  // Gershgorin bound, then from theta -/+ (||(T - theta) y|| + w) for as
  // long as a count confirms that the shift is still outside.  Accepted, as
  // in rqi, once converged and a count shows that [sigma, theta + delta]
  // (mirrored for the largest) holds exactly one eigenvalue.
  auto edge = [&](int m, double& theta, double& res) {
    const bool low = m == 0;
    if (!low && m != n - 1) return false;
    const double w = 1e-6 * scale;
    double sigma = low ? glo - w : ghi + w, rT = INFINITY;
    const int outside = low ? 0 : n;
    start_vector();
    for (int it = 0; it < 8; ++it) {
      double lmax = 0.0;
      const int c = band_count_below(n, b, Lb.data(), sigma, fwork.data(), &lmax);
      if (c != outside || !(lmax < 1e3)) return false;
      if (!ldl_steps(3)) return false;
      rayleigh(theta, rT, res);
      if (!std::isfinite(theta) || !std::isfinite(res)) return false;
      if (rT <= 1e-10 * scale) {
        const double delta = std::max(4.0 * rT, 2.0 * w);
        return low ? count(theta + delta) == 1 : count(theta - delta) == n - 1;
      }
      sigma = low ? theta - rT - w : theta + rT + w;
    }
    return false;
  };
  auto ritz = [&](int m, double& theta, double& res, double t0, double r0, double gap0) {
    // The earlier value is a good start once its residual radius is well
    // inside the gap to its neighbour.
    if (std::isfinite(r0) && r0 < 0.25 * gap0 && rqi(m, t0, r0, theta, res)) return;
    if (!std::isfinite(t0) && edge(m, theta, res)) return;
    double width = 1e-6 * scale;
    Bracket w0;
    Bracket b = warm(m, t0, r0, w0) ? bracket(m, width, &w0) : bracket(m, width, nullptr);
    while (true) {
      pair(0.5 * (b.lo + b.hi), theta, res);
      const double slack = b.hi - b.lo;
      if ((theta >= b.lo - slack && theta <= b.hi + slack) || width < 1e-14 * scale) return;
      width *= 1e-3;
      b = bracket(m, width, &b);
    }
  };
  for (int q = 0; q < nm; ++q) {
    double gap0 = INFINITY;
    if (t0)
      for (int p = 0; p < nm; ++p)
        if (p != q && std::isfinite(t0[p])) gap0 = std::min(gap0, std::fabs(t0[p] - t0[q]));
    ritz(ms[q], theta_out[q], res_out[q], t0 ? t0[q] : NAN, r0 ? r0[q] : NAN, gap0);
    if (Y) std::copy(y.begin(), y.end(), Y + (size_t)q * n);
  }
}

// Ritz values theta_k, theta_{k+1} of T_j (and, with `extremes`, the
// smallest and largest) with their residual radii; `prev` warm-starts the
// searches (the extremes too when it holds them).
void ritz_check(int j, int b, int k, const double* TA, const double* TB, bool extremes,
                RitzCheck& out, const RitzCheck* prev) {
  const int ms[2] = {k - 1, k};
  double th[2], rs[2];
  if (prev) {
    const double t0[2] = {prev->th_k, prev->th_k1}, r0[2] = {prev->res_k, prev->res_k1};
    ritz_pairs(j, b, TA, TB, 2, ms, t0, r0, th, rs, nullptr);
  } else {
    ritz_pairs(j, b, TA, TB, 2, ms, nullptr, nullptr, th, rs, nullptr);
  }
  out.th_k = th[0];
  out.th_k1 = th[1];
  out.res_k = rs[0];
  out.res_k1 = rs[1];
  if (extremes) ritz_extremes(j, b, TA, TB, out, prev);
}

void ritz_extremes(int j, int b, const double* TA, const double* TB, RitzCheck& out,
                   const RitzCheck* prev) {
  const int me[2] = {0, j * b - 1};
  double th[2], rs[2];
  if (prev && std::isfinite(prev->th_min) && std::isfinite(prev->th_max) &&
      std::isfinite(prev->res_min) && std::isfinite(prev->res_max)) {
    const double t0[2] = {prev->th_min, prev->th_max}, r0[2] = {prev->res_min, prev->res_max};
    ritz_pairs(j, b, TA, TB, 2, me, t0, r0, th, rs, nullptr);
  } else {
    ritz_pairs(j, b, TA, TB, 2, me, nullptr, nullptr, th, rs, nullptr);
  }
  out.th_min = th[0];
  out.th_max = th[1];
  out.res_min = rs[0];
  out.res_max = rs[1];
}

int ritz_vectors(int j, int b, const double* TA, const double* TB, int nvec, double* Y) {
  const int n = j * b;
  if (nvec < 1 || nvec > n) return -1;
  std::vector<int> ms(nvec);
  std::vector<double> th(nvec), rs(nvec);
  for (int q = 0; q < nvec; ++q) ms[q] = q;
  ritz_pairs(j, b, TA, TB, nvec, ms.data(), nullptr, nullptr, th.data(), rs.data(), Y);
  // Inverse iteration on close or repeated eigenvalues can return nearly
  // parallel vectors: each column is orthogonalised against the earlier ones
  // (modified Gram-Schmidt, twice); one that loses its norm is recomputed by
  // inverse iteration at its Ritz value with the earlier columns deflated,
  // from other start vectors until one survives.
  std::vector<double> Lb;
  for (int q = 0; q < nvec; ++q) {
    double* yq = Y + (size_t)q * n;
    for (int attempt = 0; attempt <= 8; ++attempt) {
      const double n0 = std::sqrt(std::inner_product(yq, yq + n, yq, 0.0));
      for (int pass = 0; pass < 2; ++pass)
        for (int p = 0; p < q; ++p) {
          const double* yp = Y + (size_t)p * n;
          const double c = std::inner_product(yp, yp + n, yq, 0.0);
          for (int i = 0; i < n; ++i) yq[i] -= c * yp[i];
        }
      const double n1 = std::sqrt(std::inner_product(yq, yq + n, yq, 0.0));
      if (n1 > 1e-8 * std::max(n0, 1e-300)) {
        for (int i = 0; i < n; ++i) yq[i] /= n1;
        break;
      }
      if (attempt == 8) return -1;
      if (Lb.empty()) Lb = lower_band_of(j, b, TA, TB);
      for (int i = 0; i < n; ++i) yq[i] = std::sin(1.0 + (2.3 + attempt) * i + 0.37 * attempt);
      band_inverse_iteration(n, b, Lb.data(), th[q], 3, yq, Y, q, true);
    }
  }
  return 0;
}

}  // namespace refl
