// Small dense host-side linear algebra used by the driver.
#pragma once

#include <cmath>

namespace refl {

// Eigen-decomposition of a symmetric n x n matrix (row-major A_in): w
// ascending, Q_out (row-major, may be NULL) with the eigenvectors as
// columns.  Returns 0, or -1 if the QL iteration failed to converge.
int sym_eig_small(int n, const double* A_in, double* w, double* Q_out);

// Symmetric band matrices of order n and half-bandwidth bw, given by their
// lower band: Lb[i * (bw + 1) + (i - j)] = T[i][j] for 0 <= i - j <= bw.

// Orthogonally similar tridiagonal matrix: diag[0..n), sub[0..n-1).
void band_tridiag(int n, int bw, const double* Lb, double* diag, double* sub);

// Number of eigenvalues of the symmetric tridiagonal (diag, sub) below x.
int tridiag_count_below(int n, const double* diag, const double* sub, double x);

// The m-th smallest eigenvalue (m = 0 .. n-1) of (diag, sub) by bisection.
double tridiag_eigval(int n, const double* diag, const double* sub, int m);

// Number of eigenvalues of the band matrix below x, from the signs of the
// pivots of T - xI = L D L^T (Sylvester's law of inertia), or -1 if the
// factorisation without pivoting grew (a multiplier above 1e8).  work holds
// n * (bw + 1) doubles and keeps the factors (L, then 1 / D); with lmax the
// largest multiplier size is returned there.
int band_count_below(int n, int bw, const double* Lb, double x, double* work,
                     double* lmax = nullptr);

// y <- (T - xI)^{-1} y from the factors that a successful band_count_below
// left in work.
void band_ldl_solve(int n, int bw, const double* work, double* y);

// Unit vector y (length n) from `iters` steps of inverse iteration with
// T - sigma I; returns ||T y - sigma y||_2.  The start vector is y itself
// when use_start, else a fixed sequence; with nq > 0 the components along
// the orthonormal columns of Q (n x nq) are removed after every solve.
double band_inverse_iteration(int n, int bw, const double* Lb, double sigma, int iters, double* y,
                              const double* Q = nullptr, int nq = 0, bool use_start = false);

// Ritz test of a block Lanczos run.  TA and TB hold the blocks A_i
// (symmetric) and B_i (upper triangular) of the block tridiagonal T_j,
// b x b column-major, i < j.  Fills theta_k, theta_{k+1} (1-based k) and
// their residual radii ||H x - theta x|| (from the Ritz vector of T_j and
// the last block B_j), and with `extremes` the smallest and largest Ritz
// values (and their radii).  With `prev` (the check of an earlier step of
// the same run) the searches start near the earlier values, the extremes
// too when prev has them (the result does not depend on the guess: every
// value is confirmed by inertia counts).
struct RitzCheck {
  double th_k = NAN, th_k1 = NAN, res_k = NAN, res_k1 = NAN, th_min = NAN, th_max = NAN;
  double res_min = NAN, res_max = NAN;  // residual radii of th_min and th_max
};
void ritz_check(int j, int b, int k, const double* TA, const double* TB, bool extremes,
                RitzCheck& out, const RitzCheck* prev = nullptr);
// Only the extremes (th_min, th_max and their radii) of T_j into out,
// warm-started from prev's extremes when it has them.
void ritz_extremes(int j, int b, const double* TA, const double* TB, RitzCheck& out,
                   const RitzCheck* prev = nullptr);

// Orthonormal Ritz vectors of T_j (n = j b) for its nvec smallest Ritz
// values, column-major in Y (n x nvec).  Returns 0, or -1 if nvec is out of
// range.
int ritz_vectors(int j, int b, const double* TA, const double* TB, int nvec, double* Y);

}  // namespace refl
