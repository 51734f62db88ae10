// Small dense host-side linear algebra used by the driver.
#pragma once

namespace refl {

// Eigen-decomposition of a symmetric n x n matrix (row-major A_in): w
// ascending, Q_out (row-major, may be NULL) with the eigenvectors as
// columns.  Returns 0, or -1 if the QL iteration failed to converge.
int sym_eig_small(int n, const double* A_in, double* w, double* Q_out);

// G = L L^T for symmetric positive definite G (row-major); -1 if not.
int cholesky_small(int n, const double* G, double* L);

// C = L^{-T} for lower-triangular L (row-major), written column-major.
void inv_lower_transpose(int n, const double* L, double* C);

}  // namespace refl
