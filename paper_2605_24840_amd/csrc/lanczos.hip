// Kernels of the block-Lanczos shift estimate (the partial-eigensolver route
// of section 4.3).  One Lanczos step, with V = [Q_1 .. Q_j] the d x n basis
// (column-major, ld = ldv) and W = H Q_j from the symmetric thin product:
//
//   two passes of block classical Gram-Schmidt against all of V
//     k_lz_proj_partial / k_lz_proj_finish   C = V^T W   (n x nb)
//     k_lz_apply_partial + k_lz_rows(SUB)    W <- W - V C
//   then three rounds of Cholesky QR, the first one shifted (shifted
//   CholQR3 of Fukaya, Kannan, Nakatsukasa, Zhang and Yamamoto, 2020)
//     k_lz_rows(GRAM)  partial Gram matrices of 256-row slabs
//     k_lz_chol        one wave: G = L L^T, R = L^T, B <- R B
//     k_lz_rows(TRSM)  W <- W R^{-1}
//   so that W_in = Q_{j+1} B_j with B_j upper triangular.
//
// The diagonal block A_j = Q_j^T H Q_j is the last block of the two
// projections, recorded by k_lz_proj_finish.  Every reduction runs in a
// fixed order (per-block partials summed by the next kernel), so the run is
// deterministic.
#include "common.h"
#include "launch.h"

namespace refl {

constexpr int LZ_RC = 512;  // rows per block of the projection partials
constexpr int LZ_CC = 128;  // basis columns per block of the update partials

static inline int lz_nblocks(int64_t n, int per) { return (int)((n + per - 1) / per); }

// part[(rc * n + c) * NB + j] = sum over the rows of chunk rc of V[r, c] W[r, j].
// Block = one wave; CV = 256 / NB basis columns, 4 outputs per lane; the
// 64-row slabs of V and W are staged in LDS.
template <int NB>
__global__ __launch_bounds__(64) void k_lz_proj_partial(const double* __restrict__ V, int64_t ldv,
                                                        int n, const double* __restrict__ W,
                                                        int64_t ldw, int nb, int d,
                                                        double* __restrict__ part) {
  constexpr int CV = 256 / NB;
  __shared__ double sV[64][CV + 1];
  __shared__ double sW[64][NB + 1];
  const int lane = threadIdx.x;
  const int c0 = blockIdx.x * CV;
  const int r0 = blockIdx.y * LZ_RC;
  const int r1 = min(d, r0 + LZ_RC);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int rs = r0; rs < r1; rs += 64) {
    const int r = rs + lane;
    const bool in = r < r1;
#pragma unroll 4
    for (int cl = 0; cl < CV; ++cl) {
      const int c = c0 + cl;
      sV[lane][cl] = (in && c < n) ? V[(int64_t)c * ldv + r] : 0.0;
    }
#pragma unroll 4
    for (int j = 0; j < NB; ++j) sW[lane][j] = (in && j < nb) ? W[(int64_t)j * ldw + r] : 0.0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = lane + 64 * q, cl = o / NB, j = o % NB;
      double a = acc[q];
      for (int i = 0; i < 64; ++i) a = fma(sV[i][cl], sW[i][j], a);
      acc[q] = a;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int o = lane + 64 * q, cl = o / NB, j = o % NB;
    const int c = c0 + cl;
    if (c < n && j < nb) part[((int64_t)blockIdx.y * n + c) * NB + j] = acc[q];
  }
}

// C[c + j n] = sum_rc part (fixed order).  The rows c >= n - b of C (the
// coefficients on the newest block Q_j) are written to, or with `accumulate`
// added to, Arec (b x b, column-major).
__global__ __launch_bounds__(256) void k_lz_proj_finish(const double* __restrict__ part, int nrc,
                                                        int n, int nb, int NB,
                                                        double* __restrict__ C,
                                                        double* __restrict__ Arec, int b,
                                                        int accumulate) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= n * nb) return;
  const int c = o % n, j = o / n;
  double s = 0.0;
  for (int rc = 0; rc < nrc; ++rc) s += part[((int64_t)rc * n + c) * NB + j];
  C[c + (int64_t)j * n] = s;
  if (Arec && c >= n - b) {
    double* a = Arec + (c - (n - b)) + (int64_t)j * b;
    *a = accumulate ? *a + s : s;
  }
}

// apart[(cc * NB + j) * d + r] = sum over the columns c of chunk cc of
// V[r, c] C[c + j n].  One row per thread; the chunk of C sits in LDS.
template <int NB>
__global__ __launch_bounds__(256) void k_lz_apply_partial(const double* __restrict__ V, int64_t ldv,
                                                          int n, const double* __restrict__ C,
                                                          int nb, int d,
                                                          double* __restrict__ apart) {
  __shared__ double sC[LZ_CC][NB];
  const int c0 = blockIdx.y * LZ_CC;
  const int cn = min(LZ_CC, n - c0);
  for (int e = threadIdx.x; e < LZ_CC * NB; e += 256) {
    const int cl = e / NB, j = e % NB;
    sC[cl][j] = (cl < cn && j < nb) ? C[(c0 + cl) + (int64_t)j * n] : 0.0;
  }
  __syncthreads();
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= d) return;
  double acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = 0.0;
  const double* v = V + (int64_t)c0 * ldv + r;
  int cl = 0;
  for (; cl + 4 <= cn; cl += 4) {
    double x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = v[(int64_t)(cl + u) * ldv];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[j] = fma(x[u], sC[cl + u][j], acc[j]);
  }
  for (; cl < cn; ++cl) {
    const double x = v[(int64_t)cl * ldv];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = fma(x, sC[cl][j], acc[j]);
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < nb) apart[((int64_t)blockIdx.y * NB + j) * d + r] = acc[j];
}

// Row-wise update of the d x nb block W (one row per thread, 256-row slabs):
//   SUB   (apart != null)  w -= sum_cc apart[cc]            (fixed order)
//   TRSM  (R != null)      x R = w for upper-triangular R (nb x nb, col-major)
//   the result goes to dst (which may be W), and with gpart != null the
//   slab's Gram matrix x^T x goes to gpart[blockIdx.x * NB * NB + i + j NB].
// W and dst may be the same block (each thread reads its row before writing
// it), so neither is declared restrict.
template <int NB>
__global__ __launch_bounds__(256) void k_lz_rows(const double* W, int64_t ldw, int nb,
                                                 int d, const double* __restrict__ apart, int ncc,
                                                 const double* __restrict__ R,
                                                 double* dst, int64_t ldd,
                                                 double* __restrict__ gpart) {
  __shared__ double sR[NB][NB];
  __shared__ double sX[256][NB + 1];
  if (R) {
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
      const int i = e % NB, j = e / NB;
      sR[i][j] = (i < nb && j < nb) ? R[i + (int64_t)j * nb] : 0.0;
    }
  }
  __syncthreads();
  const int r = blockIdx.x * 256 + threadIdx.x;
  double x[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) x[j] = 0.0;
  if (r < d) {
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (j < nb) x[j] = W[(int64_t)j * ldw + r];
    if (apart) {
      for (int cc = 0; cc < ncc; ++cc)
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (j < nb) x[j] -= apart[((int64_t)cc * NB + j) * d + r];
    }
    if (R) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < nb) {
          double s = x[j];
#pragma unroll
          for (int i = 0; i < j; ++i) s = fma(-x[i], sR[i][j], s);
          x[j] = s / sR[j][j];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (j < nb) dst[(int64_t)j * ldd + r] = x[j];
  }
  if (!gpart) return;
#pragma unroll
  for (int j = 0; j < NB; ++j) sX[threadIdx.x][j] = x[j];
  __syncthreads();
  for (int o = threadIdx.x; o < nb * nb; o += 256) {
    const int i = o % nb, j = o / nb;
    double a = 0.0;
    for (int t = 0; t < 256; ++t) a = fma(sX[t][i], sX[t][j], a);
    gpart[(int64_t)blockIdx.x * NB * NB + i + j * NB] = a;
  }
}

// One wave.  G = sum of the slab Gram matrices (fixed order), symmetrised,
// plus sigma I with sigma = shift_rel * trace(G) when shift_rel > 0.
// Cholesky G = L L^T in LDS; R = L^T (nb x nb, col-major) to Rout; Bacc = R
// (round 0) or R Bacc.  A non-positive pivot is replaced by 1 and bit 1 of
// flag[0] set.  With Brec != null (the last round of a Lanczos step), Bacc
// is also copied to Brec, and if its smallest diagonal entry is below 1e-10
// times the largest entry of Arec or Bacc, bit 2 of flag[0] is set (the
// block Krylov space has become, to working accuracy, invariant).  flag[1]
// keeps the first `tag` (the step number) at which a bit was set.
__global__ __launch_bounds__(64) void k_lz_chol(const double* __restrict__ gpart, int nblk, int nb,
                                                int NB, double shift_rel,
                                                double* __restrict__ Rout,
                                                double* __restrict__ Bacc, int round,
                                                const double* __restrict__ Arec,
                                                double* __restrict__ Brec, int* __restrict__ flag,
                                                int tag) {
  __shared__ double G[32][33];
  __shared__ double Bt[32][33];
  __shared__ double sig;
  __shared__ int bad;
  const int lane = threadIdx.x;
  for (int e = lane; e < nb * nb; e += 64) {
    const int i = e % nb, j = e / nb;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += gpart[(int64_t)b * NB * NB + i + j * NB];
    G[i][j] = s;
  }
  if (lane == 0) bad = 0;
  __syncthreads();
  for (int e = lane; e < nb * nb; e += 64) {
    const int i = e % nb, j = e / nb;
    if (i < j) {
      const double v = 0.5 * (G[i][j] + G[j][i]);
      G[i][j] = v;
      G[j][i] = v;
    }
  }
  __syncthreads();
  if (lane == 0) {
    double tr = 0.0;
    for (int i = 0; i < nb; ++i) tr += G[i][i];
    sig = shift_rel > 0.0 ? shift_rel * tr : 0.0;
  }
  __syncthreads();
  if (lane < nb) G[lane][lane] += sig;
  __syncthreads();
  // Right-looking Cholesky, lower triangle.
  for (int p = 0; p < nb; ++p) {
    if (lane == 0) {
      double piv = G[p][p];
      if (!(piv > 0.0) || !isfinite(piv)) {
        piv = 1.0;
        bad = 1;
      }
      G[p][p] = sqrt(piv);
    }
    __syncthreads();
    if (lane > p && lane < nb) G[lane][p] /= G[p][p];
    __syncthreads();
    if (lane > p && lane < nb)
      for (int j = p + 1; j <= lane; ++j) G[lane][j] -= G[lane][p] * G[j][p];
    __syncthreads();
  }
  // R = L^T (upper); R B into Bt.
  if (lane < nb) {
    for (int i = 0; i < nb; ++i) {
      const double rij = (i <= lane) ? G[lane][i] : 0.0;  // R[i][lane] = L[lane][i]
      Rout[i + lane * nb] = rij;
    }
  }
  __syncthreads();
  if (lane < nb) {
    for (int i = 0; i < nb; ++i) {
      double s;
      if (round == 0) {
        s = (i <= lane) ? G[lane][i] : 0.0;
      } else {
        s = 0.0;
        for (int m = i; m <= lane; ++m) s += G[m][i] * Bacc[m + lane * nb];  // R[i][m] B[m][lane]
      }
      Bt[i][lane] = s;
    }
  }
  __syncthreads();
  if (lane < nb)
    for (int i = 0; i < nb; ++i) Bacc[i + lane * nb] = Bt[i][lane];
  if (lane == 0 && bad) {
    flag[0] |= 1;
    if (flag[1] == 0) flag[1] = tag;
  }
  if (!Brec) return;
  if (lane < nb)
    for (int i = 0; i < nb; ++i) Brec[i + lane * nb] = Bt[i][lane];
  if (lane == 0) {
    double big = 0.0, small = INFINITY;
    for (int i = 0; i < nb; ++i) {
      small = fmin(small, fabs(Bt[i][i]));
      for (int j = 0; j < nb; ++j) big = fmax(big, fmax(fabs(Bt[i][j]), fabs(Arec[i + j * nb])));
    }
    if (!(small > 1e-10 * big)) {
      flag[0] |= 2;
      if (flag[1] == 0) flag[1] = tag;
    }
  }
}

// ---------------------------------------------------------------- launchers
#define LZ_DISPATCH(NBV, CALL) \
  if (NBV <= 4) { constexpr int NB = 4; CALL; }       \
  else if (NBV <= 8) { constexpr int NB = 8; CALL; }  \
  else if (NBV <= 16) { constexpr int NB = 16; CALL; } \
  else if (NBV <= 32) { constexpr int NB = 32; CALL; } \
  else return hipErrorInvalidValue;

int lz_nb_pad(int nb) { return nb <= 4 ? 4 : nb <= 8 ? 8 : nb <= 16 ? 16 : 32; }

size_t lz_proj_part_doubles(int d, int nmax, int nb) {
  return (size_t)lz_nblocks(d, LZ_RC) * nmax * lz_nb_pad(nb);
}
size_t lz_apply_part_doubles(int d, int nmax, int nb) {
  return (size_t)lz_nblocks(nmax, LZ_CC) * lz_nb_pad(nb) * d;
}
size_t lz_gram_part_doubles(int d, int nb) {
  const int p = lz_nb_pad(nb);
  return (size_t)lz_nblocks(d, 256) * p * p;
}

hipError_t lz_project(const double* V, int64_t ldv, int n, double* W, int64_t ldw, int nb, int d,
                      double* C, double* Arec, int b, int accumulate, double* ppart,
                      double* apart, double* gpart, hipStream_t st) {
  const int nrc = lz_nblocks(d, LZ_RC);
  const int ncc = lz_nblocks(n, LZ_CC);
  LZ_DISPATCH(nb, {
    hipLaunchKernelGGL((k_lz_proj_partial<NB>), dim3(lz_nblocks(n, 256 / NB), nrc), dim3(64), 0,
                       st, V, ldv, n, W, ldw, nb, d, ppart);
    hipLaunchKernelGGL(k_lz_proj_finish, dim3(lz_nblocks((int64_t)n * nb, 256)), dim3(256), 0, st,
                       ppart, nrc, n, nb, NB, C, Arec, b, accumulate);
    hipLaunchKernelGGL((k_lz_apply_partial<NB>), dim3(lz_nblocks(d, 256), ncc), dim3(256), 0, st,
                       V, ldv, n, C, nb, d, apart);
    hipLaunchKernelGGL((k_lz_rows<NB>), dim3(lz_nblocks(d, 256)), dim3(256), 0, st, W, ldw, nb, d,
                       apart, ncc, nullptr, W, ldw, gpart);
  })
  return hipGetLastError();
}

hipError_t lz_rows(const double* W, int64_t ldw, int nb, int d, const double* R, double* dst,
                   int64_t ldd, double* gpart, hipStream_t st) {
  LZ_DISPATCH(nb, {
    hipLaunchKernelGGL((k_lz_rows<NB>), dim3(lz_nblocks(d, 256)), dim3(256), 0, st, W, ldw, nb, d,
                       nullptr, 0, R, dst, ldd, gpart);
  })
  return hipGetLastError();
}

hipError_t lz_chol(const double* gpart, int d, int nb, double shift_rel, double* R, double* Bacc,
                   int round, const double* Arec, double* Brec, int* flag, int tag,
                   hipStream_t st) {
  if (nb > 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lz_chol, dim3(1), dim3(64), 0, st, gpart, lz_nblocks(d, 256), nb,
                     lz_nb_pad(nb), shift_rel, R, Bacc, round, Arec, Brec, flag, tag);
  return hipGetLastError();
}

#undef LZ_DISPATCH

}  // namespace refl
