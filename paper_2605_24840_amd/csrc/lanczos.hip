// Kernels of the block-Lanczos shift estimate (the partial-eigensolver route
// of section 4.3).  One Lanczos step, with V = [Q_1 .. Q_j] the d x n basis
// (column-major, ld = ldv) and W = H Q_j from the symmetric thin product:
//
//   two passes of block classical Gram-Schmidt against all of V
//     k_lz_proj_partial / k_lz_proj_finish   C = V^T W   (n x nb)
//     k_lz_apply_rows                        W <- W - V C, row slabs
//   and three rounds of Cholesky QR, the first one shifted (shifted
//   CholQR3 of Fukaya, Kannan, Nakatsukasa, Zhang and Yamamoto, 2020), on
//   the partial Gram matrices of row slabs:
//     round 0          inside the second pass: its reduction launch also
//                      sums the first pass's slab Grams, and its row update
//                      factors that sum (+ shift) and applies R^{-1}
//                      (k_lz_apply_rows<NB, true>; for the start block a
//                      stand-alone k_lz_cholqr round)
//     k_lz_cholqr      rounds 1 and 2: every block sums the slab Grams and
//                      factors G = L L^T itself (the same sum in the same
//                      order, so the same R = L^T), then W <- W R^{-1} on
//                      its slab and the slab Gram of the result for the next
//                      round; block 0 also records B <- R B and the flags
//   so that W_in = Q_{j+1} B_j with B_j upper triangular.
//
// The diagonal block A_j = Q_j^T H Q_j is the last block of the two
// projections, recorded by k_lz_proj_finish.  Every reduction runs in a
// fixed order (per-block partials summed by the next kernel), so the run is
// deterministic.
#include <type_traits>

#include "common.h"
#include "dbg.h"
#include "sync.h"
#include "launch.h"

namespace refl {

REFL_DBG_UNIT(lanczos)

constexpr int LZ_RC = 64;   // rows per block of the projection partials

static inline int lz_nblocks(int64_t n, int per) { return (int)((n + per - 1) / per); }

// part[(rc * n + c) * NB + j] = sum over the rows of chunk rc of V[r, c] W[r, j].
// Block = 256 threads, 64 basis columns x NB (>= 8) block columns; 32-row
// slabs of V and W staged in LDS; thread t owns columns t % 32 and
// t % 32 + 32 and block columns t / 32 + 8 q, q < NB / 8.
template <int NB>
__global__ __launch_bounds__(256) void k_lz_proj_partial(const double* __restrict__ V, int64_t ldv,
                                                         int n, const double* __restrict__ W,
                                                         int64_t ldw, int nb, int d,
                                                         double* __restrict__ part) {
  static_assert(NB >= 8, "block width padded to at least 8");
  constexpr int JQ = NB / 8;
  __shared__ double sV[32][65];
  __shared__ double sW[32][NB + 1];
  const int t = threadIdx.x;
  const int cg = t & 31, jg = t >> 5;
  const int c0 = blockIdx.x * 64;
  const int r0 = blockIdx.y * LZ_RC;
  REFL_GUARD(nb >= 1 && nb <= NB && c0 < n && r0 < d && ldv >= d && ldw >= d, DBG_LZ);
  const int r1 = min(d, r0 + LZ_RC);
  double acc[2][JQ];
#pragma unroll
  for (int q = 0; q < JQ; ++q) acc[0][q] = acc[1][q] = 0.0;
  // The next slab's loads are issued before the current slab is consumed.
  const int lr = t & 31;
  double pv[8], pw[JQ];
  auto load = [&](int rs) {
    const int r = rs + lr;
    const bool in = r < r1;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = c0 + (t >> 5) + 8 * u;
      pv[u] = (in && c < n) ? V[(int64_t)c * ldv + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < JQ; ++u) {
      const int j = (t >> 5) + 8 * u;
      pw[u] = (in && j < nb) ? W[(int64_t)j * ldw + r] : 0.0;
    }
  };
  if (r0 < r1) load(r0);
  for (int rs = r0; rs < r1; rs += 32) {
#pragma unroll
    for (int u = 0; u < 8; ++u) sV[lr][(t >> 5) + 8 * u] = pv[u];
#pragma unroll
    for (int u = 0; u < JQ; ++u) sW[lr][(t >> 5) + 8 * u] = pw[u];
    __syncthreads();
    if (rs + 32 < r1) load(rs + 32);
#pragma unroll 8
    for (int i = 0; i < 32; ++i) {
      const double v0 = sV[i][cg], v1 = sV[i][cg + 32];
#pragma unroll
      for (int q = 0; q < JQ; ++q) {
        const double w = sW[i][jg + 8 * q];
        acc[0][q] = fma(v0, w, acc[0][q]);
        acc[1][q] = fma(v1, w, acc[1][q]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = c0 + cg + 32 * h;
#pragma unroll
    for (int q = 0; q < JQ; ++q) {
      const int j = jg + 8 * q;
      if (c < n && j < nb) part[((int64_t)blockIdx.y * n + c) * NB + j] = acc[h][q];
    }
  }
}

// C[c + j n] = sum_rc part (fixed order).  The rows c >= n - b of C (the
// coefficients on the newest block Q_j) are written to, or with `accumulate`
// added to, Arec (b x b, column-major).  Four lanes per entry: lane q sums
// the chunks rc = q mod 4 in order (sixteen loads in flight), and the four
// sums are combined by a fixed butterfly, so every lane holds the same value.
//
// Blocks from cblocks on (when gsrc != null) sum instead the gslab slab
// Gram partials gsrc (NB x NB each, entry i + j NB) into gdst (same
// layout): sixteen lanes per entry, lane q summing the slabs q mod 16 in
// order (one round of sixteen loads for 256 slabs), then a fixed butterfly.
__global__ __launch_bounds__(256) void k_lz_proj_finish(const double* __restrict__ part, int nrc,
                                                        int n, int nb, int NB,
                                                        double* __restrict__ C,
                                                        double* __restrict__ Arec, int b,
                                                        int accumulate, int cblocks,
                                                        const double* __restrict__ gsrc,
                                                        int gslab, double* __restrict__ gdst) {
  REFL_GUARD(nb >= 1 && nb <= NB, DBG_LZ);
  if ((int)blockIdx.x >= cblocks) {
    const int g2 = ((int)blockIdx.x - cblocks) * 256 + (int)threadIdx.x;
    const int q = g2 & 15, o = g2 >> 4;
    const bool in = o < nb * nb;
    const int i = in ? o % nb : 0, j = in ? o / nb : 0;
    const double* p = gsrc + i + (int64_t)j * NB;
    const int64_t st = (int64_t)NB * NB;
    double s = 0.0;
    if (in) {
      int sl = q;
      for (; sl + 240 < gslab; sl += 256) {
        double a[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) a[u] = p[(int64_t)(sl + 16 * u) * st];
#pragma unroll
        for (int u = 0; u < 16; ++u) s += a[u];
      }
      for (; sl < gslab; sl += 16) s += p[(int64_t)sl * st];
    }
    s += __shfl_xor(s, 1, WAVE);
    s += __shfl_xor(s, 2, WAVE);
    s += __shfl_xor(s, 4, WAVE);
    s += __shfl_xor(s, 8, WAVE);
    if (in && q == 0) gdst[i + (int64_t)j * NB] = s;
    return;
  }
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int q = (int)(g & 3);
  const int64_t o = g >> 2;
  const bool in = o < (int64_t)n * nb;
  // Entries run fastest over j, so a wave's loads share cache lines (the
  // partials are stored [chunk][c][j]).
  const int c = in ? (int)(o / nb) : 0, j = in ? (int)(o % nb) : 0;
  double s = 0.0;
  if (in) {
    int rc = q;
    for (; rc + 60 < nrc; rc += 64) {
      double a[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) a[u] = part[((int64_t)(rc + 4 * u) * n + c) * NB + j];
#pragma unroll
      for (int u = 0; u < 16; ++u) s += a[u];
    }
    for (; rc + 28 < nrc; rc += 32) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = part[((int64_t)(rc + 4 * u) * n + c) * NB + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += a[u];
    }
    for (; rc < nrc; rc += 4) s += part[((int64_t)rc * n + c) * NB + j];
  }
  s += __shfl_xor(s, 1, WAVE);
  s += __shfl_xor(s, 2, WAVE);
  if (!in || q != 0) return;
  C[c + (int64_t)j * n] = s;
  if (Arec && c >= n - b) {
    double* a = Arec + (c - (n - b)) + (int64_t)j * b;
    *a = accumulate ? *a + s : s;
  }
}

// LDS state of a Cholesky factorisation by lz_chol (below).
struct LzChol {
  double G[32][33];
  double red[2];
  double dev;
  double inv[32];
  double col[64];
  int bad;
};
template <int NBP, typename F>
__device__ void lz_chol(int nb, double shift_rel, F& f);

// W <- W - V C on 16-row slabs (V: d x n basis, ld ldv; C: n x nb,
// column-major, ld n).  A block is 16 rows x AG column groups (AG = 32, or
// 16 for blocks wider than 16 columns): a lane owns one row and takes the
// columns g, g + AG, ... of each 256-column chunk of C, which passes through
// LDS; the groups' sums meet in LDS and are added in group order (a fixed
// order), so no column partials go through memory.  The result goes to dst
// (which may be W: the block reads its rows before writing them), and with
// gpart != null the slab's Gram matrix x^T x goes to
// gpart[blockIdx.x NB^2 + i + j NB].  n = 0 only copies W and forms the Gram
// partials.  Short slabs give many blocks: one compute unit streams its
// share of V (16 rows of n columns) quickly, where 64-row slabs left 64
// blocks of 64 n 8 bytes each on a 256-unit device.
//
// With QR the block also runs the first, shifted round of Cholesky QR on
// the result x: it factors gfac + sigma I = L L^T (gfac: a summed nb x nb
// Gram matrix, entry i + j NB; sigma = shift_rel trace gfac) while its loads
// are in flight, and dst and the Gram partials then hold y = x R^{-1}
// (R = L^T).  Block 0 records Bacc = R and, for a replaced pivot, bit 1 of
// flag[0] (flag[1] = tag if unset).  The second Gram-Schmidt pass passes
// the Gram matrix of its input (the first pass's output, x + V C): in exact
// arithmetic that is x^T x + C^T C with C = V^T (x + V C) of rounding size,
// a positive semidefinite perturbation that the shift already dominates,
// so the round keeps the conditioning bound of shifted Cholesky QR and one
// Gram reduction (a kernel boundary) per step is saved.
constexpr int LZ_AR = LZ_GRAM_ROWS;
constexpr int LZ_ACH = 256;  // columns of C per LDS chunk
template <int NB>
constexpr int lz_ag() { return NB <= 16 ? 32 : 16; }
template <int NB, bool QR>
__global__ __launch_bounds__(LZ_AR * lz_ag<NB>()) void k_lz_apply_rows(
    const double* __restrict__ V, int64_t ldv, int n, const double* __restrict__ C, int nb, int d,
    const double* W, int64_t ldw, double* dst, int64_t ldd, double* __restrict__ gpart,
    const double* __restrict__ gfac, double shift_rel, double* __restrict__ Bacc,
    int* __restrict__ flag, int tag) {
  constexpr int AG = lz_ag<NB>(), NT = LZ_AR * AG;
  __shared__ double sC[LZ_ACH][NB];
  __shared__ double sP[AG][LZ_AR][NB + 1];
  __shared__ double sX[LZ_AR][NB + 1];
  __shared__ typename std::conditional<QR, LzChol, char>::type fc;
  const int t = threadIdx.x, row = t % LZ_AR, g = t / LZ_AR;
  const int r0 = blockIdx.x * LZ_AR, r = r0 + row;
  REFL_GUARD(nb >= 1 && nb <= NB && r0 < d && ldv >= d, DBG_LZ);
  // With QR, the summed Gram matrix is requested first (it is needed
  // first), then the slab of W (LZ_AR x NB) and the first chunk of C; masked
  // loads without branches (a load in a branch is waited for where the
  // branch ends).
  constexpr int PERG = QR ? (NB * NB + NT - 1) / NT : 1;
  double gv[PERG];
  if constexpr (QR) {
#pragma unroll
    for (int u = 0; u < PERG; ++u) {
      const int e = t + u * NT;
      const double v = gfac[e < NB * NB ? e : 0];
      gv[u] = (e < NB * NB && e % NB < nb && e / NB < nb) ? v : 0.0;
    }
  }
  constexpr int PERW = (LZ_AR * NB + NT - 1) / NT;
  double wv[PERW];
#pragma unroll
  for (int u = 0; u < PERW; ++u) {
    const int o = t + u * NT, rr = r0 + o % LZ_AR, q = o / LZ_AR;
    const double v = W[(int64_t)min(q, nb - 1) * ldw + min(rr, d - 1)];
    wv[u] = (o < LZ_AR * NB && rr < d && q < nb) ? v : 0.0;
  }
  // Chunk cb of C (256 rows of nb columns) into cv; up to 16 columns the
  // next chunk is requested while the current one is used (wider blocks
  // have no registers to spare for it).
  constexpr bool PREFETCH = NB <= 16;
  constexpr int PERC = (LZ_ACH * NB + NT - 1) / NT;
  auto load_chunk = [&](int cb, double (&cv)[PERC]) {
    const int cn = min(LZ_ACH, n - cb);
#pragma unroll
    for (int u = 0; u < PERC; ++u) {
      const int e = t + u * NT, cl = e / NB, q = e % NB;
      const bool ok = e < LZ_ACH * NB && cl < cn && q < nb;
      const double v = C[ok ? (cb + cl) + (int64_t)q * n : 0];
      cv[u] = ok ? v : 0.0;
    }
  };
  auto store_chunk = [&](const double (&cv)[PERC]) {
#pragma unroll
    for (int u = 0; u < PERC; ++u) {
      const int e = t + u * NT;
      if (e < LZ_ACH * NB) sC[e / NB][e % NB] = cv[u];
    }
  };
  double cvp[PREFETCH ? PERC : 1];
  if constexpr (PREFETCH) {
    if (n > 0) load_chunk(0, cvp);
  }
  if constexpr (QR) {
    // The factorisation needs none of the block's rows: wave 0 runs it
    // while the loads of W and C are in flight (the barrier orders LDS
    // only; the chunk loop's first block barrier orders its result for the
    // other waves).
#pragma unroll
    for (int u = 0; u < PERG; ++u) {
      const int e = t + u * NT;
      if (e < NB * NB) fc.G[e % NB][e / NB] = gv[u];
    }
    if (t == 0) fc.bad = 0;
    lds_barrier();
    lz_chol<NB>(nb, shift_rel, fc);
  }
  double acc[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) acc[q] = 0.0;
  for (int cb = 0; cb < n; cb += LZ_ACH) {
    const int cn = min(LZ_ACH, n - cb);
    if constexpr (PREFETCH) {
      __syncthreads();
      store_chunk(cvp);
      __syncthreads();
      if (cb + LZ_ACH < n) load_chunk(cb + LZ_ACH, cvp);
    } else {
      double cv[PERC];
      load_chunk(cb, cv);
      __syncthreads();
      store_chunk(cv);
      __syncthreads();
    }
    if (r < d) {
      const double* v = V + (int64_t)cb * ldv + r;
      int cl = g;
      for (; cl + 7 * AG < cn; cl += 8 * AG) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = v[(int64_t)(cl + u * AG) * ldv];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int q = 0; q < NB; ++q) acc[q] = fma(x[u], sC[cl + u * AG][q], acc[q]);
      }
      for (; cl < cn; cl += AG) {
        const double x = v[(int64_t)cl * ldv];
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[q] = fma(x, sC[cl][q], acc[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) sP[g][row][q] = acc[q];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PERW; ++u) {
    const int o = t + u * NT;
    if (o < LZ_AR * NB) {
      const int rw = o % LZ_AR, q = o / LZ_AR, rr = r0 + rw;
      double sum = 0.0;
      for (int gg = 0; gg < AG; ++gg) sum += sP[gg][rw][q];
      const double x = wv[u] - sum;
      sX[rw][q] = x;
      if (!QR && dst && rr < d && q < nb) dst[(int64_t)q * ldd + rr] = x;
    }
  }
  if constexpr (QR) {
    // y R = x, one row per lane of the first LZ_AR lanes (R[i][j] = L[j][i]).
    __syncthreads();
    if (t < LZ_AR) {
      double y[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) y[j] = sX[t][j];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < nb) {
          double s = y[j];
#pragma unroll
          for (int i = 0; i < j; ++i) s = fma(-y[i], fc.G[j][i], s);
          y[j] = s * fc.inv[j];
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) sX[t][j] = y[j];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PERW; ++u) {
      const int o = t + u * NT;
      const int rw = o % LZ_AR, q = o / LZ_AR, rr = r0 + rw;
      if (o < LZ_AR * NB && rr < d && q < nb) dst[(int64_t)q * ldd + rr] = sX[rw][q];
    }
    if (blockIdx.x == 0) {
      for (int e = t; e < nb * nb; e += NT) {
        const int i = e % nb, j = e / nb;
        Bacc[e] = i <= j ? fc.G[j][i] : 0.0;
      }
      if (t == 0 && fc.bad) {
        flag[0] |= 1;
        if (flag[1] == 0) flag[1] = tag;
      }
    }
  }
  if (!gpart) return;
  __syncthreads();
  for (int o = t; o < nb * nb; o += NT) {
    const int i = o % nb, jj = o / nb;
    double a = 0.0;
#pragma unroll
    for (int rw = 0; rw < LZ_AR; ++rw) a = fma(sX[rw][i], sX[rw][jj], a);
    gpart[(int64_t)blockIdx.x * NB * NB + i + jj * NB] = a;
  }
}

// Shared state of one Cholesky QR round.
struct LzFactor {
  double G[32][33];
  double Bo[32][33];
  double Bt[32][33];
  double red[5];
  double dev;  // ||G - I||_F of the summed Gram matrix, before shift and factorisation
  double inv[32];  // 1 / L[j][j]
  double col[64];  // the column of multipliers of one Cholesky step
  int bad;
};

// Orders the LDS accesses of one wave (the hardware completes them in
// order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// All threads of the block.  G = sum of the slab Gram matrices gpart
// (nblk slabs of NBP x NBP, fixed order), symmetrised, plus sigma I with
// sigma = shift_rel * trace(G) when shift_rel > 0; then G = L L^T in place
// (lower triangle; R = L^T).  A non-positive pivot is replaced by 1 and
// f.bad set.  With load_bo, f.Bo = Bacc (nb x nb, column-major).
template <int NBP>
__device__ void lz_factor(const double* __restrict__ gpart, int nblk, int nb,
                          double shift_rel, const double* __restrict__ Bacc, bool load_bo,
                          LzFactor& f) {
  const int t = threadIdx.x;
  // Thread t sums entry t (and t + 256, ...) over the slabs: 64 loads in
  // flight per round, accumulated round-robin into four sums.
  for (int e = t; e < nb * nb; e += 256) {
    const int i = e % nb, j = e / nb;
    const double* g = gpart + i + j * NBP;
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    int b = 0;
    for (; b + 64 <= nblk; b += 64) {
      double a[64];
#pragma unroll
      for (int u = 0; u < 64; ++u) a[u] = g[(int64_t)(b + u) * NBP * NBP];
#pragma unroll
      for (int u = 0; u < 64; ++u) s4[u & 3] += a[u];
    }
    for (; b + 32 <= nblk; b += 32) {
      double a[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) a[u] = g[(int64_t)(b + u) * NBP * NBP];
#pragma unroll
      for (int u = 0; u < 32; ++u) s4[u & 3] += a[u];
    }
    for (; b + 16 <= nblk; b += 16) {
      double a[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) a[u] = g[(int64_t)(b + u) * NBP * NBP];
#pragma unroll
      for (int u = 0; u < 16; ++u) s4[u & 3] += a[u];
    }
    for (; b + 4 <= nblk; b += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) s4[u] += g[(int64_t)(b + u) * NBP * NBP];
    }
    for (; b < nblk; ++b) s4[0] += g[(int64_t)b * NBP * NBP];
    f.G[i][j] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    if (load_bo) f.Bo[i][j] = Bacc[i + j * nb];
  }
  if (t == 0) f.bad = 0;
  __syncthreads();
  lz_chol<NBP>(nb, shift_rel, f);
  __syncthreads();
}

// The work of wave 0 alone on f.G (nb x nb, already summed), its steps
// ordered by wavefront fences (LDS accesses of one wave complete in order)
// instead of block barriers: symmetrise, trace and ||G - I||_F (lane sums,
// then a fixed butterfly), the shift, the Cholesky factorisation and the
// reciprocals of its diagonal.  f.bad must be 0 on entry.  The caller
// orders the result for the other waves with a block barrier.
template <int NBP, typename F>
__device__ void lz_chol(int nb, double shift_rel, F& f) {
  const int t = threadIdx.x;
  if (t < 64) {
    for (int e = t; e < nb * nb; e += 64) {
      const int i = e % nb, j = e / nb;
      if (i < j) {
        const double v = 0.5 * (f.G[i][j] + f.G[j][i]);
        f.G[i][j] = v;
        f.G[j][i] = v;
      }
    }
    wave_fence();
    double tr = 0.0, dv = 0.0;
    for (int e = t; e < nb * nb; e += 64) {
      const int i = e % nb, j = e / nb;
      const double g = f.G[i][j], x = g - (i == j ? 1.0 : 0.0);
      if (i == j) tr += g;
      dv += x * x;
    }
    tr = wave_sum(tr);
    dv = wave_sum(dv);
    const double sh = shift_rel > 0.0 ? shift_rel * tr : 0.0;
    if (t == 0) {
      f.red[0] = sh;
      f.dev = sqrt(dv);
    }
    if (t < nb) f.G[t][t] += sh;
    wave_fence();
    // Right-looking Cholesky, lower triangle: lane t < nb keeps row t in
    // registers; the pivot and the new column reach the other lanes through
    // LDS (one write and one broadcast read each per pivot).  The steps are
    // unrolled over the padded width; a step past nb is skipped whole.
    const int tr_ = t < nb ? t : nb - 1;
    double row[NBP];
#pragma unroll
    for (int j = 0; j < NBP; ++j) row[j] = f.G[tr_][j];
#pragma unroll
    for (int p = 0; p < NBP; ++p) {
      const bool act = p < nb;
      if (!act) continue;  // uniform: steps past nb are skipped whole
      if (t == p && act) {
        double piv = row[p];
        if (!(piv > 0.0) || !isfinite(piv)) {
          piv = 1.0;
          f.bad = 1;
        }
        f.red[1] = sqrt(piv);
      }
      wave_fence();
      const double dg = f.red[1];
      const bool below = act && t > p && t < nb;
      const double l = below ? row[p] / dg : 0.0;
      if (act && t == p) row[p] = dg;
      if (below) row[p] = l;
      f.col[t] = l;
      wave_fence();
#pragma unroll
      for (int j = p + 1; j < NBP; ++j) row[j] = fma(-l, f.col[j], row[j]);
      wave_fence();
    }
    if (t < nb) {
#pragma unroll
      for (int j = 0; j < NBP; ++j)
        if (j <= t) f.G[t][j] = row[j];
    }
    wave_fence();
    if (t < nb) f.inv[t] = 1.0 / f.G[t][t];
  }
}

// Block 0 of a round.  Bacc = R (round 0) or R Bacc.  bit 1 of flag[0] for
// a replaced pivot.  With Brec != null (the last round of a Lanczos step),
// Bacc is also copied to Brec, and if its smallest diagonal entry is below
// 1e-10 times the largest entry of Arec or Bacc, bit 2 of flag[0] is set
// (the block Krylov space has become, to working accuracy, invariant).
// flag[1] keeps the first `tag` (the step number) at which a bit was set.
__device__ void lz_record(int nb, int round, double* __restrict__ Bacc,
                          const double* __restrict__ Arec, double* __restrict__ Brec,
                          int* __restrict__ flag, int tag, LzFactor& f) {
  const int t = threadIdx.x;
  // One entry (i, c) of the new B per thread (the sum over m in the same
  // order as one thread per column would take it).
  for (int e = t; e < nb * nb; e += 256) {
    const int i = e % nb, c = e / nb;
    double s;
    if (round == 0) {
      s = (i <= c) ? f.G[c][i] : 0.0;  // R[i][c] = L[c][i]
    } else {
      s = 0.0;
      for (int m = i; m <= c; ++m) s += f.G[m][i] * f.Bo[m][c];  // R[i][m] B[m][c]
    }
    f.Bt[i][c] = s;
  }
  __syncthreads();
  for (int e = t; e < nb * nb; e += 256) {
    const int i = e % nb, j = e / nb;
    Bacc[i + j * nb] = f.Bt[i][j];
    if (Brec) Brec[i + j * nb] = f.Bt[i][j];
  }
  if (t == 0 && f.bad) {
    flag[0] |= 1;
    if (flag[1] == 0) flag[1] = tag;
  }
  if (!Brec) return;
  double big = 0.0;
  for (int e = t; e < nb * nb; e += 256) {
    const int i = e % nb, j = e / nb;
    big = fmax(big, fmax(fabs(f.Bt[i][j]), fabs(Arec[i + j * nb])));
  }
  big = wave_max(big);
  if ((t & 63) == 0) f.red[1 + (t >> 6)] = big;
  __syncthreads();
  if (t == 0) {
    big = fmax(fmax(f.red[1], f.red[2]), fmax(f.red[3], f.red[4]));
    double small = INFINITY;
    for (int i = 0; i < nb; ++i) small = fmin(small, fabs(f.Bt[i][i]));
    if (!(small > 1e-10 * big)) {
      flag[0] |= 2;
      if (flag[1] == 0) flag[1] = tag;
    }
  }
}

// One Cholesky QR round on 256-row slabs (one row per thread): factor the
// Gram of W from gin, dst = W R^{-1}, and with gout != null the slab Gram
// partials of dst.  W and dst may be the same block (each thread reads its
// row before writing it); gin and gout must differ.
//
// The third round of shifted CholQR3 is needed only when the block was
// ill-conditioned: with mode LZ_QR_MAYBE_LAST (the second round) a Gram
// matrix within LZ_QR_DONE of I (Frobenius) makes this round the last one:
// it writes dst_last, records Arec / Brec and sets flag[2] = tag + 1 (else
// 0), and a third round launched with LZ_QR_SKIPPABLE then returns at once.  (The
// input's condition number is then below 1.01, so one CholQR round leaves
// it orthonormal to working accuracy.)  Every block sums the same partials
// in the same order, so every block takes the same branch.
constexpr double LZ_QR_DONE = 1e-3;
template <int NB>
__global__ __launch_bounds__(256) void k_lz_cholqr(const double* __restrict__ gin, int nblk,
                                                   int nb, double shift_rel,
                                                   double* __restrict__ Bacc, int round,
                                                   const double* __restrict__ Arec,
                                                   double* __restrict__ Brec,
                                                   int* __restrict__ flag, int tag,
                                                   const double* W, int64_t ldw, int d,
                                                   double* dst, int64_t ldd,
                                                   double* __restrict__ gout, int mode,
                                                   double* dst_last) {
  if (mode == LZ_QR_SKIPPABLE && flag[2] == tag + 1) return;
  REFL_GUARD(nb >= 1 && nb <= NB, DBG_LZ);
  __shared__ LzFactor f;
  __shared__ double sX[256][NB + 1];
  const int r = blockIdx.x * 256 + threadIdx.x;
  // The slab's rows are requested before the factorisation, which does not
  // depend on them.
  double x[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) x[j] = (r < d && j < nb) ? W[(int64_t)j * ldw + r] : 0.0;
  const bool rec = blockIdx.x == 0;
  lz_factor<NB>(gin, nblk, nb, shift_rel, Bacc, rec && round > 0, f);
  __syncthreads();
  const bool last_now = mode == LZ_QR_MAYBE_LAST && f.dev < LZ_QR_DONE;
  if (mode == LZ_QR_MAYBE_LAST) {
    if (rec && threadIdx.x == 0) flag[2] = last_now ? tag + 1 : 0;
    if (last_now) {
      dst = dst_last;
      gout = nullptr;
    } else {
      Arec = nullptr;
      Brec = nullptr;
    }
  }
  if (rec) lz_record(nb, round, Bacc, Arec, Brec, flag, tag, f);
  // x R = w for upper-triangular R = L^T: R[i][j] = G[j][i].
  if (r < d) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (j < nb) {
        double s = x[j];
#pragma unroll
        for (int i = 0; i < j; ++i) s = fma(-x[i], f.G[j][i], s);
        x[j] = s * f.inv[j];
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (j < nb) dst[(int64_t)j * ldd + r] = x[j];
  }
  if (!gout) return;
#pragma unroll
  for (int j = 0; j < NB; ++j) sX[threadIdx.x][j] = x[j];
  __syncthreads();
  for (int o = threadIdx.x; o < nb * nb; o += 256) {
    const int i = o % nb, j = o / nb;
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (int t = 0; t < 256; ++t) a4[t & 3] = fma(sX[t][i], sX[t][j], a4[t & 3]);
    gout[(int64_t)blockIdx.x * NB * NB + i + j * NB] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  }
}

// ---------------------------------------------------------------- launchers
#define LZ_DISPATCH(NBV, CALL) \
  if (NBV <= 8) { constexpr int NB = 8; CALL; }       \
  else if (NBV <= 16) { constexpr int NB = 16; CALL; } \
  else if (NBV <= 32) { constexpr int NB = 32; CALL; } \
  else return hipErrorInvalidValue;

int lz_nb_pad(int nb) { return nb <= 8 ? 8 : nb <= 16 ? 16 : 32; }

size_t lz_proj_part_doubles(int d, int nmax, int nb) {
  return (size_t)lz_nblocks(d, LZ_RC) * nmax * lz_nb_pad(nb);
}
size_t lz_gram_part_doubles(int d, int nb) {
  const int p = lz_nb_pad(nb);
  return (size_t)lz_nblocks(d, LZ_AR) * p * p;   // LZ_AR-row slabs (256-row for the later rounds)
}

hipError_t lz_project(const double* V, int64_t ldv, int n, double* W, int64_t ldw, int nb, int d,
                      double* C, double* Arec, int b, int accumulate, double* ppart,
                      double* gpart, hipStream_t st) {
  const int nrc = lz_nblocks(d, LZ_RC);
  const int cblocks = lz_nblocks((int64_t)n * nb * 4, 256);
  LZ_DISPATCH(nb, {
    hipLaunchKernelGGL((k_lz_proj_partial<NB>), dim3(lz_nblocks(n, 64), nrc), dim3(256), 0, st, V,
                       ldv, n, W, ldw, nb, d, ppart);
    hipLaunchKernelGGL(k_lz_proj_finish, dim3(cblocks), dim3(256), 0, st, ppart, nrc, n, nb, NB, C,
                       Arec, b, accumulate, cblocks, nullptr, 0, nullptr);
    hipLaunchKernelGGL((k_lz_apply_rows<NB, false>), dim3(lz_nblocks(d, LZ_AR)),
                       dim3(LZ_AR * lz_ag<NB>()), 0, st, V, ldv, n, C, nb, d, W, ldw, W, ldw, gpart,
                       nullptr, 0.0, nullptr, nullptr, 0);
  })
  return hipGetLastError();
}

hipError_t lz_project_qr(const double* V, int64_t ldv, int n, double* W, int64_t ldw, int nb, int d,
                         double* C, double* Arec, int b, int accumulate, double* ppart,
                         const double* gin, double* gsum, double shift_rel, double* Bacc, int* flag,
                         int tag, double* gout, hipStream_t st) {
  if (n < 1 || !gin || !gsum || !gout || gin == gout) return hipErrorInvalidValue;
  const int nrc = lz_nblocks(d, LZ_RC);
  const int cblocks = lz_nblocks((int64_t)n * nb * 4, 256);
  const int gblocks = lz_nblocks((int64_t)nb * nb * 16, 256);
  LZ_DISPATCH(nb, {
    hipLaunchKernelGGL((k_lz_proj_partial<NB>), dim3(lz_nblocks(n, 64), nrc), dim3(256), 0, st, V,
                       ldv, n, W, ldw, nb, d, ppart);
    hipLaunchKernelGGL(k_lz_proj_finish, dim3(cblocks + gblocks), dim3(256), 0, st, ppart, nrc, n,
                       nb, NB, C, Arec, b, accumulate, cblocks, gin, lz_nblocks(d, LZ_AR), gsum);
    hipLaunchKernelGGL((k_lz_apply_rows<NB, true>), dim3(lz_nblocks(d, LZ_AR)),
                       dim3(LZ_AR * lz_ag<NB>()), 0, st, V, ldv, n, C, nb, d, W, ldw, W, ldw, gout,
                       gsum, shift_rel, Bacc, flag, tag);
  })
  return hipGetLastError();
}

hipError_t lz_combine(const double* V, int64_t ldv, int n, const double* Cneg, int nb, int d,
                      const double* Wzero, double* dst, int64_t ldd, hipStream_t st) {
  LZ_DISPATCH(nb, {
    hipLaunchKernelGGL((k_lz_apply_rows<NB, false>), dim3(lz_nblocks(d, LZ_AR)),
                       dim3(LZ_AR * lz_ag<NB>()), 0, st, V, ldv, n, Cneg, nb, d, Wzero, ldd, dst, ldd,
                       nullptr, nullptr, 0.0, nullptr, nullptr, 0);
  })
  return hipGetLastError();
}

hipError_t lz_gram(const double* W, int64_t ldw, int nb, int d, double* gpart, hipStream_t st) {
  LZ_DISPATCH(nb, {
    hipLaunchKernelGGL((k_lz_apply_rows<NB, false>), dim3(lz_nblocks(d, LZ_AR)),
                       dim3(LZ_AR * lz_ag<NB>()), 0, st, nullptr, ldw, 0, nullptr, nb, d, W, ldw,
                       nullptr, ldw, gpart, nullptr, 0.0, nullptr, nullptr, 0);
  })
  return hipGetLastError();
}

hipError_t lz_cholqr(const double* gin, int gin_rows, int d, int nb, double shift_rel, double* Bacc,
                     int round, const double* Arec, double* Brec, int* flag, int tag,
                     const double* W, int64_t ldw, double* dst, int64_t ldd, double* gout,
                     int mode, double* dst_last, hipStream_t st) {
  if (gin == gout || (gin_rows != LZ_AR && gin_rows != 256)) return hipErrorInvalidValue;
  if (mode < LZ_QR_PLAIN || mode > LZ_QR_SKIPPABLE || (mode == LZ_QR_MAYBE_LAST && !dst_last))
    return hipErrorInvalidValue;
  LZ_DISPATCH(nb, {
    hipLaunchKernelGGL((k_lz_cholqr<NB>), dim3(lz_nblocks(d, 256)), dim3(256), 0, st, gin,
                       lz_nblocks(d, gin_rows), nb, shift_rel, Bacc, round, Arec, Brec, flag, tag, W,
                       ldw, d, dst, ldd, gout, mode, dst_last);
  })
  return hipGetLastError();
}

#undef LZ_DISPATCH

}  // namespace refl
