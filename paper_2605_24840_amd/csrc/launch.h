// Host-side launchers of the reflector kernels (implemented in the .hip files).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace refl {

// Epilogue of a symmetric product C = A B (both operands symmetric and
// commuting, so C is symmetric; only upper tiles are multiplied and each is
// mirrored on store).
enum GemmMode {
  GEMM_RESIDUAL = 0,  // T = X X : writes N = I - T, partial ||N||_F^2 per tile
  GEMM_UPDATE = 1,    // P = X N : writes X_new = X + P/2, partial trace per tile
  GEMM_PLAIN_NEG = 2, // C = A B^T by rows (any tile, not symmetric): writes -C
  GEMM_ADJOINT = 3    // adjoint step (launch_adjoint_step_*)
};

// FP64 / FP32 products on 16x16x4 MFMA with tile edge ts in {64, 96, 128}.
// Matrices are dp x dp, leading dimension ld, dp a multiple of ts.  tiles
// holds (I, J) in units of ts (I <= J for the symmetric modes); partials
// receives one FP64 value per tile.  With live != null the launch does
// nothing when *live == 0 (read on the device).
hipError_t launch_sym_gemm_f64(int ts, int mode, const double* A, const double* B,
                               const double* Xold, double* out, int ld, int d, int dp,
                               const int2* tiles, int ntiles, double* partials, hipStream_t st,
                               const int* live = nullptr);
hipError_t launch_sym_gemm_f32(int ts, int mode, const float* A, const float* B, const float* Xold,
                               float* out, int ld, int d, int dp, const int2* tiles, int ntiles,
                               double* partials, hipStream_t st, const int* live = nullptr);
// Blocks of the FP64 (fp64 = 1) or FP32 product with tile edge ts that one
// compute unit holds at once (from their LDS).
int sym_gemm_f_blocks_per_cu(int fp64, int ts);

// Adjoint (reverse) step of eq. NS for symmetric X and Gb, with N = I - X^2
// and Pn = -X Gb (a GEMM_PLAIN_NEG product with A = X, B = Gb over all
// tiles):  out = (Gb + Gb N + N Gb + Pn X)/2
//             = (3 Gb - (Gb X^2 + X Gb X + X^2 Gb))/2,
// symmetric, upper tiles only (mirrored); out must not alias Gb.
hipError_t launch_adjoint_step_f64(int ts, const double* Gb, const double* N, const double* Pn,
                                   const double* X, double* out, int ld, int d, int dp,
                                   const int2* tiles, int ntiles, double* partials,
                                   hipStream_t st);
hipError_t launch_adjoint_step_f32(int ts, const float* Gb, const float* N, const float* Pn,
                                   const float* X, float* out, int ld, int d, int dp,
                                   const int2* tiles, int ntiles, double* partials,
                                   hipStream_t st);

// Grouped products over the upper tiles of many problems (FP64 or FP32): the
// tile list holds (problem, I, J, slot); each problem's descriptor gives its
// iterate pair X[0..1] (element type per `fp64`), N, and sizes.  The tile's
// partial goes to partials[slot].  RESIDUAL reads X[parity] and writes N;
// UPDATE reads X[parity] and N and writes X[parity ^ 1].
struct GemmProblem {
  void* X[2];
  void* N;
  int ld, d, dp, pad;
};
// One launch covers the problems of one tile edge ts (their dp multiples of ts).
// With live != null the tiles of problems p with live[p] == 0 do nothing.
hipError_t launch_sym_gemm_grouped(int fp64, int mode, int ts, const GemmProblem* probs,
                                   const int4* tiles, int ntiles, int parity, double* partials,
                                   const int* live, hipStream_t st);

// Products of matrices held as W BF16 words per entry (planes ps elements
// apart), FP32 accumulation on 32x32x16 BF16 MFMA.  Word products kept:
// W=1 {00}; W=2 {00,01,10}; W=3 {00,01,10,02,11,20}.  tile = 128 or 192
// (192 for W <= 2); tiles in units of `tile`; the matrices are zero outside
// the leading d x d block and K runs over dk = d rounded up to 32.  With
// live != null the launch does nothing when *live == 0 (read on the device).
hipError_t launch_sym_gemm_words(int words, int tile, int mode, const uint16_t* A,
                                 const uint16_t* B, const uint16_t* Xold, uint16_t* out, int ld,
                                 int64_t ps, int d, int dk, const int2* tiles, int ntiles,
                                 double* partials, hipStream_t st, const int* live = nullptr);

// scal[slot] = max_{i<j} |H_ij - H_ji|, scal[slot + 1] = max |H_ij| over the
// full d x d matrix (NaN if any entry is NaN).
hipError_t launch_asym_max(const double* H, int64_t ldh, int d, double* scal, int slot,
                           hipStream_t st);
// ---- set-up: H (upper triangle) -> padded full FP64 copy, scale, X_0 ----
hipError_t launch_mirror_upper(const double* H, int64_t ldh, int d, double* Hf, int dp,
                               hipStream_t st);
// scal[SC_ALPHA] = ||Hf - sI||_inf (norm 0) or ||Hf - sI||_F (norm 1), or
// alpha_given if scale_given; scal[SC_NONFINITE] = count of non-finite.
hipError_t launch_scale_inf(const double* Hf, int dp, int d, double s, int norm, int scale_given,
                            double alpha_given, double* rowsum, double* scal, hipStream_t st);
// X_0 = (Hf - sI)/scal[SC_ALPHA] into FP64, FP32 or W-word storage; partial
// traces per 256-row block into partials (nblk = dp/256 rounded up).
hipError_t launch_init_x0_f64(const double* Hf, int dp, int d, double s, const double* scal,
                              double* X, hipStream_t st);
hipError_t launch_init_x0_f32(const double* Hf, int dp, int d, double s, const double* scal,
                              float* X, hipStream_t st);
// With H32 != null the same pass also writes the FP32 copy of H (dp x dp).
hipError_t launch_init_x0_words(int words, const double* Hf, int dp, int d, double s,
                                const double* scal, uint16_t* X, int64_t ps, float* H32,
                                hipStream_t st);
// FP32 copy of H - sI (the operator of the inner solves).
hipError_t launch_shifted_f32(const double* Hf, int dp, int d, double s, float* Hs,
                              hipStream_t st);
// ---- derivatives ----
// out (dp x dp) = (G + G^T)/2 on the leading d x d block, divided by
// scal[SC_ALPHA] if scal != null; zero padding.  G: d x d, ldg, read in full.
hipError_t launch_sym_in_f64(const double* G, int64_t ldg, int d, const double* scal, double* out,
                             int dp, hipStream_t st);
hipError_t launch_sym_in_f32(const double* G, int64_t ldg, int d, const double* scal, float* out,
                             int dp, hipStream_t st);
// R (d x d, ldr) = X / scal[SC_ALPHA].
hipError_t launch_copy_out_scaled_f64(const double* X, int dp, int d, const double* scal,
                                      double* R, int64_t ldr, hipStream_t st);
hipError_t launch_copy_out_scaled_f32(const float* X, int dp, int d, const double* scal,
                                      double* R, int64_t ldr, hipStream_t st);
// scal[slot] = sum_i A_i B_i over n elements (FP64 sums); partials holds
// dot_partials() doubles.
int dot_partials();
hipError_t launch_dot_f64(const double* A, const double* B, int64_t n, double* partials,
                          double* scal, int slot, hipStream_t st);
hipError_t launch_dot_f32(const float* A, const float* B, int64_t n, double* partials,
                          double* scal, int slot, hipStream_t st);

// ---- shift policy ----
// scal[slot] = ||A - B||_F^2 for the symmetric matrices given by their upper
// triangles; partials: diff_fro_partials(d) doubles.
int diff_fro_partials(int d);
hipError_t launch_diff_fro_upper(const double* A, int64_t lda, const double* B, int64_t ldb, int d,
                                 double* partials, double* scal, int slot, hipStream_t st);
// Upper triangle of B = that of A.
hipError_t launch_copy_upper(const double* A, int64_t lda, double* B, int64_t ldb, int d,
                             hipStream_t st);

// Per-problem descriptor of the batched set-up and output kernels.
struct BatchDesc {
  const double* H;   // input, upper triangle read
  int64_t ldh;
  double* Hf;        // dp x dp FP64 copy of H
  void* X[2];        // iterate pair (FP32 or FP64 per launch)
  double* rowsum;    // 2 dp doubles: row sums, then non-finite flags
  double* scal;      // [SC_ALPHA], [SC_NONFINITE]
  double* R;         // output, d x d, ldr
  int64_t ldr;
  double s, alpha_given;
  int d, dp, scale_given, par;  // par: which X holds the final iterate
  int norm, pad;                // norm of the scale: 0 inf, 1 Frobenius
};
// Blocks of k_batch_init for one problem.
int batch_init_blocks(int dp);
// Set-up of every problem g < ng (the same values as launch_mirror_upper,
// launch_scale_inf, launch_init_x0_* and launch_trace_* per problem): the
// block ranges of the three grouped grids are given by prefix arrays
// (ng + 1 entries) of (dp/64)^2, ceil(d/4) and batch_init_blocks(dp) blocks;
// trace[g] = trace X_0.
hipError_t launch_batch_setup(int fp64, const BatchDesc* desc, int ng, const int* mirror_begin,
                              int mirror_blocks, const int* row_begin, int row_blocks,
                              const int* init_begin, int init_blocks, double* trace,
                              hipStream_t st);
// Copy of X[par] of problems ids[g] (g < ng; ids == null: g) by groups of
// BATCH_COPY_ROWS rows: to_hf == 0 writes R (d rows per problem), to_hf == 1
// the FP64 copy Hf (dp rows); begin is the prefix array of the per-problem
// block counts ceil(rows / BATCH_COPY_ROWS).
constexpr int BATCH_COPY_ROWS = 8;
hipError_t launch_batch_copy(int fp64, const BatchDesc* desc, const int* begin, const int* ids,
                             int ng, int nblocks_total, int to_hf, hipStream_t st);
// Stopping rule of the batched solve evaluated on the device (the rule of
// refl_sign, problem by problem): per-problem limits, and the state of each
// problem's iteration.
struct BatchRule {
  double tol;
  int fixed_steps, max_iter;
};
// Rounding floor of the stopping rule: one step of eq. NS maps each
// eigenvalue x of the symmetric iterate, with e = 1 - x^2, to
// e' = e^2 (3 + e)/4.  ||X^2 - I||_F < 0.2 bounds every |e| by 0.2, so two
// exact steps shrink each e, and the residual, by a factor of at least
// 0.16 x 0.03: a residual below STAG_R that has not halved over two steps is
// the arithmetic's floor, whatever the precision and order, and further
// steps cannot reach a smaller tol.
constexpr double STAG_R = 0.1;
struct BatchStep {
  double h1, h2;      // ||X^2 - I||_F of the previous two steps
  double resid, trace;  // of the last step evaluated
  int m, par, state;  // steps taken; buffer of the final iterate; BATCH_*
  int cert;           // MIXED: steps so far at which the index certificate held
};
constexpr int BATCH_LIVE = 0, BATCH_CONVERGED = 1, BATCH_STOPPED = 2, BATCH_NONFINITE = 3;
// LDS-resident iteration of small problems: one work-group per problem runs
// every Newton-Schulz step with X and N held in LDS, the stopping rule on the
// device, and leaves X_m (the iterate it stops at) in X[m & 1].  On entry
// X[0] holds X_0 (dp x dp, ld = dp, zero outside the leading d x d block)
// and stp[slot].trace = trace X_0; on exit stp[slot] holds the step record
// (state, m, par = m & 1, resid of X_m, trace X_m).  Orders up to
// SMALL_MAX_F32 (FP32) and SMALL_MAX_F64 (FP64), which fit two padded
// matrices in the 160 KiB of LDS of a compute unit.
constexpr int SMALL_MAX_F32 = 128, SMALL_MAX_F64 = 96;
struct SmallProb {
  void* X[2];
  int d, dp, slot, pad;
};
hipError_t launch_ns_small(int fp64, const SmallProb* probs, int nprob, const BatchRule* rules,
                           BatchStep* stp, hipStream_t st);
// One step's decision for every problem with live[p]: resid = sqrt(res[p]),
// trace of X_m from trace[p] (m > 0), then the rule; a problem that stops
// gets live[p] = 0 and par.  ctl[0] is the step m (read, then incremented),
// ctl[1] receives the number of problems still live.
hipError_t launch_batch_decide(int nprob, const double* res, const double* trace,
                               const BatchRule* rules, BatchStep* stp, int* live, int* ctl,
                               int par, hipStream_t st);
// Stopping rule of the MIXED bulk (split-BF16 words), evaluated on the device
// after each residual product; the FP64 correction then restores accuracy.
// Index certificate: with b = sqrt(d) ||X^2 - I||_F < 1 the number j of
// negative eigenvalues of the symmetric iterate is the integer with
// |trace X - (d - 2j)| < 1.  The bulk stops (CONVERGED) at the first step
// where the certificate holds plus `extra` steps, or earlier once it holds
// and the residual no longer falls quadratically (above 1/4 of the previous
// one: the words' rounding floor); it stops without a certificate (STOPPED)
// at the floor of STAG_R, at the step cap, or on a non-finite residual.
struct MixedRule {
  int d, extra, cap, pad;
};
// One step of a single-problem device loop in one launch: scal[SC_RESID2] =
// sum of pr[0..n) = ||X_m^2 - I||_F^2 and, for m = ctl[0] > 0,
// scal[SC_TRACE] = sum of pt[0..n) = trace X_m (both in launch_reduce_sum's
// order; for m = 0 the record holds trace X_0), then one step of the rule:
// the MIXED rule above (MixedRule) or that of launch_batch_decide with
// nprob = 1 (BatchRule).  ctl[0] is m (read, then incremented); live[0] and
// ctl[1] become 0 at the stop, and the record's par then names the buffer
// of X_m.  pr and pt are distinct buffers of n >= 1 doubles.
hipError_t launch_reduce_decide(const double* pr, const double* pt, int n, double* scal,
                                const MixedRule* rule, BatchStep* stp, int* live, int* ctl, int par,
                                hipStream_t st);
hipError_t launch_reduce_decide(const double* pr, const double* pt, int n, double* scal,
                                const BatchRule* rule, BatchStep* stp, int* live, int* ctl, int par,
                                hipStream_t st);
// out[slot ? slot[q] : q] = sum of partials[begin[q] .. begin[q + 1]), q < nq,
// summed in the same order as launch_reduce_sum over that range.
hipError_t launch_reduce_ranges(const double* partials, const int* begin, const int* slot, int nq,
                                double* out, hipStream_t st);
// dst[slot] = sum of partials[0..n) in a fixed order.
hipError_t launch_reduce_sum(const double* partials, int n, double* scal, int slot,
                             hipStream_t st);
// trace of an FP64/FP32/word matrix (diagonal sum) into scal[slot].
hipError_t launch_trace_f64(const double* X, int dp, int d, double* scal, int slot,
                            hipStream_t st);
hipError_t launch_trace_f32(const float* X, int dp, int d, double* scal, int slot,
                            hipStream_t st);
hipError_t launch_trace_words(int words, const uint16_t* X, int64_t ps, int dp, int d,
                              double* scal, int slot, hipStream_t st);

// R (d x d, ldr) from an FP64 / FP32 iterate.
hipError_t launch_copy_out_f64(const double* X, int dp, int d, double* R, int64_t ldr,
                               hipStream_t st);
hipError_t launch_copy_out_f32(const float* X, int dp, int d, double* R, int64_t ldr,
                               hipStream_t st);

// R (d x d, ldr) = sum of the words of a W-word iterate.
hipError_t launch_copy_out_words(int words, const uint16_t* X, int64_t ps, int dp, int d,
                                 double* R, int64_t ldr, hipStream_t st);

// ---- thin products and block-vector kernels (FP64 vectors, column-major) ----
// Y[:, c] = M V[:, c], c < nb <= 32.  work: thin_work_doubles(d) doubles.
size_t thin_work_doubles(int d);
hipError_t thin_gemm_f64(const double* M, int64_t ldm, int d, const double* V, int64_t ldv, int nb,
                         double* Y, int64_t ldy, double* work, hipStream_t st);
hipError_t thin_gemm_f32(const float* M, int64_t ldm, int d, const double* V, int64_t ldv, int nb,
                         double* Y, int64_t ldy, double* work, hipStream_t st);
hipError_t thin_gemm_words(int words, const uint16_t* X, int ld, int64_t ps, int d,
                           const double* V, int64_t ldv, int nb, double* Y, int64_t ldy,
                           double* work, hipStream_t st);
// The same for SYMMETRIC M (faster: column-per-lane, no cross-lane sums).
hipError_t symthin_f64(const double* M, int64_t ldm, int d, const double* V, int64_t ldv, int nb,
                       double* Y, int64_t ldy, double* work, hipStream_t st);
hipError_t symthin_words(int words, const uint16_t* X, int ld, int64_t ps, int d, const double* V,
                         int64_t ldv, int nb, double* Y, int64_t ldy, double* work,
                         hipStream_t st);
// G (na x nb, column-major) = A^T B; work: gram_work_doubles(d) doubles.
size_t gram_work_doubles(int d);
hipError_t gram(const double* A, int64_t lda, int na, const double* B, int64_t ldb, int nb, int d,
                double* G, double* work, hipStream_t st);
// Y = alpha Y + beta A C  (A: d x na, C: na x nb column-major, Y must not alias A).
hipError_t block_axpy(int d, int na, int nb, double alpha, double* Y, int64_t ldy, double beta,
                      const double* A, int64_t lda, const double* C, hipStream_t st);
// Y[:, c] += coef[c] X[:, c]  (coef on the device).
hipError_t col_axpy(int d, int nb, double* Y, int64_t ldy, const double* coef, const double* X,
                    int64_t ldx, hipStream_t st);
// Y = a X + b Y (d x nb blocks).
hipError_t lincomb(int d, int nb, double a, const double* X, int64_t ldx, double b, double* Y,
                   int64_t ldy, hipStream_t st);
// out = c (Z V^T + V Z^T) (d x d, ldo) for d x k blocks Z, V (ld), k <= 32.
hipError_t form_sym_pair(const double* Z, const double* V, int64_t ld, int k, int d, double c,
                         double* out, int64_t ldo, hipStream_t st);
// R = I - 2 V V^T (d x d, ldr).
hipError_t form_reflector(const double* V, int64_t ldv, int k, int d, double* R, int64_t ldr,
                          hipStream_t st);
// V[:, c] uniform in (-1, 1) from a counter-based hash of (seed, c, row).
hipError_t random_block(double* V, int64_t ldv, int d, int nb, uint64_t seed, hipStream_t st);

// ---- block CG (see misc.hip) ----
struct CgHost {
  double theta[32], rho0[32], gam[2][32], alpha[2][32];
  double tol2;
  int iters, done, k, nb;
};
// d x nb blocks (ld = ldv) of one solve: r, p and s alternate between two
// buffers by iteration parity; R[0] holds r_0 and Z = 0 on entry; HR is
// (H - theta) r.  The pipelined solve keeps r in R[0], w = A r in HR, p in
// P[0], the recurrence of A p in P[1], s in S[0], and U = M V (d x k) in U;
// R[1] and S[1] are unused there.
struct CgBufs {
  double* R[2];
  double* P[2];
  double* S[2];
  double* HR;
  double* Z;
  double* U;
};
size_t cg_state_bytes();
size_t cg_part_doubles(int d);
// One CG iteration; `it` counts from 0 within a solve, and a solve runs
// iterations 0 .. max_iter + 1 (the last only tests convergence).  With
// M32 != null the products with H read its FP32 copy M32 (same ldm)
// instead of M.
hipError_t cg_iteration(const double* M, const float* M32, int64_t ldm, int d, int nb,
                        const double* V, int64_t ldv, const CgBufs& bufs, void* state,
                        double* work, double* part, int it, int max_iter, hipStream_t st);
// The same solve by the pipelined recurrences (misc.hip): the pass over M
// of each launch pair multiplies a block known at launch, every reduction
// of an iteration going to the update launch.  k (<= 32) is the number of
// columns of V (k <= nb); iteration 0 also forms U = M V into bufs.U.  Iteration
// counts and the state are as for cg_iteration.
hipError_t cg_pipe_iteration(const double* M, const float* M32, int64_t ldm, int d, int nb, int k,
                             const double* V, int64_t ldv, const CgBufs& bufs, void* state,
                             double* work, double* part, int it, int max_iter, hipStream_t st);

// ---- block Lanczos (see lanczos.hip) ----
// Rows per slab of the Gram partials that the projection writes (the first
// CholQR round reads slabs of this many rows).
constexpr int LZ_GRAM_ROWS = 16;
// Workspace sizes (doubles) for a d-row basis of up to nmax columns and
// blocks of nb <= 32 columns.
int lz_nb_pad(int nb);
size_t lz_proj_part_doubles(int d, int nmax, int nb);
size_t lz_gram_part_doubles(int d, int nb);
// One block Gram-Schmidt pass of W (d x nb) against V (d x n): C = V^T W,
// W <- W - V C.  The rows of C on the last b columns of V go to Arec
// (accumulate: added).  With gpart != null the Gram partials of the new W
// (LZ_GRAM_ROWS-row slabs) are written for lz_cholqr.
hipError_t lz_project(const double* V, int64_t ldv, int n, double* W, int64_t ldw, int nb, int d,
                      double* C, double* Arec, int b, int accumulate, double* ppart,
                      double* gpart, hipStream_t st);
// The second pass of lz_project (n >= 1) with the first, shifted Cholesky
// QR round fused into its update: the Gram matrix factored is the sum of
// gin (LZ_GRAM_ROWS-row slab partials of this pass's input W, as the first
// pass writes them), summed into gsum (lz_nb_pad(nb)^2 doubles) by the
// projection's reduction launch; then W <- (W - V C) R^{-1} with
// R^T R = that sum + shift_rel * trace I, gout = the Gram partials of the
// new W (LZ_GRAM_ROWS-row slabs, for the next lz_cholqr round), Bacc = R,
// and bit 1 of flag[0] (flag[1] = tag if unset) for a replaced pivot.
hipError_t lz_project_qr(const double* V, int64_t ldv, int n, double* W, int64_t ldw, int nb, int d,
                         double* C, double* Arec, int b, int accumulate, double* ppart,
                         const double* gin, double* gsum, double shift_rel, double* Bacc, int* flag,
                         int tag, double* gout, hipStream_t st);
// dst = V Y for the d x n basis V and Y = -Cneg (n x nb, column-major, ld
// n), computed as Wzero - V Cneg with Wzero an all-zero d x nb block of
// leading dimension ldd (the projection kernels' update).
hipError_t lz_combine(const double* V, int64_t ldv, int n, const double* Cneg, int nb, int d,
                      const double* Wzero, double* dst, int64_t ldd, hipStream_t st);
// Gram partials of the LZ_GRAM_ROWS-row slabs of W (d x nb): gpart[slab NB^2 + i + j NB].
hipError_t lz_gram(const double* W, int64_t ldw, int nb, int d, double* gpart, hipStream_t st);
// One Cholesky QR round: factor the summed Gram partials gin (slabs of
// gin_rows = LZ_GRAM_ROWS or 256 rows) (+ shift_rel * trace I) as L L^T,
// dst = W R^{-1} with R = L^T (W and dst may alias), and with gout != null
// (gout != gin) the Gram partials of dst (256-row slabs).  Bacc = R
// (round 0) or R Bacc; see lanczos.hip for Brec and flag (4 ints).
// mode LZ_QR_MAYBE_LAST: when the Gram matrix is within 1e-3 of I this
// round writes dst_last instead of dst, records Arec / Brec and is the last
// one; a following round with LZ_QR_SKIPPABLE then does nothing.
constexpr int LZ_QR_PLAIN = 0, LZ_QR_MAYBE_LAST = 1, LZ_QR_SKIPPABLE = 2;
hipError_t lz_cholqr(const double* gin, int gin_rows, int d, int nb, double shift_rel, double* Bacc,
                     int round, const double* Arec, double* Brec, int* flag, int tag,
                     const double* W, int64_t ldw, double* dst, int64_t ldd, double* gout,
                     int mode, double* dst_last, hipStream_t st);

// ---- allocation-free entry point ----
// Bytes of the fixed per-device scratch array (noalloc.hip) that serves as
// the workspace of refl_sign_noalloc (REFL_NOALLOC_SCRATCH_BYTES in refl.h).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
// Device address of that array on `device`, which must be the current
// device; resolved by hipGetSymbolAddress on the first call per device and
// cached.  Never use the array's name on the host.
hipError_t noalloc_scratch(int device, void** ptr);

}  // namespace refl
