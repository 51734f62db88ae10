/*
 * refl.h -- prescribed-index reflectors R_k = I - 2 P_k = sgn(H - sI) of a
 * dense symmetric matrix on one MI355X (gfx950), by the shifted
 * Newton-Schulz matrix-sign iteration.
 *
 * Problem statement (paper, section 1 eq. Rk_intro and section 2.1 eq. Pk):
 * H in R^{d x d} symmetric with eigenvalues lambda_1 <= ... <= lambda_d,
 * k in {1, ..., d-1}, P_k the spectral projector onto the eigenvectors of the
 * k smallest eigenvalues.  For any shift s in (lambda_k, lambda_{k+1}),
 * R_k = sgn(H - sI) (Prop. 2.1).  R_k is computed by the scaled iteration
 * X_0 = (H - sI)/alpha, X_{m+1} = X_m (3I - X_m^2)/2 (section 3.3, eq. NS),
 * with the midpoint shift s = (lambda_k + lambda_{k+1})/2 (Prop. 4.1)
 * supplied or estimated by block Lanczos (section 4.3, recommended default
 * realization), and alpha = ||H - sI||_inf (the cheap surrogate of
 * section 4.3) or a supplied value.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - Pointers named d* are DEVICE pointers on the handle's device; they are
 *   owned by the caller and never freed or retained by the library.
 * - Matrices are dense FP64, row-major with a leading dimension >= d.
 *   H is read from its UPPER triangle only (entries (i, j), i <= j); the
 *   strictly lower triangle is never read.  R is written in full and is
 *   exactly symmetric.  Blocks of vectors V, Y are d x nrhs, column-major
 *   (column c starts at V + c*ldv, ldv >= d).
 * - All device work is enqueued on the handle's HIP stream.  refl_sign,
 *   refl_sign_apply, refl_sign_batched and refl_estimate_shift synchronise
 *   that stream before returning (their info outputs live on the host);
 *   refl_apply does not.
 * - A handle is not thread-safe; use one handle per host thread.  Calls on
 *   one handle are serialised by its stream.
 * - Errors are reported only through refl_status_t; nothing throws or aborts
 *   across this boundary.  refl_last_error(h) gives a message for the last
 *   failing call on h.  On REFL_ERR_NOT_CONVERGED, R holds the last iterate
 *   and info is complete; on any other error the outputs are unspecified.
 */
#ifndef REFL_H_
#define REFL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct refl_handle_s *refl_handle_t;

typedef enum {
  REFL_OK = 0,
  REFL_ERR_INVALID_ARG = 1,    /* null pointer, d < 2, k outside 1..d-1, ld < d, bad mode */
  REFL_ERR_DEVICE = 2,         /* a HIP runtime call failed */
  REFL_ERR_NO_MEMORY = 3,      /* workspace allocation failed or caller workspace too small */
  REFL_ERR_NOT_CONVERGED = 4,  /* max_iter reached before the stopping rule held */
  REFL_ERR_NOT_ADMISSIBLE = 5, /* the iterate's index certificate found j != k negatives,
                                  or the Lanczos margin test of Prop. 4.2 failed */
  REFL_ERR_NO_GAP = 6,         /* lambda_k == lambda_{k+1} to working precision */
  REFL_ERR_NOT_SYMMETRIC = 7,  /* params.check_symmetric: max |H_ij - H_ji| exceeds
                                  params.sym_tol times max |H_ij| (section 2.1 takes H
                                  symmetric; by default only the upper triangle is read and
                                  this is not checked) */
  REFL_ERR_UNSUPPORTED = 8,    /* valid request the library does not implement */
  REFL_ERR_NOT_FINITE = 9,     /* H (or the shift/scale) holds a NaN or an infinity */
  REFL_ERR_BOUNDS = 10         /* debug build only: a kernel's launch-extent guard tripped
                                  (refl_last_error names the kernel); outputs are undefined */
} refl_status_t;

/* Arithmetic of the Newton-Schulz matrix products. */
typedef enum {
  REFL_PREC_FP64 = 0,  /* FP64 MFMA products, FP64 iterate: the plain method */
  REFL_PREC_FP32 = 1,  /* FP32 MFMA products, FP32 iterate (error floor ~1e-5 relative) */
  REFL_PREC_MIXED = 2  /* products on split-BF16 words with FP32 accumulation, then an
                          FP64 correction of the target subspace that uses H itself */
} refl_precision_t;

typedef enum { REFL_SHIFT_GIVEN = 0, REFL_SHIFT_LANCZOS = 1 } refl_shift_mode_t;

typedef enum {
  REFL_SCALE_INF = 0,    /* alpha = ||H - sI||_inf (max absolute row sum) */
  REFL_SCALE_FRO = 1,    /* alpha = ||H - sI||_F, another cheap bound on the spectral
                            radius of H - sI (looser than the inf-norm for spread spectra,
                            tighter for a few dominant eigenvalues) */
  REFL_SCALE_LANCZOS = 2,/* alpha = 1.05 rho_hat with rho_hat the Lanczos estimate of
                            max_i |lambda_i - s| (the spectral-norm scaling of section 4.3);
                            needs shift_mode == REFL_SHIFT_LANCZOS */
  REFL_SCALE_GIVEN = 3   /* alpha = params.alpha; X_0 = (H - sI)/alpha */
} refl_scale_mode_t;

typedef struct {
  int32_t k;            /* target index, 1 <= k <= d-1 (section 2.1); 0 with a given
                           shift: no target, the certified index j of the iterate is
                           reported in info.index_j and R = sgn(H - sI) is returned for
                           it (no admissibility test against k) */
  double s;             /* shift (shift_mode == REFL_SHIFT_GIVEN) */
  int32_t shift_mode;   /* refl_shift_mode_t */
  int32_t scale_mode;   /* refl_scale_mode_t */
  int32_t precision;    /* refl_precision_t */
  double alpha;         /* scale (scale_mode == REFL_SCALE_GIVEN), must exceed 0 */
  double tol;           /* FP64/FP32: stop when ||X^2 - I||_F < tol; a residual below 0.1
                           that has not halved over two steps is the arithmetic's floor
                           (exact steps shrink it far more), and the iteration stops there
                           with REFL_ERR_NOT_CONVERGED.
                           MIXED: stop the FP64 correction when the certified bound on
                           ||R - R_k||_F falls below tol */
  int32_t max_iter;     /* cap on Newton-Schulz steps (default 100) */
  int32_t fixed_steps;  /* > 0: exactly this many steps, no convergence test: the
                           finite-step filter p_m of eq. pm (FP64/FP32 only) */
  int32_t words;        /* MIXED: BF16 words per operand the bulk starts with: 1 (bf16),
                           2 (bf16x3, default) or 3 (bf16x6); see words_max */
  int32_t polish_sweeps;/* MIXED: maximum FP64 correction sweeps (default 2) */
  double cg_tol;        /* MIXED: relative residual target of the inner solves (default 1e-6) */
  int32_t cg_max_iter;  /* MIXED: cap on inner iterations per sweep (default 400) */
  int32_t lanczos_steps;/* REFL_SHIFT_LANCZOS: cap on block steps (0 = automatic) */
  uint64_t seed;        /* start blocks of Lanczos and of the subspace extraction */
  int32_t timing;       /* 1: record HIP events around every bulk product and report their
                           summed durations in info (adds no synchronisation); N > 1: in
                           the MIXED bulk, only around the products of every N-th step
                           (a sample: each event pair costs the device some microseconds) */
  int32_t grad_mode;    /* refl_sign_grad: REFL_GRAD_REVERSE (default) or REFL_GRAD_TANGENT */
  int32_t ckpt_every;   /* refl_sign_grad, reverse mode: keep every c-th iterate and
                           recompute the others.  0: keep every iterate and its N = I - X^2
                           when 2 (step cap + 1) d^2 elements fit in 16 GiB, else
                           c = ceil(sqrt(step cap)) */
  int32_t cg_f32;       /* MIXED: operator precision of the inner solves, refl_cg_prec_t
                           (default REFL_CG_AUTO) */
  int32_t check_symmetric; /* 1: before any other work, read H in full and return
                           REFL_ERR_NOT_SYMMETRIC if max_{i<j} |H_ij - H_ji| > sym_tol
                           max_ij |H_ij| (a NaN anywhere also fails).  0 (default): only
                           the upper triangle is read, the lower is never touched.
                           One extra pass over H (d^2 doubles).  refl_sign, refl_sign_apply,
                           refl_sign_grad and each problem of refl_sign_batched */
  double sym_tol;       /* check_symmetric: relative tolerance, >= 0 (default 0: exact) */
  int32_t words_max;    /* MIXED: largest word count the bulk may move to (default 3; 0 or
                           words: no change).  A bulk that ends without the index
                           certificate, or (k given) certifies another index, is run
                           again with one more word per operand; with a Lanczos shift and
                           an estimated scaled margin gamma below 5e-6 the bulk starts
                           with three words.  info.bulk_words reports the count used */
} refl_params_t;

typedef enum {
  REFL_CG_FP64 = 0, /* the inner solves read H in FP64 */
  REFL_CG_FP32 = 1, /* they read an FP32 copy of H (half the bytes per iteration; a solve
                       then corrects to about u32 alpha / (s - theta_max) relative, while
                       the Rayleigh-Ritz step and the certificate of every sweep use H in
                       FP64, so the bound and the result stay FP64-certified) */
  REFL_CG_AUTO = 2  /* FP32 when u32 alpha / (s - theta_max) < 1e-3 at the first sweep,
                       else FP64 */
} refl_cg_prec_t;

typedef enum {
  REFL_GRAD_REVERSE = 0, /* reverse sweep over checkpointed iterates */
  REFL_GRAD_TANGENT = 1  /* forward tangent in direction G, carried beside the iteration
                            (no checkpoints; equal to the gradient because the derivative
                            of X -> p_m(X) is self-adjoint) */
} refl_grad_mode_t;

typedef struct {
  int32_t ns_steps;       /* Newton-Schulz steps taken */
  int32_t polish_sweeps;  /* MIXED: correction sweeps taken */
  int32_t cg_iters;       /* MIXED: inner iterations, summed over sweeps */
  int32_t index_j;        /* number of negative eigenvalues certified for the iterate
                             (-1 if the certificate did not hold) */
  int32_t lanczos_steps;  /* block Lanczos steps (shift estimated) */
  double s;               /* shift used */
  double alpha;           /* scale used: X_0 = (H - sI)/alpha */
  double lam_k, lam_k1;   /* Lanczos estimates of lambda_k, lambda_{k+1} (NaN if s given) */
  double eps;             /* Lanczos residual bound on both estimates (Prop. 4.2) */
  double margin;          /* certified shift margin m_hat - eps (Prop. 4.2), NaN if s given */
  double resid_fro;       /* ||X^2 - I||_F of the last bulk iterate */
  double trace;           /* trace of the last bulk iterate */
  double commutator_fro;  /* MIXED: ||H R - R H||_F of the returned R (= 2 sqrt2 ||E||_F,
                             E = (I - V V^T) H V); FP64/FP32: NaN */
  double dk_bound;        /* MIXED: Davis-Kahan bound on ||R - R_k||_F; FP64/FP32: NaN */
  double ms_setup, ms_bulk, ms_polish, ms_total; /* host wall-clock per phase */
  double ms_gemm;         /* params.timing: summed device time of the bulk products (HIP events) */
  int32_t gemm_launches;  /* params.timing: number of bulk product launches timed */
  double rho;             /* Lanczos estimate of max_i |lambda_i - s| (NaN if s given) */
  double gamma;           /* estimated scaled margin min(s - lam_k, lam_k1 - s)/alpha
                             (section 3.3 gamma, from the Lanczos estimates; NaN if s given) */
  int32_t bulk_tile;      /* edge of the square output tiles of the bulk products */
  int32_t bulk_words;     /* MIXED: BF16 words per operand of the bulk that produced the
                             result (params.words, or the automatic choice) */
} refl_info_t;

/* Fill *p with defaults: k = 1, s = 0, shift given, scale inf-norm, FP64,
 * tol = 1e-12, max_iter = 100, fixed_steps = 0, words = 2, polish_sweeps = 2,
 * cg_tol = 1e-6, cg_max_iter = 400, lanczos_steps = 0, seed = 0, timing = 0,
 * grad_mode = REFL_GRAD_REVERSE, ckpt_every = 0, cg_f32 = REFL_CG_AUTO,
 * check_symmetric = 0, sym_tol = 0, words_max = 3. */
refl_status_t refl_params_default(refl_params_t *p);

/* Create a handle bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t, or NULL for the device's null stream).  Allocates no
 * device memory. */
refl_status_t refl_create(refl_handle_t *h, int device, void *hip_stream);

/* Release the handle and any workspace the library allocated itself.  Waits
 * for the handle's stream first. */
refl_status_t refl_destroy(refl_handle_t h);

refl_status_t refl_set_stream(refl_handle_t h, void *hip_stream);

/* Bytes of device workspace refl_sign / refl_sign_apply need for order d
 * and parameters *p.  With shift_mode = REFL_SHIFT_LANCZOS this includes the
 * Lanczos basis (d x (cap + 1) b doubles), and covers refl_estimate_shift
 * for the same d, k and lanczos_steps. */
refl_status_t refl_workspace_size(refl_handle_t h, int64_t d, const refl_params_t *p,
                                  size_t *bytes);

/* Hand the library a caller-owned device workspace (256-byte aligned).  If
 * none is set, or it is too small, the library allocates its own and keeps
 * it until refl_destroy.  Passing NULL reverts to the library's own. */
refl_status_t refl_set_workspace(refl_handle_t h, void *dptr, size_t bytes);

/* Shift estimation by block Lanczos with full reorthogonalisation on H
 * (section 4.3, recommended default realization: a partial eigensolver near
 * the target gap; Prop. 4.1 midpoint; Prop. 4.2 margin test).
 *
 * Block width b = min(k + 4, 32, d), start block from the SplitMix64 hash of
 * (seed, column, row) mapped to (-1, 1), at most floor(d / b) block steps
 * (`steps` > 0 lowers that cap).  After step ceil((k + 1) / b), then every
 * ceil(64 / b) steps and at the cap, the Ritz values theta of the block
 * tridiagonal projection and the residual norms ||H x - theta x|| of the
 * Ritz pairs k and k+1 are formed; the run stops once
 * eps = max(res_k, res_k+1) < (theta_k+1 - theta_k) / 4.
 *
 * Outputs: *lam_k, *lam_k1 the Ritz values theta_k, theta_k+1; *eps the
 * residual bound (each estimate lies within eps of an eigenvalue of H:
 * |lam_hat - lam| <= eps when the Ritz values are attributed to the right
 * eigenvalues, which the index certificate of refl_sign then confirms);
 * *s = (lam_k + lam_k1)/2; *rho = max(theta_max - s, s - theta_min), an
 * estimate (from below) of max_i |lambda_i - s|.  The outputs are written
 * also on REFL_ERR_NOT_ADMISSIBLE and REFL_ERR_NO_GAP.
 *
 * Status: REFL_OK when the margin m_hat = min(s - lam_k, lam_k1 - s)
 * exceeds eps (Prop. 4.2), REFL_ERR_NOT_ADMISSIBLE when it does not at the
 * step cap, REFL_ERR_NO_GAP when the two estimates coincide.  REFL_OK
 * certifies the shift only under the premise of Prop. 4.2 that theta_k and
 * theta_k+1 estimate lambda_k and lambda_k+1: a residual radius holds SOME
 * eigenvalue, and an eigenvalue below theta_k+1 that the Krylov space
 * missed (multiplicity above b, a start block deficient in its direction)
 * would put s in another gap.  refl_sign's index certificate (exactly k
 * negative eigenvalues of the iterate) is what confirms the index; the
 * shift policies inherit the same premise.  Device
 * workspace: as refl_workspace_size for shift_mode = REFL_SHIFT_LANCZOS. */
refl_status_t refl_estimate_shift(refl_handle_t h, int64_t d, const double *dH, int64_t ldh,
                                  int32_t k, int32_t steps, uint64_t seed, double *s,
                                  double *lam_k, double *lam_k1, double *eps, double *rho);

/* R_k = sgn(H - sI) into dR (d x d, leading dimension ldr).  info may be
 * NULL.  See refl_params_t for the modes.
 *
 * FP32 orders d <= 128 and FP64 orders d <= 96 run every Newton-Schulz step
 * of eq. NS in one launch, with X and X^2 - I held in on-chip memory and the
 * stopping rule evaluated on the device (same rule, same results up to
 * rounding as the tiled products larger orders use; with params.timing that
 * launch is the one timed).  The environment variable REFL_SMALL=0 sends
 * them through the tiled products instead. */
refl_status_t refl_sign(refl_handle_t h, int64_t d, const double *dH, int64_t ldh,
                        const refl_params_t *p, double *dR, int64_t ldr, refl_info_t *info);

/* Bytes of the fixed device scratch that serves as the workspace of
 * refl_sign_noalloc on each device (64 MiB). */
#define REFL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* refl_sign for callers that cannot allocate memory: serving loops that must
 * not call hipMalloc between requests, harnesses that forbid allocation, and
 * code that records the caller's own work around the call.  Same arguments,
 * computation, results and status codes as refl_sign, except:
 * - The workspace is a fixed array of REFL_NOALLOC_SCRATCH_BYTES in device
 *   memory that the library holds on every device it runs on, from the first
 *   refl_create on that device until the process ends.  Nothing inside the
 *   call allocates or frees device or pinned host memory or creates events:
 *   the pinned staging and the events it needs come with the handle
 *   (refl_create).  A workspace set with refl_set_workspace is not used.
 * - Every call on a device shares that device's array, across handles: calls
 *   that overlap on one device (two host threads, or two streams) race and
 *   give undefined results.  The array keeps the last call's contents; a
 *   call reads nothing it has not written itself.
 * - Limit: when refl_workspace_size(h, d, p) exceeds REFL_NOALLOC_SCRATCH_BYTES
 *   the call returns REFL_ERR_INVALID_ARG before any device work (about
 *   d <= 1400 in FP64, 1800 in FP32, 1500 MIXED with a given shift; less with
 *   shift_mode = REFL_SHIFT_LANCZOS, whose basis is another 8 d^2 bytes).
 * - params.timing (which creates events) gives REFL_ERR_INVALID_ARG.
 * - FP64/FP32 orders whose tile edge the autotuner has not yet timed in this
 *   process (a refl_sign call does that once per order) take the edge of its
 *   cost model; every entry of R is the same sum in the same order for every
 *   edge, only the grouping of the residual's tile sums may differ.
 * - REFL_ERR_DEVICE if refl_create could not resolve the array's address. */
refl_status_t refl_sign_noalloc(refl_handle_t h, int64_t d, const double *dH, int64_t ldh,
                                const refl_params_t *p, double *dR, int64_t ldr,
                                refl_info_t *info);

/* Y = R V for a d x d matrix R (full storage, row-major, ldr >= d) and a
 * d x nrhs block V; the direction d = -R g of eq. discrete_step and
 * Prop. 3.3 is refl_apply with V = -g.  Asynchronous. */
refl_status_t refl_apply(refl_handle_t h, int64_t d, const double *dR, int64_t ldr,
                         int64_t nrhs, const double *dV, int64_t ldv, double *dY, int64_t ldy);

/* Y = R_k V without writing R: the same computation as refl_sign, then the
 * product with the d x nrhs block V. */
refl_status_t refl_sign_apply(refl_handle_t h, int64_t d, const double *dH, int64_t ldh,
                              const refl_params_t *p, int64_t nrhs, const double *dV,
                              int64_t ldv, double *dY, int64_t ldy, refl_info_t *info);

/* Reflectors of nprob independent problems in one call (the batched dense
 * regime of the section on computational regime and complexity: many
 * moderate-size Hessians make full-matrix products efficient).
 *
 * Arguments are HOST arrays of length nprob: d[p], the device pointers
 * dH[p] / dR[p] with leading dimensions ldh[p] / ldr[p] (each as in
 * refl_sign), and params[p].  Every problem must use the same precision,
 * REFL_PREC_FP64 or REFL_PREC_FP32, and a given shift (shift_mode
 * REFL_SHIFT_GIVEN); k, s, scale, tol, max_iter and fixed_steps may differ.
 * MIXED or a Lanczos shift gives REFL_ERR_UNSUPPORTED.
 *
 * Each Newton-Schulz product runs as one grouped launch over the upper tiles
 * of every problem still iterating; problems of the orders refl_sign runs in
 * one launch (FP32 d <= 128, FP64 d <= 96) run there instead, one work-group
 * each, beside the grouped launches.  Each problem stops by refl_sign's rule
 * and its R (and steps, scale, trace) equal, bit for bit, those of refl_sign
 * with params[p].  In FP32 the certificate ||X^2 - I||_F reported in
 * info[p].resid_fro and used for info[p].index_j is recomputed in FP64 from
 * the final FP32 iterate.  info[p].ms_* and ms_gemm are batch-wide.
 *
 * info and status (length nprob, host) may be NULL.  status[p] is what
 * refl_sign would return for problem p.  Returns REFL_OK if every problem
 * succeeded, else the status of the first problem that did not (its index
 * is in refl_last_error); argument errors are returned before any work.
 * Device workspace: refl_sign_batched_workspace_size (the sum over the
 * problems of about 28 dp^2 bytes in FP32 or 32 dp^2 in FP64, dp = d[p]
 * rounded up to 128). */
refl_status_t refl_sign_batched(refl_handle_t h, int32_t nprob, const int64_t *d,
                                const double *const *dH, const int64_t *ldh,
                                const refl_params_t *params, double *const *dR,
                                const int64_t *ldr, refl_info_t *info, refl_status_t *status);
refl_status_t refl_sign_batched_workspace_size(refl_handle_t h, int32_t nprob, const int64_t *d,
                                               const refl_params_t *params, size_t *bytes);

/* Gradient of L(H) = <G, R_m(H)> (Frobenius inner product) for the reflector
 * R_m = p_m((H - sI)/alpha) that refl_sign computes (eq. NS, eq. pm; m its
 * step count), with respect to SYMMETRIC perturbations of H, the shift s and
 * the scale alpha held fixed.  Only the symmetric part of G matters; G is
 * d x d FP64 (ldg), read in full.
 *
 * FP64 / FP32: the forward pass is refl_sign's with the same steps and
 * stopping rule (a Lanczos shift gives REFL_ERR_UNSUPPORTED).  The
 * derivative follows the steps of eq. NS exactly (product rule), in the
 * bulk precision:
 *   reverse  Gb_m = sym(G); Gb_j = (3 Gb - (Gb X_j^2 + X_j Gb X_j + X_j^2 Gb))/2
 *            with Gb = Gb_{j+1}; gradient = Gb_0 / alpha.  The forward's X_j
 *            and N_j are all kept when they fit (see ckpt_every), else X_j
 *            every c steps, recomputed segment by segment; the gradient is
 *            the same bit for bit.
 *   tangent  Xdot_0 = sym(G)/alpha, Xdot_{j+1} = the same map applied to Xdot_j
 *            beside the forward steps; gradient = Xdot_m.
 * Per step the derivative costs one general and one symmetric three-term
 * product (5 d^3 flops) against 2 d^3 for the forward step.
 *
 * MIXED: the gradient of the limit L(H) = <G, R_k(H)> = <G, sgn(H - sI)>,
 * which is what the MIXED forward returns (fixed_steps must be 0; the shift
 * may be given or estimated, R_k not depending on it).  The forward is
 * refl_sign's MIXED solve; its certified basis V of the target eigenspace and
 * Ritz values theta then give the derivative of sgn in Daleckii-Krein form,
 * self-adjoint, applied to sym(G):
 *   gradient = 2 (Z V^T + V Z^T),
 *   (I - V V^T)(H - theta_c I)(I - V V^T) z_c = (I - V V^T) sym(G) v_c,
 * solved by block CG with H in FP64 to a relative residual of 1e-10 (at
 * most 4 cg_max_iter iterations, else REFL_ERR_NOT_CONVERGED with the
 * gradient written); the operator is positive definite on the complement of
 * V.  loss = tr G - 2 tr(V^T sym(G) V).  info.cg_iters and ms_polish
 * include the gradient solve.  The workspace is refl_sign's (sym(G) is
 * stored over the bulk's word planes once the forward is done).
 *
 * Outputs: dGrad (d x d, ldgr, symmetric), *loss = <G, R_m> (may be NULL),
 * and R_m into dR (ldr) unless dR is NULL.  Status and info as refl_sign.
 * Device workspace is allocated by the library, in dp^2 elements of the bulk
 * precision (dp = d rounded up to the tile, cap = fixed_steps or max_iter):
 * about 2 (cap + 1) + 8 when every iterate is kept (ckpt_every = 0, reverse
 * mode, and that fits in 16 GiB: sized for the cap, not the steps taken),
 * else about ceil(cap / c) + 2c + 8 for checkpoints every c steps.  A
 * caller that must bound memory passes ckpt_every > 0 (or a smaller
 * max_iter). */
refl_status_t refl_sign_grad(refl_handle_t h, int64_t d, const double *dH, int64_t ldh,
                             const refl_params_t *p, const double *dG, int64_t ldg,
                             double *dGrad, int64_t ldgr, double *loss, double *dR, int64_t ldr,
                             refl_info_t *info);

/* Shift policies over a sequence of Hessians H_0, H_1, ... (Alg. 4.3 step 4,
 * with the certificates of Prop. 4.2).  A policy object keeps the state of
 * the sequence; refl_policy_shift returns the shift for the current H.
 *
 *   MIDPOINT  every call estimates lam_k, lam_k+1 and eps by block Lanczos
 *             (as refl_estimate_shift) and returns the midpoint (Prop. 4.1).
 *   DAMPED    every call estimates; s = (1 - beta) s_prev + beta midpoint,
 *             clipped into [lam_k + eps + c w, lam_k+1 - eps - c w] with
 *             w = (lam_k+1 - lam_k)/2 - eps the certified half-width and
 *             c = clip in (0, 1]; the first call returns the midpoint.
 *   REUSE     (reuse/refresh) the shift of the last refresh is kept while its
 *             certified margin at the current H,
 *               min(s - lam_k, lam_k+1 - s) - eps - ||H - H_ref||_F
 *             (Prop. 4.2 with the Weyl bound, the drift measured from the
 *             Hessian H_ref of the last refresh), exceeds tau times the
 *             estimated half-gap of that refresh; otherwise the call
 *             refreshes: it estimates on H, returns the new midpoint and
 *             keeps a device copy of H's upper triangle as H_ref.
 *
 * A returned shift is certified admissible (REFL_OK) when its margin (in
 * info) is positive; otherwise the status is REFL_ERR_NOT_ADMISSIBLE (or
 * REFL_ERR_NO_GAP from the estimate) and the policy keeps no state from the
 * call.  The policy owns a d x d FP64 device copy (REUSE only), with
 * warm_start a d x b block (b = min(k + 4, 32, d)), and is tied to the
 * handle's device; calls on one policy are not thread-safe.
 *
 * Warm start: on a slowly varying sequence the previous refresh's Ritz
 * vectors span the wanted eigenvectors of the current H to about the drift
 * over the gap, so the run needs few steps.  The estimate and its
 * certificate do not depend on the start block (a failed warm run is
 * repeated from the seeded block). */
typedef enum {
  REFL_POLICY_MIDPOINT = 0,
  REFL_POLICY_DAMPED = 1,
  REFL_POLICY_REUSE = 2
} refl_policy_mode_t;

typedef struct refl_policy_s *refl_policy_t;

typedef struct {
  int32_t mode;           /* refl_policy_mode_t */
  int32_t k;              /* target index, 1 <= k <= d-1 */
  double beta;            /* DAMPED: weight of the new midpoint, 0 < beta <= 1 */
  double clip;            /* DAMPED: 0 < clip <= 1 (see above) */
  double tau;             /* REUSE: 0 <= tau < 1 */
  int32_t lanczos_steps;  /* cap on block Lanczos steps per refresh (0 = automatic) */
  uint64_t seed;          /* Lanczos start block */
  int32_t warm_start;     /* 1: each refresh after the first starts block Lanczos from the
                             Ritz vectors of the b smallest Ritz values of the previous
                             refresh (same d); 0: from the seeded block every time */
} refl_policy_params_t;

typedef struct {
  double s;               /* shift returned */
  double lam_k, lam_k1;   /* estimates in force (from this call or the last refresh) */
  double eps;             /* their residual bound */
  double margin;          /* certified margin of s at this H (Prop. 4.2) */
  double drift;           /* REUSE: ||H - H_ref||_F (NaN on a refresh and in other modes) */
  int32_t refreshed;      /* 1 if this call ran block Lanczos */
  int32_t lanczos_steps;  /* block steps of this call's estimate (0 if reused) */
  int32_t calls, refreshes; /* totals over the policy's life */
} refl_policy_info_t;

refl_status_t refl_policy_create(refl_handle_t h, const refl_policy_params_t *pp,
                                 refl_policy_t *out);
refl_status_t refl_policy_destroy(refl_policy_t pol);
/* Shift for the current H (d x d FP64, upper triangle, ldh).  info may be
 * NULL.  Device work runs on the handle's stream, which is synchronised. */
refl_status_t refl_policy_shift(refl_handle_t h, refl_policy_t pol, int64_t d, const double *dH,
                                int64_t ldh, double *s, refl_policy_info_t *info);

/* Static strings; never NULL. */
const char *refl_status_string(refl_status_t s);
const char *refl_last_error(refl_handle_t h);

/* 1 if this library is the bounds-checked debug build (compiled with
 * -DREFL_DEBUG), else 0.  In that build every guarded kernel checks on
 * entry that the tiles, rows, K-slices and block columns it touches lie
 * inside the extents it was launched with; a block that fails returns
 * before any memory access and records the kernel.  Each entry point that
 * runs device work then synchronises the handle's stream, reads and clears
 * the records, and returns REFL_ERR_BOUNDS if one is set.  Not a check of
 * the paper's mathematics: a development aid, slower than the release
 * build by one stream synchronisation per call. */
int refl_debug_build(void);

#ifdef __cplusplus
}
#endif
#endif /* REFL_H_ */
