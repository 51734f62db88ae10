// Memory-bound kernels around the Newton-Schulz products: set-up of the
// scaled iterate (section 3.3 eq. NS with the inf-norm scaling of section
// 4.3), reductions, output, and the thin products and block-vector updates
// of the FP64 subspace correction and of block Lanczos.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "dbg.h"
#include "sync.h"
#include "launch.h"
#include "rule.h"

namespace refl {

REFL_DBG_UNIT(misc)

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------- set-up
// Hf (dp x dp, ld dp) = symmetric matrix whose upper triangle is that of H,
// zero outside the leading d x d block.  Block (bx, by) handles the 64 x 64
// tile (I, J) = (by, bx); tiles with I > J are written by their mirror.
__device__ __forceinline__ void mirror_tile(const double* __restrict__ H, int64_t ldh, int d,
                                            double* __restrict__ Hf, int dp, int I, int J,
                                            double (*t)[65]) {
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int i0 = I * 64, j0 = J * 64;
  for (int r = ty; r < 64; r += 4) {
    const int i = i0 + r, j = j0 + tx;
    double v = 0.0;
    if (i < d && j < d && i <= j) v = H[(int64_t)i * ldh + j];
    t[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int i = i0 + r, j = j0 + tx;
    // Diagonal tile: lower part from the upper part.
    const double v = (I == J && r > tx) ? t[tx][r] : t[r][tx];
    Hf[(int64_t)i * dp + j] = v;
  }
  if (I != J) {
    for (int r = ty; r < 64; r += 4) Hf[(int64_t)(j0 + r) * dp + i0 + tx] = t[tx][r];
  }
}

__global__ __launch_bounds__(256) void k_mirror_upper(const double* __restrict__ H, int64_t ldh,
                                                      int d, double* __restrict__ Hf, int dp) {
  const int I = blockIdx.y, J = blockIdx.x;
  if (I > J) return;
  REFL_GUARD(J * 64 < dp && d <= dp && ldh >= d, DBG_MIRROR);
  __shared__ double t[64][65];
  mirror_tile(H, ldh, d, Hf, dp, I, J, t);
}

// rowsum[i] = sum_j |Hf_ij - s delta_ij| (norm 0) or sum_j (Hf_ij - s delta_ij)^2
// (norm 1), one wave per row; counts non-finite entries.
__device__ __forceinline__ void rowabs_row(const double* __restrict__ Hf, int dp, int d, double s,
                                           int norm, double* __restrict__ rowsum,
                                           double* __restrict__ nonfinite_rows, int row) {
  const int lane = threadIdx.x & 63;
  if (row >= d) return;
  const double* h = Hf + (int64_t)row * dp;
  double acc = 0.0;
  int bad = 0;
  for (int j = lane; j < d; j += 64) {
    double v = h[j];
    if (!isfinite(v)) bad = 1;
    if (j == row) v -= s;
    acc += norm ? v * v : fabs(v);
  }
  acc = wave_sum(acc);
  const double nb = wave_sum((double)bad);
  if (lane == 0) {
    rowsum[row] = acc;
    nonfinite_rows[row] = nb;
  }
}

__global__ __launch_bounds__(256) void k_rowabs(const double* __restrict__ Hf, int dp, int d,
                                                double s, int norm, double* __restrict__ rowsum,
                                                double* __restrict__ nonfinite_rows) {
  REFL_GUARD(d <= dp, DBG_ROWABS);
  rowabs_row(Hf, dp, d, s, norm, rowsum, nonfinite_rows, blockIdx.x * 4 + (threadIdx.x >> 6));
}

// scal[SC_ALPHA] = max rowsum (norm 0: the inf-norm) or sqrt(sum rowsum)
// (norm 1: the Frobenius norm), or alpha_given; scal[SC_NONFINITE] = sum of
// the flags.
__device__ __forceinline__ void scale_finish_block(const double* __restrict__ rowsum,
                                                   const double* __restrict__ nonfinite_rows,
                                                   int d, int norm, int scale_given,
                                                   double alpha_given, double* __restrict__ scal,
                                                   double* red, double* redb) {
  double m = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) {
    m = norm ? m + rowsum[i] : fmax(m, rowsum[i]);
    b += nonfinite_rows[i];
  }
  m = norm ? wave_sum(m) : wave_max(m);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
    red[w] = m;
    redb[w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double mx = norm ? sqrt((red[0] + red[1]) + (red[2] + red[3]))
                           : fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    scal[SC_ALPHA] = scale_given ? alpha_given : mx;
    scal[SC_NONFINITE] = (redb[0] + redb[1]) + (redb[2] + redb[3]);
  }
}

__global__ __launch_bounds__(256) void k_scale_finish(const double* __restrict__ rowsum,
                                                      const double* __restrict__ nonfinite_rows,
                                                      int d, int norm, int scale_given,
                                                      double alpha_given,
                                                      double* __restrict__ scal) {
  __shared__ double red[4], redb[4];
  scale_finish_block(rowsum, nonfinite_rows, d, norm, scale_given, alpha_given, scal, red, redb);
}

// X = (Hf - sI)/alpha on the elements first, first + stride, ... < end.
template <typename T>
__device__ __forceinline__ void init_x0_elems(const double* __restrict__ Hf, int dp, int d,
                                              double s, double inv, T* __restrict__ X,
                                              int64_t first, int64_t end, int64_t stride) {
  for (int64_t idx = first; idx < end; idx += stride) {
    const int i = (int)(idx / dp), j = (int)(idx % dp);
    double v = Hf[idx];
    if (i == j && i < d) v -= s;
    X[idx] = (T)(v * inv);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_init_x0(const double* __restrict__ Hf, int dp, int d,
                                                 double s, const double* __restrict__ scal,
                                                 T* __restrict__ X) {
  REFL_GUARD(d <= dp, DBG_INIT_X0);
  const double inv = 1.0 / scal[SC_ALPHA];
  init_x0_elems(Hf, dp, d, s, inv, X, (int64_t)blockIdx.x * 256 + threadIdx.x, (int64_t)dp * dp,
                (int64_t)gridDim.x * 256);
}

// With H32 != null it also writes the FP32 copy of H (unshifted) that the
// correction's inner solves read, saving that pass its own read of H.
template <int W>
__global__ __launch_bounds__(256) void k_init_x0_w(const double* __restrict__ Hf, int dp, int d,
                                                   double s, const double* __restrict__ scal,
                                                   uint16_t* __restrict__ X, int64_t ps,
                                                   float* __restrict__ H32) {
  REFL_GUARD(d <= dp && ps >= (int64_t)dp * dp, DBG_INIT_X0);
  const int64_t n = (int64_t)dp * dp;
  const double inv = 1.0 / scal[SC_ALPHA];
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx / dp), j = (int)(idx % dp);
    double v = Hf[idx];
    if (H32) H32[idx] = (float)v;
    if (i == j && i < d) v -= s;
    uint16_t w[W];
    split_words<W>((float)(v * inv), w);
#pragma unroll
    for (int q = 0; q < W; ++q) X[q * ps + idx] = w[q];
  }
}

__global__ __launch_bounds__(256) void k_shifted_f32(const double* __restrict__ Hf, int dp, int d,
                                                     double s, float* __restrict__ Hs) {
  REFL_GUARD(d <= dp, DBG_SHIFTED_F32);
  const int64_t n = (int64_t)dp * dp;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx / dp), j = (int)(idx % dp);
    double v = Hf[idx];
    if (i == j && i < d) v -= s;
    Hs[idx] = (float)v;
  }
}

// ------------------------------------------------------------- reductions
__global__ __launch_bounds__(256) void k_reduce_sum(const double* __restrict__ p, int n,
                                                    double* __restrict__ scal, int slot) {
  __shared__ double red[4];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += p[i];
  const double t = block_sum_256(a, red);
  if (threadIdx.x == 0) scal[slot] = t;
}

// out[slot[q]] (or out[q]) = sum of p[begin[q] .. begin[q + 1]), in the same
// order as k_reduce_sum over that range.
__global__ __launch_bounds__(256) void k_reduce_ranges(const double* __restrict__ p,
                                                       const int* __restrict__ begin,
                                                       const int* __restrict__ slot,
                                                       double* __restrict__ out) {
  __shared__ double red[4];
  const int q = blockIdx.x;
  const int b = begin[q], n = begin[q + 1] - b;
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += p[b + i];
  const double t = block_sum_256(a, red);
  if (threadIdx.x == 0) out[slot ? slot[q] : q] = t;
}

// The stopping rule of refl_sign for every live problem of the batched
// solve (one block; problems strided over the threads).
__global__ __launch_bounds__(256) void k_batch_decide(int nprob, const double* __restrict__ res,
                                                      const double* __restrict__ trace,
                                                      const BatchRule* __restrict__ rules,
                                                      BatchStep* __restrict__ stp,
                                                      int* __restrict__ live, int* __restrict__ ctl,
                                                      int par) {
  __shared__ double red[4];
  const int m = ctl[0];
  int n = 0;
  for (int p = threadIdx.x; p < nprob; p += 256) {
    if (!live[p]) continue;
    BatchStep s = stp[p];
    const BatchRule ru = rules[p];
    const double r = sqrt(fmax(res[p], 0.0));
    if (m > 0) s.trace = trace[p];
    if (batch_rule(s, ru, r, m, par))
      live[p] = 0;
    else
      ++n;
    stp[p] = s;
  }
  const double t = block_sum_256((double)n, red);
  if (threadIdx.x == 0) {
    ctl[1] = (int)t;
    ctl[0] = m + 1;
  }
}

// The reductions and the decision of one step of a single-problem device
// loop in one launch.  res = sum of pr[0..n) and, from step 1 on, trace =
// sum of pt[0..n) (the previous update product's trace partials), each in
// k_reduce_sum's order, go to scal[SC_RESID2] / scal[SC_TRACE]; then the
// rule: mixed_rule (MixedRule) or batch_rule (BatchRule, the effect of
// k_batch_decide for one problem).  ctl[0] is the step m (read, then
// incremented); at the stop live[0] and ctl[1] become 0 and the record's par
// names the buffer of X_m.  Once live[0] is 0 the partials are stale and only
// the step counter moves.
template <typename Rule>
__global__ __launch_bounds__(256) void k_reduce_decide(const double* __restrict__ pr,
                                                       const double* __restrict__ pt, int n,
                                                       double* __restrict__ scal,
                                                       const Rule* __restrict__ rule,
                                                       BatchStep* __restrict__ stp,
                                                       int* __restrict__ live,
                                                       int* __restrict__ ctl, int par) {
  __shared__ double red[4];
  const int m = ctl[0];
  const bool on = live[0] != 0;
  double r2 = 0.0, tr = 0.0;
  if (on) {
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += pr[i];
    r2 = block_sum_256(a, red);
    if (m > 0) {
      double b = 0.0;
      for (int i = threadIdx.x; i < n; i += 256) b += pt[i];
      tr = block_sum_256(b, red);
    }
  }
  if (threadIdx.x != 0) return;
  ctl[0] = m + 1;
  if (!on) return;
  scal[SC_RESID2] = r2;
  BatchStep s = stp[0];
  if (m > 0) {
    scal[SC_TRACE] = tr;
    s.trace = tr;
  }
  const double r = sqrt(fmax(r2, 0.0));
  bool stop;
  if constexpr (std::is_same<Rule, MixedRule>::value)
    stop = mixed_rule(s, rule[0], r, m, par);
  else
    stop = batch_rule(s, rule[0], r, m, par);
  if (stop) {
    live[0] = 0;
    ctl[1] = 0;
  }
  stp[0] = s;
}

template <typename T>
__device__ __forceinline__ void trace_block(const T* __restrict__ X, int dp, int d,
                                            double* __restrict__ out, double* red) {
  double a = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) a += (double)X[(int64_t)i * dp + i];
  const double t = block_sum_256(a, red);
  if (threadIdx.x == 0) *out = t;
}

template <typename T>
__global__ __launch_bounds__(256) void k_trace(const T* __restrict__ X, int dp, int d,
                                               double* __restrict__ scal, int slot) {
  __shared__ double red[4];
  trace_block(X, dp, d, scal + slot, red);
}

template <int W>
__global__ __launch_bounds__(256) void k_trace_w(const uint16_t* __restrict__ X, int64_t ps,
                                                 int dp, int d, double* __restrict__ scal,
                                                 int slot) {
  __shared__ double red[4];
  REFL_GUARD(d <= dp && ps >= (int64_t)dp * dp && slot >= 0 && slot < SC_COUNT, DBG_TRACE);
  double a = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) {
    float x = 0.f;
#pragma unroll
    for (int q = 0; q < W; ++q) x += bf16_to_f32(X[q * ps + (int64_t)i * dp + i]);
    a += (double)x;
  }
  const double t = block_sum_256(a, red);
  if (threadIdx.x == 0) scal[slot] = t;
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy_out(const T* __restrict__ X, int dp, int d,
                                                  double* __restrict__ R, int64_t ldr) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * 256 + threadIdx.x; j < d; j += gridDim.x * 256)
    R[(int64_t)i * ldr + j] = (double)X[(int64_t)i * dp + j];
}

// ------------------------------------------------------------- derivatives
// out (dp x dp) = (G + G^T)/2 on the leading d x d block (times 1/scal[SC_ALPHA]
// if scal != null), zero elsewhere; G is d x d with leading dimension ldg.
// Block (bx, by) handles the 64 x 64 tile (by, bx) and its transpose.
template <typename T>
__global__ __launch_bounds__(256) void k_sym_in(const double* __restrict__ G, int64_t ldg, int d,
                                                const double* __restrict__ scal,
                                                T* __restrict__ out, int dp) {
  const int I = blockIdx.y, J = blockIdx.x;
  __shared__ double t[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int i0 = I * 64, j0 = J * 64;
  // t = tile (J, I) of G, transposed on the way in.
  for (int r = ty; r < 64; r += 4) {
    const int gi = j0 + r, gj = i0 + tx;
    t[tx][r] = (gi < d && gj < d) ? G[(int64_t)gi * ldg + gj] : 0.0;
  }
  __syncthreads();
  const double f = scal ? 1.0 / scal[SC_ALPHA] : 1.0;
  for (int r = ty; r < 64; r += 4) {
    const int i = i0 + r, j = j0 + tx;
    const double g = (i < d && j < d) ? G[(int64_t)i * ldg + j] : 0.0;
    out[(int64_t)i * dp + j] = (T)(0.5 * (g + t[r][tx]) * f);
  }
}

// R = X / scal[SC_ALPHA] (d x d, ldr), FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_copy_out_scaled(const T* __restrict__ X, int dp, int d,
                                                         const double* __restrict__ scal,
                                                         double* __restrict__ R, int64_t ldr) {
  const int i = blockIdx.y;
  const double inv = 1.0 / scal[SC_ALPHA];
  for (int j = blockIdx.x * 256 + threadIdx.x; j < d; j += gridDim.x * 256)
    R[(int64_t)i * ldr + j] = (double)X[(int64_t)i * dp + j] * inv;
}

// partials[block] = sum over the block's share of (double) A_i * B_i.
template <typename T>
__global__ __launch_bounds__(256) void k_dot(const T* __restrict__ A, const T* __restrict__ B,
                                             int64_t n, double* __restrict__ partials) {
  __shared__ double red[4];
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    a += (double)A[i] * (double)B[i];
  const double t = block_sum_256(a, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// ------------------------------------------------------------ shift policy
// partials[block] = sum over the block's rows i of
//   sum_{j >= i} w_ij (A_ij - B_ij)^2,  w = 1 on the diagonal, 2 above,
// i.e. ||A - B||_F^2 of the symmetric matrices whose upper triangles are
// given.  One wave per row, 4 rows per block.
__global__ __launch_bounds__(256) void k_diff_fro_upper(const double* __restrict__ A, int64_t lda,
                                                        const double* __restrict__ B, int64_t ldb,
                                                        int d, double* __restrict__ partials) {
  __shared__ double red[4];
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  double acc = 0.0;
  if (row < d) {
    const double* a = A + (int64_t)row * lda;
    const double* b = B + (int64_t)row * ldb;
    for (int j = row + lane; j < d; j += 64) {
      const double e = a[j] - b[j];
      acc += (j == row ? 1.0 : 2.0) * e * e;
    }
  }
  const double t = block_sum_256(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// B (upper triangle, ldb) = A (upper triangle, lda).
__global__ __launch_bounds__(256) void k_copy_upper(const double* __restrict__ A, int64_t lda,
                                                    double* __restrict__ B, int64_t ldb, int d) {
  const int row = blockIdx.y;
  for (int j = row + blockIdx.x * 256 + threadIdx.x; j < d; j += gridDim.x * 256)
    B[(int64_t)row * ldb + j] = A[(int64_t)row * lda + j];
}

// ------------------------------------------------- batched set-up / output
// Grouped forms of the kernels above over many problems (one descriptor per
// problem): the blocks of problem ids[g] (or g) are begin[g] .. begin[g+1),
// and each block does what the single-problem kernel's block does, so every
// value equals the single-problem one bit for bit.
__device__ __forceinline__ int find_group(const int* __restrict__ begin, int n, int b) {
  int lo = 0, hi = n - 1;  // largest g with begin[g] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

constexpr int INIT_CHUNK = 2048;  // elements per block of k_batch_init

// Blocks: (dp/64)^2 per problem, tile (I, J) = (local / nt, local % nt).
__global__ __launch_bounds__(256) void k_batch_mirror(const BatchDesc* __restrict__ desc,
                                                      const int* __restrict__ begin,
                                                      const int* __restrict__ ids, int ng) {
  const int g = find_group(begin, ng, blockIdx.x);
  const BatchDesc q = desc[ids ? ids[g] : g];
  const int local = blockIdx.x - begin[g], nt = q.dp / 64;
  const int I = local / nt, J = local % nt;
  if (I > J) return;
  __shared__ double t[64][65];
  mirror_tile(q.H, q.ldh, q.d, q.Hf, q.dp, I, J, t);
}

// Blocks: ceil(d / 4) per problem (one wave per row).
__global__ __launch_bounds__(256) void k_batch_rowabs(const BatchDesc* __restrict__ desc,
                                                      const int* __restrict__ begin,
                                                      const int* __restrict__ ids, int ng) {
  const int g = find_group(begin, ng, blockIdx.x);
  const BatchDesc q = desc[ids ? ids[g] : g];
  const int local = blockIdx.x - begin[g];
  rowabs_row(q.Hf, q.dp, q.d, q.s, q.norm, q.rowsum, q.rowsum + q.dp,
             local * 4 + (threadIdx.x >> 6));
}

// One block per problem.
__global__ __launch_bounds__(256) void k_batch_scale_finish(const BatchDesc* __restrict__ desc,
                                                            const int* __restrict__ ids) {
  __shared__ double red[4], redb[4];
  const BatchDesc q = desc[ids ? ids[blockIdx.x] : blockIdx.x];
  scale_finish_block(q.rowsum, q.rowsum + q.dp, q.d, q.norm, q.scale_given, q.alpha_given, q.scal,
                     red, redb);
}

// Blocks: ceil(dp^2 / INIT_CHUNK) per problem; X_0 into X[0].
template <typename T>
__global__ __launch_bounds__(256) void k_batch_init(const BatchDesc* __restrict__ desc,
                                                    const int* __restrict__ begin,
                                                    const int* __restrict__ ids, int ng) {
  const int g = find_group(begin, ng, blockIdx.x);
  const BatchDesc q = desc[ids ? ids[g] : g];
  const int64_t first = (int64_t)(blockIdx.x - begin[g]) * INIT_CHUNK;
  const int64_t end = min(first + INIT_CHUNK, (int64_t)q.dp * q.dp);
  init_x0_elems(q.Hf, q.dp, q.d, q.s, 1.0 / q.scal[SC_ALPHA], reinterpret_cast<T*>(q.X[0]),
                first + threadIdx.x, end, 256);
}

// One block per problem: out[p] = trace of X[par].
template <typename T>
__global__ __launch_bounds__(256) void k_batch_trace(const BatchDesc* __restrict__ desc,
                                                     const int* __restrict__ ids,
                                                     double* __restrict__ out) {
  __shared__ double red[4];
  const int p = ids ? ids[blockIdx.x] : blockIdx.x;
  const BatchDesc q = desc[p];
  trace_block(reinterpret_cast<const T*>(q.X[q.par]), q.dp, q.d, out + p, red);
}

// Blocks: BATCH_COPY_ROWS rows each.  to_hf == 0: R = X[par] (d x d, ldr);
// to_hf == 1: Hf = X[par] over the whole padded dp x dp matrix (FP64 copy).
template <typename T>
__global__ __launch_bounds__(256) void k_batch_copy(const BatchDesc* __restrict__ desc,
                                                    const int* __restrict__ begin,
                                                    const int* __restrict__ ids, int ng,
                                                    int to_hf) {
  const int g = find_group(begin, ng, blockIdx.x);
  const BatchDesc q = desc[ids ? ids[g] : g];
  const int n = to_hf ? q.dp : q.d;
  const int i0 = (blockIdx.x - begin[g]) * BATCH_COPY_ROWS;
  const int i1 = min(i0 + BATCH_COPY_ROWS, n);
  for (int i = i0; i < i1; ++i) {
    const T* X = reinterpret_cast<const T*>(q.X[q.par]) + (int64_t)i * q.dp;
    double* dst = to_hf ? q.Hf + (int64_t)i * q.dp : q.R + (int64_t)i * q.ldr;
    for (int j = threadIdx.x; j < n; j += 256) dst[j] = (double)X[j];
  }
}

// ------------------------------------------------------- thin products
// Partial sums of the symmetric thin passes are stored per block, not per
// column: chunk q, row block rb (256 rows), column c, row t of the block at
//   work[((q nrb + rb) NB + c) 256 + t],  nrb = ceil(d / 256),
// so each block writes NB contiguous 2 KB runs (one column-major d-long
// vector per chunk and column, 32 KB apart, cost about 10 us more per pass
// at d = 4096 in a probe of the FP32 pass, for 2.6 MB of partials).
template <int NB>
__device__ __forceinline__ int64_t thin_block_base(int q, int rb, int nrb) {
  return ((int64_t)q * nrb + rb) * NB * 256;
}

// Y (d x nb, column-major) = M V.  Grid (row groups of 64, column chunks of
// CH); each wave owns 16 rows.  A lane keeps V[j, 0..NB) for the CH/64
// columns j it reads in registers, multiplies them into one row at a time
// (row-contiguous, coalesced), and the wave sums its lanes.  Per-chunk
// partial sums go to work[chunk][c][row]; k_thin_finish adds the chunks in
// a fixed order.
template <typename MT>
struct MLoad {
  static __device__ __forceinline__ double at(const MT* M, int64_t idx, int64_t) {
    return (double)M[idx];
  }
};
template <int W>
struct WordsM {};
template <int W>
struct MLoad<WordsM<W>> {
  static __device__ __forceinline__ double at(const WordsM<W>* M, int64_t idx, int64_t ps) {
    const uint16_t* m = reinterpret_cast<const uint16_t*>(M);
    float x = 0.f;
#pragma unroll
    for (int q = 0; q < W; ++q) x += bf16_to_f32(m[q * ps + idx]);
    return (double)x;
  }
};

template <typename MT, int NB, int CH>
__global__ __launch_bounds__(256) void k_thin_partial(const MT* __restrict__ M, int64_t ldm,
                                                      int64_t ps, int d, const double* __restrict__ V,
                                                      int64_t ldv, int nb, double* __restrict__ work,
                                                      int64_t wld) {
  constexpr int PER = CH / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j0 = blockIdx.y * CH;
  REFL_GUARD(nb >= 1 && nb <= NB && j0 < d && ldv >= d, DBG_THIN_PARTIAL);
  double v[PER][NB];
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int j = j0 + t * 64 + lane;
#pragma unroll
    for (int c = 0; c < NB; ++c) v[t][c] = (j < d && c < nb) ? V[(int64_t)c * ldv + j] : 0.0;
  }
  const int rbeg = blockIdx.x * 64 + wave * 16;
  for (int rr = 0; rr < 16; ++rr) {
    const int row = rbeg + rr;
    if (row >= d) break;
    double acc[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[c] = 0.0;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int j = j0 + t * 64 + lane;
      const double m = (j < d) ? MLoad<MT>::at(M, (int64_t)row * ldm + j, ps) : 0.0;
#pragma unroll
      for (int c = 0; c < NB; ++c) acc[c] = fma(m, v[t][c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const double s = wave_sum(acc[c]);
      if (lane == 0 && c < nb) work[((int64_t)blockIdx.y * NB + c) * wld + row] = s;
    }
  }
}

// Grid (row blocks of 256, columns).  BLK: the partials are in the block
// layout of the symmetric passes (rows of a block of 256 contiguous), else
// at work[chunk][c][row] (leading dimension wld).
template <int NB, bool BLK>
__global__ __launch_bounds__(256) void k_thin_finish(const double* __restrict__ work, int64_t wld,
                                                     int nchunk, int d, int nb,
                                                     double* __restrict__ Y, int64_t ldy) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  REFL_GUARD(nb <= NB && (int)blockIdx.x * 256 < d && ldy >= d, DBG_THIN_FINISH);
  if (row >= d || c >= nb) return;
  double s = 0.0;
  if (BLK) {
    const int nrb = gridDim.x;
    const double* wp = work + c * 256 + threadIdx.x;
    int q = 0;
    for (; q + 8 <= nchunk; q += 8) {  // eight loads in flight, summed in order
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = wp[thin_block_base<NB>(q + u, blockIdx.x, nrb)];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += a[u];
    }
    for (; q < nchunk; ++q) s += wp[thin_block_base<NB>(q, blockIdx.x, nrb)];
  } else {
    for (int q = 0; q < nchunk; ++q) s += work[((int64_t)q * NB + c) * wld + row];
  }
  Y[(int64_t)c * ldy + row] = s;
}


// ---------------------------------------------------- block-vector kernels
// work[block][i + na*j] = sum over the block's 64 rows of A[r, i] B[r, j].
__global__ __launch_bounds__(256) void k_gram_partial(const double* __restrict__ A, int64_t lda,
                                                      int na, const double* __restrict__ B,
                                                      int64_t ldb, int nb, int d,
                                                      double* __restrict__ work) {
  __shared__ double sa[64][33], sb[64][33];
  const int r0 = blockIdx.x * 64;
  REFL_GUARD(na >= 0 && na <= 32 && nb >= 0 && nb <= 32 && r0 < d && lda >= d && ldb >= d, DBG_GRAM);
  for (int e = threadIdx.x; e < 64 * 32; e += 256) {
    const int r = e & 63, c = e >> 6;
    const int row = r0 + r;
    sa[r][c] = (row < d && c < na) ? A[(int64_t)c * lda + row] : 0.0;
    sb[r][c] = (row < d && c < nb) ? B[(int64_t)c * ldb + row] : 0.0;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < na * nb; o += 256) {
    const int i = o % na, j = o / na;
    double acc = 0.0;
    for (int r = 0; r < 64; ++r) acc = fma(sa[r][i], sb[r][j], acc);
    work[(int64_t)blockIdx.x * na * nb + o] = acc;
  }
}
__global__ __launch_bounds__(256) void k_gram_finish(const double* __restrict__ work, int nblk,
                                                     int n, double* __restrict__ G) {
  // One wave per output; lanes own blocks in a fixed order.
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (o >= n) return;
  double s = 0.0;
  for (int b = lane; b < nblk; b += 64) s += work[(int64_t)b * n + o];
  s = wave_sum(s);
  if (lane == 0) G[o] = s;
}

// Y[:, c] = alpha Y[:, c] + beta sum_i A[:, i] C[i, c]
__global__ __launch_bounds__(256) void k_block_axpy(int d, int na, int nb, double alpha,
                                                    double* __restrict__ Y, int64_t ldy,
                                                    double beta, const double* __restrict__ A,
                                                    int64_t lda, const double* __restrict__ C) {
  __shared__ double sc[32 * 32];
  for (int e = threadIdx.x; e < na * nb; e += 256) sc[e] = C[e];
  __syncthreads();
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= d) return;
  double a[32];
  for (int i = 0; i < na; ++i) a[i] = A[(int64_t)i * lda + row];
  for (int c = 0; c < nb; ++c) {
    double acc = 0.0;
    for (int i = 0; i < na; ++i) acc = fma(a[i], sc[i + na * c], acc);
    double* y = Y + (int64_t)c * ldy + row;
    *y = (alpha == 0.0 ? 0.0 : alpha * *y) + beta * acc;
  }
}

// Y[:, c] *= 1 (columns c >= ncol zeroed) -- and per-column scale: Y[:, c] = Y[:, c] - sh[c] V[:, c]
__global__ __launch_bounds__(256) void k_col_axpy(int d, int nb, double* __restrict__ Y, int64_t ldy,
                                                  const double* __restrict__ coef,
                                                  const double* __restrict__ X, int64_t ldx) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= d) return;
  for (int c = 0; c < nb; ++c) Y[(int64_t)c * ldy + row] += coef[c] * X[(int64_t)c * ldx + row];
}

// R = I - 2 V V^T on the d x d block (ldr), 64 x 64 tiles.
__global__ __launch_bounds__(256) void k_form_reflector(const double* __restrict__ V, int64_t ldv,
                                                        int k, int d, double* __restrict__ R,
                                                        int64_t ldr) {
  __shared__ double vi[64][33], vj[64][33];
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  REFL_GUARD(k >= 0 && k <= 32 && ldv >= d && ldr >= d && i0 < d && j0 < d, DBG_FORM_R);
  for (int e = threadIdx.x; e < 64 * 32; e += 256) {
    const int r = e & 63, c = e >> 6;
    vi[r][c] = (i0 + r < d && c < k) ? V[(int64_t)c * ldv + i0 + r] : 0.0;
    vj[r][c] = (j0 + r < d && c < k) ? V[(int64_t)c * ldv + j0 + r] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int i = i0 + r, j = j0 + tx;
    if (i >= d || j >= d) continue;
    double acc = 0.0;
    for (int c = 0; c < k; ++c) acc = fma(vi[r][c], vj[tx][c], acc);
    R[(int64_t)i * ldr + j] = (i == j ? 1.0 : 0.0) - 2.0 * acc;
  }
}

// out = c (Z V^T + V Z^T) on the d x d block (ldo), 64 x 64 tiles; Z and V
// are d x k blocks (ld), k <= 32.
__global__ __launch_bounds__(256) void k_form_sym_pair(const double* __restrict__ Z,
                                                       const double* __restrict__ V, int64_t ld,
                                                       int k, int d, double c,
                                                       double* __restrict__ out, int64_t ldo) {
  __shared__ double zi[64][33], vi[64][33], zj[64][33], vj[64][33];
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * 32; e += 256) {
    const int r = e & 63, q = e >> 6;
    const bool in_i = i0 + r < d && q < k, in_j = j0 + r < d && q < k;
    zi[r][q] = in_i ? Z[(int64_t)q * ld + i0 + r] : 0.0;
    vi[r][q] = in_i ? V[(int64_t)q * ld + i0 + r] : 0.0;
    zj[r][q] = in_j ? Z[(int64_t)q * ld + j0 + r] : 0.0;
    vj[r][q] = in_j ? V[(int64_t)q * ld + j0 + r] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int i = i0 + r, j = j0 + tx;
    if (i >= d || j >= d) continue;
    // Entry (i, j) is evaluated with the roles of lo = min(i, j) and
    // hi = max(i, j) fixed, z_lo v_hi + v_lo z_hi, so (i, j) and (j, i) run
    // the same operations on the same operands: exactly symmetric.
    const bool sw = i > j;
    double acc = 0.0;
    for (int q = 0; q < k; ++q) {
      const double zl = sw ? zj[tx][q] : zi[r][q], vl = sw ? vj[tx][q] : vi[r][q];
      const double zh = sw ? zi[r][q] : zj[tx][q], vh = sw ? vi[r][q] : vj[tx][q];
      acc = fma(zl, vh, fma(vl, zh, acc));
    }
    out[(int64_t)i * ldo + j] = c * acc;
  }
}

// Seeded start block: V[j + c ldv] uniform in (-1, 1) from splitmix64.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
// Grid (row blocks, columns): one entry per thread (the 64-bit multiplies of
// the hash are long; a loop over the columns per thread kept only a few
// compute units busy).
__global__ __launch_bounds__(256) void k_random_block(double* __restrict__ V, int64_t ldv, int d,
                                                      int nb, uint64_t seed) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= d) return;
  for (int c = blockIdx.y; c < nb; c += gridDim.y) {
    const uint64_t h = splitmix64(seed * 0x100000001B3ull + (uint64_t)c * (uint64_t)d + row);
    V[(int64_t)c * ldv + row] = ((double)(h >> 11) * 0x1.0p-53) * 2.0 - 1.0;
  }
}

// ------------------------------------------------- symmetric thin products
// Y = M V for SYMMETRIC M, computed as M^T V: y_r = sum_j M[j, r] V[j, :].
// A block takes 256 consecutive output rows r (one per lane of each group of
// four waves) and a chunk of CHUNK rows j of M, split between KS groups of
// four waves: group g sums rows [g CHUNK/KS, (g + 1) CHUNK/KS) of the chunk.
// The rows of M stream coalesced across the lanes, the CHUNK x NB block of V
// sits in LDS and is read as wave-uniform broadcasts, and the KS group sums
// are added in LDS in group order.  Partial sums per chunk go to work in the
// block layout above; a finishing kernel adds the chunks in order.
constexpr int SRC = 128;

template <int KS, int NB>
struct ThinRed {
  double v[KS > 1 ? (KS - 1) * NB * 256 : 1];
};

// p[i] if ok, else 0, loaded without a branch (the index falls back to 0,
// which must be valid).  A load inside a branch is waited for where the
// branch ends, so a run of conditional loads made as many round trips to
// memory as there were loads.
template <typename T>
__device__ __forceinline__ double ldsel(const T* __restrict__ p, int64_t i, bool ok) {
  const T v = p[ok ? i : 0];
  return ok ? (double)v : 0.0;
}
// The same for p[i], p[i + 1] with one 16-byte load (p + i 16-byte aligned
// when ok).
__device__ __forceinline__ double2 ld2sel(const double* __restrict__ p, int64_t i, bool ok) {
  const double2 v = *reinterpret_cast<const double2*>(p + (ok ? i : 0));
  return ok ? v : make_double2(0.0, 0.0);
}

// The first eight rows of M of a lane (they do not depend on V), so that a
// kernel can request them before it sets up the V block in LDS.
template <typename MT, int CHUNK, int KS>
__device__ __forceinline__ void symthin_first(const MT* __restrict__ M, int64_t ldm, int64_t ps,
                                              int d, double (&m0)[8]) {
  constexpr int PART = CHUNK / KS;
  const int t = threadIdx.x & 255, g = threadIdx.x >> 8;
  const int r = blockIdx.x * 256 + t;
  const int j0 = blockIdx.y * CHUNK + g * PART;
  const int jn = max(0, min(PART, d - j0));
  const int rc = min(r, d - 1);  // in bounds for every lane; masked below
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const double v = MLoad<MT>::at(M, (int64_t)min(j0 + u, d - 1) * ldm + rc, ps);
    m0[u] = (r < d && u < jn) ? v : 0.0;
  }
}

// With HAVE0 the first eight rows of M come in m0 (symthin_first), else
// the body loads them.
template <typename MT, int NB, int CHUNK, int KS, bool HAVE0 = true>
__device__ __forceinline__ void symthin_body(const MT* __restrict__ M, int64_t ldm, int64_t ps, int d,
                                             const double (*pv)[NB], double* __restrict__ work,
                                             int64_t wld, int nb, ThinRed<KS, NB>& red,
                                             const double (&m0)[8]) {
  static_assert(CHUNK % KS == 0, "chunk must split evenly");
  constexpr int PART = CHUNK / KS;
  const int t = threadIdx.x & 255, g = threadIdx.x >> 8;
  const int r = blockIdx.x * 256 + t;
  const int j0 = blockIdx.y * CHUNK + g * PART;
  const int jn = max(0, min(PART, d - j0));
  double acc[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) acc[c] = 0.0;
  if (r < d) {
    const double (*pp)[NB] = pv + g * PART;
    // For the narrow types a full chunk (every chunk but the last) runs a
    // loop of known length, unrolled, so that the compiler requests later
    // rows before the products of earlier ones.  (The FP64 pass with 12
    // columns ran slower that way: 28 against 24 us at d = 4096.)
    if (sizeof(MT) < 8 && jn == PART) {
#pragma unroll
      for (int jb = 0; jb < PART; jb += 8) {
        double m[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          m[u] = (HAVE0 && jb == 0) ? m0[u] : MLoad<MT>::at(M, (int64_t)(j0 + jb + u) * ldm + r, ps);
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int c = 0; c < NB; ++c) acc[c] = fma(m[u], pp[jb + u][c], acc[c]);
      }
    } else {
      int jj = 0;
      for (; jj + 8 <= jn; jj += 8) {
        double m[8];
        if (HAVE0 && jj == 0) {
#pragma unroll
          for (int u = 0; u < 8; ++u) m[u] = m0[u];
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u) m[u] = MLoad<MT>::at(M, (int64_t)(j0 + jj + u) * ldm + r, ps);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int c = 0; c < NB; ++c) acc[c] = fma(m[u], pp[jj + u][c], acc[c]);
      }
      for (; jj < jn; ++jj) {
        const double m = (HAVE0 && jj < 8) ? m0[jj] : MLoad<MT>::at(M, (int64_t)(j0 + jj) * ldm + r, ps);
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[c] = fma(m, pp[jj][c], acc[c]);
      }
    }
  }
  if constexpr (KS > 1) {
    if (g > 0) {
#pragma unroll
      for (int c = 0; c < NB; ++c) red.v[((g - 1) * NB + c) * 256 + t] = acc[c];
    }
    __syncthreads();
    if (g > 0) return;
#pragma unroll
    for (int q = 0; q < KS - 1; ++q)
#pragma unroll
      for (int c = 0; c < NB; ++c) acc[c] += red.v[(q * NB + c) * 256 + t];
  }
  if (r < d) {
    double* wb = work + thin_block_base<NB>(blockIdx.y, blockIdx.x, gridDim.x) + t;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nb) wb[c * 256] = acc[c];
  }
}

// The stand-alone product (Lanczos steps, Rayleigh-Ritz, subspace
// extraction) splits each chunk over KS groups of 64 rows: 4 groups
// (256-row chunks) up to 12 columns, 2 (128-row chunks) up to 32, within the
// LDS of the group sums and the registers of 1024-thread blocks.  More
// waves, each with fewer dependent round trips to memory (measured at
// d = 4096, 12 columns: one group 36 us, two 24 us).
template <int NB>
constexpr int symthin_ks() { return NB <= 12 ? 4 : 2; }
template <int NB>
constexpr int symthin_chunk() { return 64 * symthin_ks<NB>(); }

template <typename MT, int NB, int KS = symthin_ks<NB>(), int CHUNK = symthin_chunk<NB>()>
__global__ __launch_bounds__(256 * KS) void k_symthin(const MT* __restrict__ M, int64_t ldm,
                                                      int64_t ps, int d,
                                                      const double* __restrict__ V, int64_t ldv,
                                                      int nb, double* __restrict__ work,
                                                      int64_t wld) {
  __shared__ double pv[CHUNK][NB];
  __shared__ ThinRed<KS, NB> red;
  const int j0 = blockIdx.y * CHUNK;
  REFL_GUARD(nb >= 1 && nb <= NB && j0 < d && ldv >= d, DBG_SYMTHIN);
  for (int e = threadIdx.x; e < CHUNK * NB; e += 256 * KS) {
    const int jj = e / NB, c = e % NB, j = j0 + jj;
    pv[jj][c] = ldsel(V, (int64_t)c * ldv + j, j < d && c < nb);
  }
  __syncthreads();
  const double m0[8] = {};
  symthin_body<MT, NB, CHUNK, KS, false>(M, ldm, ps, d, pv, work, wld, nb, red, m0);
}

// ------------------------------------------------------------ block CG
// Solves, column by column (c < nb), the projected correction equations
//   A_c z_c = b_c,  A_c = (I - V V^T)(H - theta_c I)(I - V V^T),
// z_c and b_c orthogonal to V, by conjugate gradients (A_c is positive
// definite on the complement of V when theta_c lies below the spectrum
// there).  The recurrences are those of Chronopoulos and Gear (1989): with
// w = A r, the two inner products of an iteration, gamma = r.r and
// delta = r.w, come from the same operator application, so one iteration
// has a single reduction point:
//   beta_i  = gamma_i / gamma_{i-1}                        (beta_0 = 0)
//   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1})
//                                                      (alpha_0 = gamma_0 / delta_0)
//   p_i = r_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1},
//   z_{i+1} = z_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i.
// Iteration `it` is two launches with no atomics or fences between blocks:
//   k_cg_step   (it >= 1) every block re-reduces, in a fixed order, the
//               partials of the previous k_cg_apply: C = V^T (H - theta) r,
//               gamma, delta per column; convergence test on gamma;
//               alpha, beta; then the update above for the rows of its
//               chunk (w = (H - theta) r - V C), written by the blocks of
//               column 0 of the grid.  Then the chunk partials of H r.
//   k_cg_apply  (H - theta) r = chunk sums - theta r, and per-block
//               partials of V^T (H - theta) r, r.r and r.(H - theta) r.
// The kernel boundary makes each kernel's stores visible to the next.
// r, p and s alternate between two buffers by iteration parity, so a
// block never reads a row another block of the same launch writes.  Every
// kernel returns at once when state->done is set, so batches of
// iterations are enqueued without host synchronisation.
struct CgState {
  double theta[32], rho0[32], gam[2][32], alpha[2][32];
  double tol2;
  int iters, done, k, nb;
};

// Grid (column blocks of 256 output rows, chunks of CHUNK rows of M).  M is
// H in FP64, or its FP32 copy (the products still accumulate in FP64).  The
// chunks are split over KS groups of four waves, each summing 64 rows (FP32;
// FP64 up to 8 columns) or 64 to 128 rows (FP64): more waves keep more bytes
// in flight and share the reduction and the row update at the start of
// k_cg_step, and longer chunks leave fewer chunk partials for k_cg_apply.
// KS is 4 up to 8 columns, 2 up to 16, and 1 beyond (the LDS of the group
// sums).  Measured at d = 4096, 5 columns, against two groups of 64 rows:
// FP32 18.8 -> 17.3 us, FP64 26.8 -> 26.2 us per iteration, and the
// partial sums 6.6 -> 6.2 us.
constexpr int CG_SRC = SRC / 2;
template <typename MT, int NB>
constexpr int cg_ks() { return NB <= 8 ? 4 : (NB <= 16 ? 2 : 1); }
template <typename MT, int NB>
constexpr int cg_chunk() {
  return sizeof(MT) == 4 ? CG_SRC * cg_ks<MT, NB>() : (cg_ks<MT, NB>() == 4 ? 2 * SRC : SRC);
}

template <typename MT, int NB, int CHUNK = cg_chunk<MT, NB>(), int KS = cg_ks<MT, NB>()>
__global__ __launch_bounds__(256 * KS) void k_cg_step(const MT* __restrict__ M, int64_t ldm, int d,
                                                      const double* __restrict__ V, int64_t ldv,
                                                      CgBufs b, CgState* __restrict__ st,
                                                      const double* __restrict__ apart,
                                                      int ngroups, double* __restrict__ work,
                                                      int64_t wld, int it, int max_iter) {
  if (st->done) return;
  constexpr int NT = 256 * KS, NW = NT / 64;
  __shared__ double pv[CHUNK][NB];
  __shared__ ThinRed<KS, NB> red;
  __shared__ double sC[NB][34];
  __shared__ double sal[NB], sbe[NB];
  __shared__ int sconv;
  const int nb = st->nb, k = st->k;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j0 = blockIdx.y * CHUNK;
  REFL_GUARD(nb >= 1 && nb <= NB && k <= 32 && j0 < d && ldv >= d, DBG_CG_STEP);
  const bool first = blockIdx.x == 0 && blockIdx.y == 0;
  // Every global load of the block's set-up is issued before the first wait
  // (and the first rows of M after them), and the barriers between the
  // set-up steps order only LDS: the set-up's chain of dependent round trips
  // to memory then overlaps the start of the pass over M.
  double m0[8];
  if (it == 0) {
    double rv[(NB * CHUNK + NT - 1) / NT];
#pragma unroll
    for (int u = 0; u < (NB * CHUNK + NT - 1) / NT; ++u) {
      const int e = tid + u * NT;
      const int c = e / CHUNK, j = j0 + e % CHUNK;
      rv[u] = ldsel(b.R[0], (int64_t)c * ldv + j, e < NB * CHUNK && c < nb && j < d);
    }
    symthin_first<MT, CHUNK, KS>(M, ldm, 0, d, m0);
#pragma unroll
    for (int u = 0; u < (NB * CHUNK + NT - 1) / NT; ++u) {
      const int e = tid + u * NT;
      if (e < NB * CHUNK) pv[e % CHUNK][e / CHUNK] = rv[u];
    }
    if (first && tid == 0) st->iters = 0;
  } else {
    // Partials of the previous apply: apart[((c (k + 2) + v) ngroups + g],
    // v < k the entries of C[:, c], then gamma and delta (pair q = c (k + 2)
    // + v; the groups of a pair are contiguous, so a wave's loads share cache
    // lines).  A wave takes up to four
    // (c, v) pairs at once, so that their loads are in flight together.
    const int nv = k + 2, npairs = nb * nv;
    const int tc = min(tid, nb - 1);  // values of threads >= nb are not used
    const double gp = st->gam[it & 1][tc], ap = st->alpha[it & 1][tc];
    const double tol2 = st->tol2, rho0 = st->rho0[tc];
    // The first 64 groups' partials (a lane each); any more are added later.
    double acc0[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = wave + u * NW;
      acc0[u] = ldsel(apart, (int64_t)q * ngroups + lane, lane < ngroups && q < npairs);
    }
    // The rows of the update (the block's chunk), V up to KV columns.
    const double* Rin = b.R[(it - 1) & 1];
    double* Rout = b.R[it & 1];
    const double* Pin = b.P[it & 1];
    double* Pout = b.P[(it - 1) & 1];
    const double* Sin = b.S[it & 1];
    double* Sout = b.S[(it - 1) & 1];
    const bool writer = blockIdx.x == 0;
    // A thread takes pairs of rows (j, j + 1), j even, with 16-byte loads
    // (ldv is even): half the load instructions of one row per thread.
    constexpr int HC = CHUNK / 2, NP = NB * HC, PERP = (NP + NT - 1) / NT, KV = NB < 8 ? NB : 8;
    double2 hr[PERP], r[PERP], pprev[PERP], sprev[PERP], z[PERP], vv[PERP][KV];
    const double* Vb = k > 0 ? V : b.HR;  // a valid address for the masked loads
#pragma unroll
    for (int u = 0; u < PERP; ++u) {
      const int ep = tid + u * NT;
      const int c = ep / HC, j = j0 + 2 * (ep % HC);
      const bool ok = ep < NP && c < nb && j < d;
      const int64_t o = ok ? (int64_t)c * ldv + j : 0;
      hr[u] = ld2sel(b.HR, o, ok);
#pragma unroll
      for (int i = 0; i < KV; ++i) vv[u][i] = ld2sel(Vb, (int64_t)i * ldv + j, ok && i < k);
      r[u] = ld2sel(Rin, o, ok);
      pprev[u] = ld2sel(Pin, o, ok && it >= 2);
      sprev[u] = ld2sel(Sin, o, ok && it >= 2);
      z[u] = ld2sel(b.Z, o, ok && writer);
    }
    symthin_first<MT, CHUNK, KS>(M, ldm, 0, d, m0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = wave + u * NW;
      if (q < npairs) {  // wave-uniform
        double acc = acc0[u];
        for (int g = lane + 64; g < ngroups; g += 64) acc += apart[(int64_t)q * ngroups + g];
        const double t = wave_sum(acc);
        if (lane == 0) sC[q / nv][q % nv] = t;
      }
    }
    for (int q0 = wave + 4 * NW; q0 < npairs; q0 += 4 * NW) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int g = lane; g < ngroups; g += 64) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = q0 + u * NW;
          if (q < npairs) acc[u] += apart[(int64_t)q * ngroups + g];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + u * NW;
        if (q < npairs) {  // wave-uniform
          const double t = wave_sum(acc[u]);
          if (lane == 0) sC[q / nv][q % nv] = t;
        }
      }
    }
    if (tid == 0) sconv = 1;
    lds_barrier();
    if (tid < nb) {
      const int c = tid;
      const double gam = sC[c][k], del = sC[c][k + 1];
      double alpha, beta = 0.0;
      if (it >= 2) {
        beta = gp > 0.0 ? gam / gp : 0.0;
        const double den = del - (ap != 0.0 ? beta * gam / ap : 0.0);
        alpha = den != 0.0 ? gam / den : 0.0;
      } else {
        alpha = del != 0.0 ? gam / del : 0.0;
      }
      sal[c] = alpha;
      sbe[c] = beta;
      if (!(gam <= tol2 * rho0)) sconv = 0;
      if (first) {
        st->gam[(it - 1) & 1][c] = gam;
        st->alpha[(it - 1) & 1][c] = alpha;
      }
    }
    lds_barrier();
    // Iteration it applies update it - 1; the test is on r_{it-1}.
    if (sconv || it - 1 >= max_iter) {
      if (first && tid == 0) {
        st->iters = it - 1;
        st->done = 1;
      }
      return;
    }
#pragma unroll
    for (int u = 0; u < PERP; ++u) {
      const int ep = tid + u * NT;
      if (ep >= NP) break;
      const int c = ep / HC, jj = 2 * (ep % HC), j = j0 + jj;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double rn = 0.0;
        if (c < nb && j + h < d) {
          const int64_t o = (int64_t)c * ldv + j + h;
          double w = h ? hr[u].y : hr[u].x;
#pragma unroll
          for (int i = 0; i < KV; ++i)
            if (i < k) w = fma(-(h ? vv[u][i].y : vv[u][i].x), sC[c][i], w);
          for (int i = KV; i < k; ++i) w = fma(-V[(int64_t)i * ldv + j + h], sC[c][i], w);
          const double al = sal[c], ri = h ? r[u].y : r[u].x;
          double pn = ri, sn = w;
          if (it >= 2) {
            pn = fma(sbe[c], h ? pprev[u].y : pprev[u].x, ri);
            sn = fma(sbe[c], h ? sprev[u].y : sprev[u].x, w);
          }
          rn = fma(-al, sn, ri);
          if (writer) {
            Pout[o] = pn;
            Sout[o] = sn;
            b.Z[o] = fma(al, pn, h ? z[u].y : z[u].x);
            Rout[o] = rn;
          }
        }
        pv[jj + h][c] = rn;
      }
    }
    if (first && tid == 0) st->iters = it;
  }
  lds_barrier();
  symthin_body<MT, NB, CHUNK, KS>(M, ldm, 0, d, pv, work, wld, nb, red, m0);
}

// Grid (row groups of 64, column c), 256 threads: four lanes per row, each
// summing every fourth chunk (four times the loads in flight of one lane per
// row), combined by shuffles; lane 0 of each group of four holds the row.
template <int NB>
__global__ __launch_bounds__(256) void k_cg_apply(const double* __restrict__ work, int64_t wld,
                                                  int nchunk, int d, const double* __restrict__ V,
                                                  int64_t ldv, const double* __restrict__ R,
                                                  double* __restrict__ HR,
                                                  const CgState* __restrict__ st,
                                                  double* __restrict__ apart) {
  if (st->done) return;
  __shared__ double red[4][35];
  const int nb = st->nb, k = st->k;
  const int c = blockIdx.y;
  REFL_GUARD(nb >= 1 && nb <= NB && k <= 32 && c < nb && (int)blockIdx.x * 64 < d && ldv >= d,
             DBG_CG_APPLY);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sub = tid & 3;
  const int row = blockIdx.x * 64 + (tid >> 2);
  const bool owner = sub == 0 && row < d;
  // Loads that do not wait for the chunk sums are requested first, and
  // without branches (masked loads).
  constexpr int KV = NB < 8 ? NB : 8;
  const int64_t o = (int64_t)c * ldv + row;
  const double r0 = ldsel(R, o, owner);
  const double th = st->theta[c];
  const double* Vb = k > 0 ? V : R;  // a valid address for the masked loads
  double vr[KV];
#pragma unroll
  for (int i = 0; i < KV; ++i) vr[i] = ldsel(Vb, (int64_t)i * ldv + row, owner && i < k);
  // Partials in the block layout of the symmetric passes.
  const int rowc = row < d ? row : d - 1;
  const int nrb = (d + 255) / 256;
  const double* wr = work + (int64_t)c * 256 + (rowc & 255);
  const int rb = rowc >> 8;
  double acc[4] = {0, 0, 0, 0};
  int q = sub;
  for (; q + 12 < nchunk; q += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += wr[thin_block_base<NB>(q + 4 * u, rb, nrb)];
  }
  for (; q < nchunk; q += 4) acc[0] += wr[thin_block_base<NB>(q, rb, nrb)];
  double s = row < d ? (acc[0] + acc[1]) + (acc[2] + acc[3]) : 0.0;
  s += __shfl_xor(s, 1, WAVE);
  s += __shfl_xor(s, 2, WAVE);
  const double rc = owner ? r0 : 0.0;
  if (owner) {
    s -= th * rc;
    HR[o] = s;
  } else {
    s = 0.0;
  }
  // Partials: V^T (H - theta) r (k values), r.r, r.(H - theta) r at
  // apart[(c (k + 2) + v) gridDim.x + group]; the four waves' sums are added
  // in a fixed order.
  for (int i = 0; i < k; ++i) {
    double vi;
    if (i < KV) {
      vi = vr[0];
#pragma unroll
      for (int u = 1; u < KV; ++u) vi = i == u ? vr[u] : vi;
    } else {
      vi = owner ? V[(int64_t)i * ldv + row] : 0.0;
    }
    const double t = wave_sum(vi * s);
    if (lane == 0) red[wave][i] = t;
  }
  const double t1 = wave_sum(rc * rc);
  const double t2 = wave_sum(rc * s);
  if (lane == 0) {
    red[wave][k] = t1;
    red[wave][k + 1] = t2;
  }
  __syncthreads();
  if (tid < k + 2)
    apart[((int64_t)c * (k + 2) + tid) * gridDim.x + blockIdx.x] =
        (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// ------------------------------------------------------- pipelined block CG
// The same projected systems A_c z_c = b_c by the pipelined recurrences of
// Ghysels and Vanroose (2014), which carry w = A r and q = A w as vectors
// so that the operator application of an iteration needs no reduction of
// that iteration:
//   gamma_i = r_i.r_i, delta_i = w_i.r_i, q_i = A w_i,
//   beta_i, alpha_i as in the Chronopoulos-Gear form above,
//   zz_i = q_i + beta_i zz_{i-1}, s_i = w_i + beta_i s_{i-1},
//   p_i = r_i + beta_i p_{i-1},
//   z_{i+1} = z_i + alpha_i p_i, r_{i+1} = r_i - alpha_i s_i,
//   w_{i+1} = w_i - alpha_i zz_i.
// The projection of (M - theta) w onto the complement of V needs
// V^T (M - theta) w = U^T w - theta V^T w with U = M V, formed once per
// solve (M is symmetric).  So the pass over M of launch `it` multiplies a
// block known when the launch starts (r_0 for it = 0, else w), and every
// reduction of an iteration (U^T w, V^T w, gamma, delta) is a per-group
// partial that the update launch writes for the next update launch:
//   k_cg_pass    chunk partials of M r_0 (it = 0) or M w (no set-up);
//   k_cg_update  (M - theta) x = chunk sums - theta x for its rows; sums,
//                in a fixed order, the partials the previous update (or
//                k_cg_init) wrote; it = 0 forms w_0 = A r_0, it >= 1 tests
//                r_{it-1} (all columns) and applies update it - 1; then
//                writes the partials of the new rows.
// Each row belongs to one update block, so the vectors are updated in
// place.  The partials alternate between two buffers by parity:
//   part[par][((c NV + v) nrg + g)],  NV = 2k + 2, nrg = ceil(d / 64),
// v < k: U^T x, k <= v < 2k: V^T x, then gamma and delta (x = w, or r_0).
// Pipelining trades some attainable accuracy for the shorter dependency
// chain, so it serves the correction's loose inner tolerance; the
// gradient's tight solve keeps the form above.

// Partials of one column over a block's 64 rows (lane sub == 0 of each
// group of four holds the row): U^T x, V^T x, g0 and g1 (the gamma and
// delta terms of the row), into part at group blockIdx.x.  The row values
// go through LDS (sp[v][row]) and thread v sums its 64 rows in order: a
// wave reduction per value (a chain of cross-lane permutes) cost several
// times more for the twelve values of five columns.
template <int KV>
__device__ __forceinline__ void cg_write_parts(int k, int c, int nrg, double x, const double (&ur)[KV],
                                               const double (&vr)[KV], const double* __restrict__ U,
                                               const double* __restrict__ V, int64_t ldv, int row,
                                               bool owner, double g0, double g1,
                                               double* __restrict__ part, double (*sp)[65]) {
  const int tid = threadIdx.x, rl = tid >> 2;
  const int nv = 2 * k + 2;
  if ((tid & 3) == 0) {
    for (int i = 0; i < k; ++i) {
      double ui, vi;
      if (i < KV) {
        ui = ur[0];
        vi = vr[0];
#pragma unroll
        for (int u = 1; u < KV; ++u) {
          ui = i == u ? ur[u] : ui;
          vi = i == u ? vr[u] : vi;
        }
      } else {
        ui = owner ? U[(int64_t)i * ldv + row] : 0.0;
        vi = owner ? V[(int64_t)i * ldv + row] : 0.0;
      }
      sp[i][rl] = ui * x;
      sp[k + i][rl] = vi * x;
    }
    sp[2 * k][rl] = g0;
    sp[2 * k + 1][rl] = g1;
  }
  lds_barrier();
  if (tid < nv) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 16
    for (int r = 0; r < 64; ++r) a[r & 3] += sp[tid][r];
    part[((int64_t)c * nv + tid) * nrg + blockIdx.x] = (a[0] + a[1]) + (a[2] + a[3]);
  }
}

// Partials of r_0 (U^T r_0, V^T r_0) for the first update launch.
template <int NB>
__global__ __launch_bounds__(256) void k_cg_init(int d, const double* __restrict__ V,
                                                 const double* __restrict__ U, int64_t ldv,
                                                 const double* __restrict__ R,
                                                 const CgState* __restrict__ st,
                                                 double* __restrict__ part) {
  __shared__ double sp[2 * NB + 2][65];
  const int k = st->k, c = blockIdx.y;
  REFL_GUARD(k <= NB && (int)blockIdx.x * 64 < d && ldv >= d, DBG_CG_INIT);
  const int tid = threadIdx.x, sub = tid & 3;
  const int row = blockIdx.x * 64 + (tid >> 2);
  const bool owner = sub == 0 && row < d;
  constexpr int KV = NB < 8 ? NB : 8;
  const double* Vb = k > 0 ? V : R;
  const double* Ub = k > 0 ? U : R;
  double ur[KV], vr[KV];
#pragma unroll
  for (int i = 0; i < KV; ++i) {
    ur[i] = ldsel(Ub, (int64_t)i * ldv + row, owner && i < k);
    vr[i] = ldsel(Vb, (int64_t)i * ldv + row, owner && i < k);
  }
  const double x = ldsel(R, (int64_t)c * ldv + row, owner);
  cg_write_parts<KV>(k, c, gridDim.x, x, ur, vr, U, V, ldv, row, owner, 0.0, 0.0, part, sp);
}

// The pass over M: chunk partials of M x, x = r_0 (it = 0) or w.
template <typename MT, int NB, int CHUNK = cg_chunk<MT, NB>(), int KS = cg_ks<MT, NB>()>
__global__ __launch_bounds__(256 * KS) void k_cg_pass(const MT* __restrict__ M, int64_t ldm, int d,
                                                      const double* __restrict__ X, int64_t ldx,
                                                      const CgState* __restrict__ st,
                                                      double* __restrict__ work, int64_t wld) {
  if (st->done) return;
  constexpr int NT = 256 * KS;
  __shared__ double pv[CHUNK][NB];
  __shared__ ThinRed<KS, NB> red;
  const int nb = st->nb;
  const int tid = threadIdx.x;
  const int j0 = blockIdx.y * CHUNK;
  REFL_GUARD(nb >= 1 && nb <= NB && j0 < d && ldx >= d, DBG_CG_PASS);
  double rv[(NB * CHUNK + NT - 1) / NT];
#pragma unroll
  for (int u = 0; u < (NB * CHUNK + NT - 1) / NT; ++u) {
    const int e = tid + u * NT;
    const int c = e / CHUNK, j = j0 + e % CHUNK;
    rv[u] = ldsel(X, (int64_t)c * ldx + j, e < NB * CHUNK && c < nb && j < d);
  }
  double m0[8];
  symthin_first<MT, CHUNK, KS>(M, ldm, 0, d, m0);
#pragma unroll
  for (int u = 0; u < (NB * CHUNK + NT - 1) / NT; ++u) {
    const int e = tid + u * NT;
    if (e < NB * CHUNK) pv[e % CHUNK][e / CHUNK] = rv[u];
  }
  lds_barrier();
  symthin_body<MT, NB, CHUNK, KS>(M, ldm, 0, d, pv, work, wld, nb, red, m0);
}

// Grid (row groups of 64, column c), 256 threads: four lanes per row sum
// every fourth chunk of the pass (as k_cg_apply); the update is done by
// lane 0 of each group of four.
template <int NB>
__global__ __launch_bounds__(256) void k_cg_update(const double* __restrict__ work, int64_t wld,
                                                   int nchunk, int d, const double* __restrict__ V,
                                                   const double* __restrict__ U, int64_t ldv,
                                                   CgBufs b, CgState* __restrict__ st,
                                                   const double* __restrict__ pin,
                                                   double* __restrict__ pout, int it,
                                                   int max_iter) {
  if (st->done) return;
  __shared__ double spr[2 * NB + 2][65];  // per-row values of the new partials (k <= NB)
  __shared__ double sq[4 * NB][65];       // the previous partials, a row per value
  __shared__ double sv[3 * 32 + 68];  // gamma, delta of every column, then this column's sums
  const int nb = st->nb, k = st->k, nv = 2 * k + 2;
  const int c = blockIdx.y, nrg = gridDim.x;
  REFL_GUARD(nb >= 1 && nb <= NB && nb <= 32 && k <= NB && c < nb && (int)blockIdx.x * 64 < d &&
                 ldv >= d,
             DBG_CG_UPDATE);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sub = tid & 3;
  const int row = blockIdx.x * 64 + (tid >> 2);
  const bool owner = sub == 0 && row < d;
  constexpr int KV = NB < 8 ? NB : 8;
  const int64_t o = (int64_t)c * ldv + row;
  // Loads that do not wait for any sum come first, without branches.
  double* R = b.R[0];
  double* Wv = b.HR;
  double* ZZ = b.P[1];
  double* S = b.S[0];
  double* P = b.P[0];
  const double rv = ldsel(R, o, owner);
  const double wv = ldsel(Wv, o, owner && it >= 1);
  const double zzp = ldsel(ZZ, o, owner && it >= 2);
  const double sp = ldsel(S, o, owner && it >= 2);
  const double pp = ldsel(P, o, owner && it >= 2);
  const double xv = ldsel(b.Z, o, owner && it >= 1);
  const double* Vb = k > 0 ? V : R;
  const double* Ub = k > 0 ? U : R;
  double ur[KV], vr[KV];
#pragma unroll
  for (int i = 0; i < KV; ++i) {
    ur[i] = ldsel(Ub, (int64_t)i * ldv + row, owner && i < k);
    vr[i] = ldsel(Vb, (int64_t)i * ldv + row, owner && i < k);
  }
  // The state this launch reads, requested up front (a load waited for
  // where it is used costs a round trip to memory each).
  const double th = st->theta[c], tol2 = st->tol2;
  const double rho = st->rho0[lane < nb ? lane : 0];
  const double gprev = st->gam[(it - 1) & 1][c], aprev = st->alpha[(it - 1) & 1][c];
  // The previous partials: value q of the list (gamma, delta of every
  // column when it >= 1, then the 2k sums of this column), a lane per
  // group; all of a wave's values (q = wave + 4u, at most 4 NB) at once.
  const int ngd = it >= 1 ? 2 * nb : 0, nq = ngd + 2 * k;
  auto qsrc = [&](int q) -> int64_t {
    if (q < ngd) {
      const int cc = q >> 1;
      return ((int64_t)cc * nv + 2 * k + (q & 1)) * nrg;
    }
    return ((int64_t)c * nv + (q - ngd)) * nrg;
  };
  double pa[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int q = wave + 4 * u;
    pa[u] = ldsel(pin, (q < nq ? qsrc(q) : 0) + lane, q < nq && lane < nrg);
  }
  // (M - theta) x for the row.
  const int rowc = row < d ? row : d - 1;
  const int nrb = (d + 255) / 256;
  const double* wr = work + (int64_t)c * 256 + (rowc & 255);
  const int rb = rowc >> 8;
  double acc[4] = {0, 0, 0, 0};
  int q = sub;
  for (; q + 12 < nchunk; q += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += wr[thin_block_base<NB>(q + 4 * u, rb, nrb)];
  }
  for (; q < nchunk; q += 4) acc[0] += wr[thin_block_base<NB>(q, rb, nrb)];
  double y = row < d ? (acc[0] + acc[1]) + (acc[2] + acc[3]) : 0.0;
  y += __shfl_xor(y, 1, WAVE);
  y += __shfl_xor(y, 2, WAVE);
  const double xop = it == 0 ? rv : wv;
  y = owner ? y - th * xop : 0.0;
  // Sums of the previous partials: a lane's groups (g = lane, lane + 64,
  // ...) first, then the 64 lanes' sums in LDS, summed in order by thread q.
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int qq = wave + 4 * u;
    if (qq < nq) {  // wave-uniform
      double a = pa[u];
      for (int g = lane + 64; g < nrg; g += 64) a += pin[qsrc(qq) + g];
      sq[qq][lane] = a;
    }
  }
  lds_barrier();
  if (tid < nq) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 16
    for (int g = 0; g < 64; ++g) a[g & 3] += sq[tid][g];
    sv[tid] = (a[0] + a[1]) + (a[2] + a[3]);
  }
  lds_barrier();
  // q = (M - theta) x - V (U^T x - theta V^T x)
  const double* cs = sv + ngd;
  double qv = y;
  for (int i = 0; i < k; ++i) {
    double vi;
    if (i < KV) {
      vi = vr[0];
#pragma unroll
      for (int u = 1; u < KV; ++u) vi = i == u ? vr[u] : vi;
    } else {
      vi = owner ? V[(int64_t)i * ldv + row] : 0.0;
    }
    qv = fma(-vi, cs[i] - th * cs[k + i], qv);
  }
  const bool first = blockIdx.x == 0 && blockIdx.y == 0;
  if (it == 0) {
    // w_0 = A r_0; partials of w_0 (U^T w_0, V^T w_0, gamma_0, delta_0).
    if (owner) Wv[o] = qv;
    const double w0 = owner ? qv : 0.0;
    if (first && tid == 0) st->iters = 0;
    cg_write_parts<KV>(k, c, nrg, w0, ur, vr, U, V, ldv, row, owner, rv * rv, w0 * rv, pout, spr);
    return;
  }
  // Update it - 1: the test is on r_{it-1}, every column (lane cc tests
  // column cc; every wave takes the same vote).
  const int i_up = it - 1;
  const bool miss = lane < nb && !(sv[2 * (lane < nb ? lane : 0)] <= tol2 * rho);
  const bool conv = __ballot(miss) == 0;
  if (conv || i_up >= max_iter) {
    if (first && tid == 0) {
      st->iters = i_up;
      st->done = 1;
    }
    return;
  }
  const double gam = sv[2 * c], del = sv[2 * c + 1];
  double alpha, beta = 0.0;
  if (i_up >= 1) {
    beta = gprev > 0.0 ? gam / gprev : 0.0;
    const double den = del - (aprev != 0.0 ? beta * gam / aprev : 0.0);
    alpha = den != 0.0 ? gam / den : 0.0;
  } else {
    alpha = del != 0.0 ? gam / del : 0.0;
  }
  if (blockIdx.x == 0 && tid == 0) {
    st->gam[it & 1][c] = gam;
    st->alpha[it & 1][c] = alpha;
  }
  if (first && tid == 0) st->iters = it;
  double wn = 0.0, rn = 0.0;
  if (owner) {
    const double zz = i_up >= 1 ? fma(beta, zzp, qv) : qv;
    const double sn = i_up >= 1 ? fma(beta, sp, wv) : wv;
    const double pn = i_up >= 1 ? fma(beta, pp, rv) : rv;
    b.Z[o] = fma(alpha, pn, xv);
    rn = fma(-alpha, sn, rv);
    wn = fma(-alpha, zz, wv);
    ZZ[o] = zz;
    S[o] = sn;
    P[o] = pn;
    R[o] = rn;
    Wv[o] = wn;
  }
  cg_write_parts<KV>(k, c, nrg, wn, ur, vr, U, V, ldv, row, owner, rn * rn, wn * rn, pout, spr);
}

template <int W>
__global__ __launch_bounds__(256) void k_copy_out_w(const uint16_t* __restrict__ X, int64_t ps,
                                                    int dp, int d, double* __restrict__ R,
                                                    int64_t ldr) {
  const int i = blockIdx.y;
  REFL_GUARD(i < d && d <= dp && ps >= (int64_t)dp * dp && ldr >= d, DBG_COPY_OUT);
  for (int j = blockIdx.x * 256 + threadIdx.x; j < d; j += gridDim.x * 256) {
    float x = 0.f;
#pragma unroll
    for (int q = 0; q < W; ++q) x += bf16_to_f32(X[q * ps + (int64_t)i * dp + j]);
    R[(int64_t)i * ldr + j] = (double)x;
  }
}

__global__ __launch_bounds__(256) void k_lincomb(int d, int nb, double a, const double* __restrict__ X,
                                                 int64_t ldx, double b, double* __restrict__ Y,
                                                 int64_t ldy) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= d) return;
  for (int c = 0; c < nb; ++c) {
    double* y = Y + (int64_t)c * ldy + row;
    *y = a * X[(int64_t)c * ldx + row] + (b == 0.0 ? 0.0 : b * *y);
  }
}

// Symmetry check (opt-in): over the 64 x 64 tiles (I, J), I <= J, of the
// full d x d matrix, max_{i<j} |H_ij - H_ji| and max |H_ij|.  The maxima
// are taken on the bit patterns of the absolute values (non-negative
// doubles order like their bits; a NaN's bits exceed every number's), so a
// NaN anywhere survives into the result.
__global__ __launch_bounds__(256) void k_asym_max(const double* __restrict__ H, int64_t ldh, int d,
                                                  unsigned long long* __restrict__ out) {
  const int I = blockIdx.y, J = blockIdx.x;
  if (I > J) return;
  __shared__ double t[64][65];
  const int i0 = I * 64, j0 = J * 64;
  unsigned long long amax = 0, asym = 0;
  // Tile (J, I) transposed into LDS.
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e / 64, c = e % 64;
    const int gi = j0 + r, gj = i0 + c;
    double v = 0.0;
    if (gi < d && gj < d) {
      v = H[(int64_t)gi * ldh + gj];
      amax = max(amax, (unsigned long long)__double_as_longlong(fabs(v)));
    }
    t[c][r] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e / 64, c = e % 64;
    const int gi = i0 + r, gj = j0 + c;
    if (gi < d && gj < d && gi < gj) {
      const double v = H[(int64_t)gi * ldh + gj];
      if (I != J) amax = max(amax, (unsigned long long)__double_as_longlong(fabs(v)));
      asym = max(asym, (unsigned long long)__double_as_longlong(fabs(v - t[r][c])));
    }
  }
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    amax = max(amax, (unsigned long long)__shfl_xor((long long)amax, o, WAVE));
    asym = max(asym, (unsigned long long)__shfl_xor((long long)asym, o, WAVE));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out, asym);
    atomicMax(out + 1, amax);
  }
}

// ---------------------------------------------------------------- launchers
static inline int nblocks(int64_t n, int per) { return (int)((n + per - 1) / per); }

hipError_t launch_mirror_upper(const double* H, int64_t ldh, int d, double* Hf, int dp,
                               hipStream_t st) {
  const int nt = dp / 64;
  hipLaunchKernelGGL(k_mirror_upper, dim3(nt, nt), dim3(256), 0, st, H, ldh, d, Hf, dp);
  return hipGetLastError();
}

hipError_t launch_asym_max(const double* H, int64_t ldh, int d, double* scal, int slot,
                           hipStream_t st) {
  hipError_t e = hipMemsetAsync(scal + slot, 0, 2 * sizeof(double), st);
  if (e != hipSuccess) return e;
  const int nt = nblocks(d, 64);
  hipLaunchKernelGGL(k_asym_max, dim3(nt, nt), dim3(256), 0, st, H, ldh, d,
                     reinterpret_cast<unsigned long long*>(scal + slot));
  return hipGetLastError();
}

hipError_t launch_scale_inf(const double* Hf, int dp, int d, double s, int norm, int scale_given,
                            double alpha_given, double* rowsum, double* scal, hipStream_t st) {
  double* flags = rowsum + dp;
  hipLaunchKernelGGL(k_rowabs, dim3(nblocks(d, 4)), dim3(256), 0, st, Hf, dp, d, s, norm, rowsum,
                     flags);
  hipLaunchKernelGGL(k_scale_finish, dim3(1), dim3(256), 0, st, rowsum, flags, d, norm,
                     scale_given, alpha_given, scal);
  return hipGetLastError();
}

static int grid_elems(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b > 65536 ? 65536 : b);
}

hipError_t launch_init_x0_f64(const double* Hf, int dp, int d, double s, const double* scal,
                              double* X, hipStream_t st) {
  hipLaunchKernelGGL(k_init_x0<double>, dim3(grid_elems((int64_t)dp * dp)), dim3(256), 0, st, Hf,
                     dp, d, s, scal, X);
  return hipGetLastError();
}
hipError_t launch_init_x0_f32(const double* Hf, int dp, int d, double s, const double* scal,
                              float* X, hipStream_t st) {
  hipLaunchKernelGGL(k_init_x0<float>, dim3(grid_elems((int64_t)dp * dp)), dim3(256), 0, st, Hf,
                     dp, d, s, scal, X);
  return hipGetLastError();
}
hipError_t launch_init_x0_words(int words, const double* Hf, int dp, int d, double s,
                                const double* scal, uint16_t* X, int64_t ps, float* H32,
                                hipStream_t st) {
  const dim3 g(grid_elems((int64_t)dp * dp));
  switch (words) {
    case 1: hipLaunchKernelGGL(k_init_x0_w<1>, g, dim3(256), 0, st, Hf, dp, d, s, scal, X, ps, H32); break;
    case 2: hipLaunchKernelGGL(k_init_x0_w<2>, g, dim3(256), 0, st, Hf, dp, d, s, scal, X, ps, H32); break;
    case 3: hipLaunchKernelGGL(k_init_x0_w<3>, g, dim3(256), 0, st, Hf, dp, d, s, scal, X, ps, H32); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_shifted_f32(const double* Hf, int dp, int d, double s, float* Hs,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_shifted_f32, dim3(grid_elems((int64_t)dp * dp)), dim3(256), 0, st, Hf, dp,
                     d, s, Hs);
  return hipGetLastError();
}
hipError_t launch_reduce_sum(const double* partials, int n, double* scal, int slot,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, st, partials, n, scal, slot);
  return hipGetLastError();
}
hipError_t launch_reduce_ranges(const double* partials, const int* begin, const int* slot, int nq,
                                double* out, hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_ranges, dim3(nq), dim3(256), 0, st, partials, begin, slot, out);
  return hipGetLastError();
}
hipError_t launch_batch_decide(int nprob, const double* res, const double* trace,
                               const BatchRule* rules, BatchStep* stp, int* live, int* ctl,
                               int par, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_decide, dim3(1), dim3(256), 0, st, nprob, res, trace, rules, stp, live,
                     ctl, par);
  return hipGetLastError();
}
hipError_t launch_reduce_decide(const double* pr, const double* pt, int n, double* scal,
                                const MixedRule* rule, BatchStep* stp, int* live, int* ctl, int par,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_decide<MixedRule>, dim3(1), dim3(256), 0, st, pr, pt, n, scal, rule,
                     stp, live, ctl, par);
  return hipGetLastError();
}
hipError_t launch_reduce_decide(const double* pr, const double* pt, int n, double* scal,
                                const BatchRule* rule, BatchStep* stp, int* live, int* ctl, int par,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_decide<BatchRule>, dim3(1), dim3(256), 0, st, pr, pt, n, scal, rule,
                     stp, live, ctl, par);
  return hipGetLastError();
}
hipError_t launch_trace_f64(const double* X, int dp, int d, double* scal, int slot,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_trace<double>, dim3(1), dim3(256), 0, st, X, dp, d, scal, slot);
  return hipGetLastError();
}
hipError_t launch_trace_f32(const float* X, int dp, int d, double* scal, int slot,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_trace<float>, dim3(1), dim3(256), 0, st, X, dp, d, scal, slot);
  return hipGetLastError();
}
hipError_t launch_trace_words(int words, const uint16_t* X, int64_t ps, int dp, int d,
                              double* scal, int slot, hipStream_t st) {
  switch (words) {
    case 1: hipLaunchKernelGGL(k_trace_w<1>, dim3(1), dim3(256), 0, st, X, ps, dp, d, scal, slot); break;
    case 2: hipLaunchKernelGGL(k_trace_w<2>, dim3(1), dim3(256), 0, st, X, ps, dp, d, scal, slot); break;
    case 3: hipLaunchKernelGGL(k_trace_w<3>, dim3(1), dim3(256), 0, st, X, ps, dp, d, scal, slot); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_copy_out_f64(const double* X, int dp, int d, double* R, int64_t ldr,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_copy_out<double>, dim3(nblocks(d, 256), d), dim3(256), 0, st, X, dp, d, R, ldr);
  return hipGetLastError();
}
hipError_t launch_copy_out_f32(const float* X, int dp, int d, double* R, int64_t ldr,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_copy_out<float>, dim3(nblocks(d, 256), d), dim3(256), 0, st, X, dp, d, R, ldr);
  return hipGetLastError();
}

template <typename T>
static hipError_t sym_in(const double* G, int64_t ldg, int d, const double* scal, T* out, int dp,
                         hipStream_t st) {
  const int nt = dp / 64;
  hipLaunchKernelGGL(k_sym_in<T>, dim3(nt, nt), dim3(256), 0, st, G, ldg, d, scal, out, dp);
  return hipGetLastError();
}
hipError_t launch_sym_in_f64(const double* G, int64_t ldg, int d, const double* scal, double* out,
                             int dp, hipStream_t st) {
  return sym_in<double>(G, ldg, d, scal, out, dp, st);
}
hipError_t launch_sym_in_f32(const double* G, int64_t ldg, int d, const double* scal, float* out,
                             int dp, hipStream_t st) {
  return sym_in<float>(G, ldg, d, scal, out, dp, st);
}
hipError_t launch_copy_out_scaled_f64(const double* X, int dp, int d, const double* scal,
                                      double* R, int64_t ldr, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_out_scaled<double>, dim3(nblocks(d, 256), d), dim3(256), 0, st, X, dp,
                     d, scal, R, ldr);
  return hipGetLastError();
}
hipError_t launch_copy_out_scaled_f32(const float* X, int dp, int d, const double* scal,
                                      double* R, int64_t ldr, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_out_scaled<float>, dim3(nblocks(d, 256), d), dim3(256), 0, st, X, dp,
                     d, scal, R, ldr);
  return hipGetLastError();
}
constexpr int DOT_BLOCKS = 512;
int dot_partials() { return DOT_BLOCKS; }
hipError_t launch_dot_f64(const double* A, const double* B, int64_t n, double* partials,
                          double* scal, int slot, hipStream_t st) {
  hipLaunchKernelGGL(k_dot<double>, dim3(DOT_BLOCKS), dim3(256), 0, st, A, B, n, partials);
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, st, partials, DOT_BLOCKS, scal, slot);
  return hipGetLastError();
}
hipError_t launch_dot_f32(const float* A, const float* B, int64_t n, double* partials,
                          double* scal, int slot, hipStream_t st) {
  hipLaunchKernelGGL(k_dot<float>, dim3(DOT_BLOCKS), dim3(256), 0, st, A, B, n, partials);
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, st, partials, DOT_BLOCKS, scal, slot);
  return hipGetLastError();
}

int diff_fro_partials(int d) { return nblocks(d, 4); }
hipError_t launch_diff_fro_upper(const double* A, int64_t lda, const double* B, int64_t ldb, int d,
                                 double* partials, double* scal, int slot, hipStream_t st) {
  const int nb = nblocks(d, 4);
  hipLaunchKernelGGL(k_diff_fro_upper, dim3(nb), dim3(256), 0, st, A, lda, B, ldb, d, partials);
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, st, partials, nb, scal, slot);
  return hipGetLastError();
}
hipError_t launch_copy_upper(const double* A, int64_t lda, double* B, int64_t ldb, int d,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_copy_upper, dim3(nblocks(d, 256), d), dim3(256), 0, st, A, lda, B, ldb, d);
  return hipGetLastError();
}

int batch_init_blocks(int dp) { return (int)(((int64_t)dp * dp + INIT_CHUNK - 1) / INIT_CHUNK); }

hipError_t launch_batch_setup(int fp64, const BatchDesc* desc, int ng, const int* mirror_begin,
                              int mirror_blocks, const int* row_begin, int row_blocks,
                              const int* init_begin, int init_blocks, double* trace,
                              hipStream_t st) {
  if (ng <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_mirror, dim3(mirror_blocks), dim3(256), 0, st, desc, mirror_begin,
                     (const int*)nullptr, ng);
  hipLaunchKernelGGL(k_batch_rowabs, dim3(row_blocks), dim3(256), 0, st, desc, row_begin,
                     (const int*)nullptr, ng);
  hipLaunchKernelGGL(k_batch_scale_finish, dim3(ng), dim3(256), 0, st, desc, (const int*)nullptr);
  if (fp64) {
    hipLaunchKernelGGL(k_batch_init<double>, dim3(init_blocks), dim3(256), 0, st, desc,
                       init_begin, (const int*)nullptr, ng);
    hipLaunchKernelGGL(k_batch_trace<double>, dim3(ng), dim3(256), 0, st, desc,
                       (const int*)nullptr, trace);
  } else {
    hipLaunchKernelGGL(k_batch_init<float>, dim3(init_blocks), dim3(256), 0, st, desc,
                       init_begin, (const int*)nullptr, ng);
    hipLaunchKernelGGL(k_batch_trace<float>, dim3(ng), dim3(256), 0, st, desc,
                       (const int*)nullptr, trace);
  }
  return hipGetLastError();
}

hipError_t launch_batch_copy(int fp64, const BatchDesc* desc, const int* begin, const int* ids,
                             int ng, int nblocks_total, int to_hf, hipStream_t st) {
  if (ng <= 0 || nblocks_total <= 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(k_batch_copy<double>, dim3(nblocks_total), dim3(256), 0, st, desc, begin,
                       ids, ng, to_hf);
  else
    hipLaunchKernelGGL(k_batch_copy<float>, dim3(nblocks_total), dim3(256), 0, st, desc, begin,
                       ids, ng, to_hf);
  return hipGetLastError();
}

// Thin products: column chunk CH = 256 for up to 16 columns, 128 above.
template <typename MT>
static hipError_t thin_dispatch(const MT* M, int64_t ldm, int64_t ps, int d, const double* V,
                                int64_t ldv, int nb, double* Y, int64_t ldy, double* work,
                                hipStream_t st) {
  const int64_t wld = d;
  const int rows = nblocks(d, 64);
#define REFL_THIN(NBV, CHV)                                                                      \
  {                                                                                              \
    const int nch = nblocks(d, CHV);                                                             \
    hipLaunchKernelGGL((k_thin_partial<MT, NBV, CHV>), dim3(rows, nch), dim3(256), 0, st, M, ldm, \
                       ps, d, V, ldv, nb, work, wld);                                            \
    hipLaunchKernelGGL((k_thin_finish<NBV, false>), dim3(nblocks(d, 256), nb), dim3(256), 0, st,  \
                       work, wld, nch, d, nb, Y, ldy);                                           \
  }
  if (nb <= 0) return hipSuccess;
  if (nb <= 1) REFL_THIN(1, 512)
  else if (nb <= 4) REFL_THIN(4, 256)
  else if (nb <= 8) REFL_THIN(8, 256)
  else if (nb <= 16) REFL_THIN(16, 256)
  else if (nb <= 32) REFL_THIN(32, 128)
  else return hipErrorInvalidValue;
#undef REFL_THIN
  return hipGetLastError();
}

hipError_t thin_gemm_f64(const double* M, int64_t ldm, int d, const double* V, int64_t ldv, int nb,
                         double* Y, int64_t ldy, double* work, hipStream_t st) {
  return thin_dispatch<double>(M, ldm, 0, d, V, ldv, nb, Y, ldy, work, st);
}
hipError_t thin_gemm_f32(const float* M, int64_t ldm, int d, const double* V, int64_t ldv, int nb,
                         double* Y, int64_t ldy, double* work, hipStream_t st) {
  return thin_dispatch<float>(M, ldm, 0, d, V, ldv, nb, Y, ldy, work, st);
}
hipError_t thin_gemm_words(int words, const uint16_t* X, int ld, int64_t ps, int d,
                           const double* V, int64_t ldv, int nb, double* Y, int64_t ldy,
                           double* work, hipStream_t st) {
  switch (words) {
    case 1: return thin_dispatch<WordsM<1>>(reinterpret_cast<const WordsM<1>*>(X), ld, ps, d, V, ldv, nb, Y, ldy, work, st);
    case 2: return thin_dispatch<WordsM<2>>(reinterpret_cast<const WordsM<2>*>(X), ld, ps, d, V, ldv, nb, Y, ldy, work, st);
    case 3: return thin_dispatch<WordsM<3>>(reinterpret_cast<const WordsM<3>*>(X), ld, ps, d, V, ldv, nb, Y, ldy, work, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_copy_out_words(int words, const uint16_t* X, int64_t ps, int dp, int d,
                                 double* R, int64_t ldr, hipStream_t st) {
  const dim3 g(nblocks(d, 256), d);
  switch (words) {
    case 1: hipLaunchKernelGGL(k_copy_out_w<1>, g, dim3(256), 0, st, X, ps, dp, d, R, ldr); break;
    case 2: hipLaunchKernelGGL(k_copy_out_w<2>, g, dim3(256), 0, st, X, ps, dp, d, R, ldr); break;
    case 3: hipLaunchKernelGGL(k_copy_out_w<3>, g, dim3(256), 0, st, X, ps, dp, d, R, ldr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t lincomb(int d, int nb, double a, const double* X, int64_t ldx, double b, double* Y,
                   int64_t ldy, hipStream_t st) {
  hipLaunchKernelGGL(k_lincomb, dim3(nblocks(d, 256)), dim3(256), 0, st, d, nb, a, X, ldx, b, Y, ldy);
  return hipGetLastError();
}
hipError_t gram(const double* A, int64_t lda, int na, const double* B, int64_t ldb, int nb, int d,
                double* G, double* work, hipStream_t st) {
  const int nblk = nblocks(d, 64);
  hipLaunchKernelGGL(k_gram_partial, dim3(nblk), dim3(256), 0, st, A, lda, na, B, ldb, nb, d, work);
  hipLaunchKernelGGL(k_gram_finish, dim3(nblocks(na * nb, 4)), dim3(256), 0, st, work, nblk,
                     na * nb, G);
  return hipGetLastError();
}
hipError_t block_axpy(int d, int na, int nb, double alpha, double* Y, int64_t ldy, double beta,
                      const double* A, int64_t lda, const double* C, hipStream_t st) {
  hipLaunchKernelGGL(k_block_axpy, dim3(nblocks(d, 256)), dim3(256), 0, st, d, na, nb, alpha, Y,
                     ldy, beta, A, lda, C);
  return hipGetLastError();
}
hipError_t col_axpy(int d, int nb, double* Y, int64_t ldy, const double* coef, const double* X,
                    int64_t ldx, hipStream_t st) {
  hipLaunchKernelGGL(k_col_axpy, dim3(nblocks(d, 256)), dim3(256), 0, st, d, nb, Y, ldy, coef, X, ldx);
  return hipGetLastError();
}
hipError_t form_reflector(const double* V, int64_t ldv, int k, int d, double* R, int64_t ldr,
                          hipStream_t st) {
  const int nt = nblocks(d, 64);
  hipLaunchKernelGGL(k_form_reflector, dim3(nt, nt), dim3(256), 0, st, V, ldv, k, d, R, ldr);
  return hipGetLastError();
}
hipError_t form_sym_pair(const double* Z, const double* V, int64_t ld, int k, int d, double c,
                         double* out, int64_t ldo, hipStream_t st) {
  if (k < 0 || k > 32) return hipErrorInvalidValue;
  const int nt = nblocks(d, 64);
  hipLaunchKernelGGL(k_form_sym_pair, dim3(nt, nt), dim3(256), 0, st, Z, V, ld, k, d, c, out, ldo);
  return hipGetLastError();
}
hipError_t random_block(double* V, int64_t ldv, int d, int nb, uint64_t seed, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_random_block, dim3(nblocks(d, 256), std::min(nb, 1024)), dim3(256), 0, st, V, ldv, d,
                     nb, seed);
  return hipGetLastError();
}

size_t cg_state_bytes() {
  static_assert(sizeof(CgState) == sizeof(CgHost), "CgState and CgHost must match");
  return sizeof(CgState);
}
// nb (k + 2) per group for the Chronopoulos-Gear solve, two parities of
// nb (2k + 2) per group for the pipelined one.
size_t cg_part_doubles(int d) { return (size_t)2 * nblocks(d, 64) * 32 * 66; }
size_t thin_work_doubles(int d) {
  const size_t dr = (size_t)nblocks(d, 256) * 256;  // the block layout rounds d up
  const size_t a = (size_t)nblocks(d, 128) * 32 * dr;
  const size_t b = (size_t)nblocks(d, SRC) * 32 * dr;
  const size_t c = (size_t)nblocks(d, CG_SRC) * 32 * dr;  // the CG pass
  return std::max(a, std::max(b, c));
}
size_t gram_work_doubles(int d) { return (size_t)nblocks(d, 64) * 32 * 32; }

// Block widths the thin products are instantiated for: exact up to 8
// columns (the loop over columns is unrolled, so padding costs FMAs and LDS
// reads), then 12, 16, 24 and 32.
#define REFL_NB_DISPATCH(nb, X)                                                                  \
  if ((nb) == 1) X(1) else if ((nb) == 2) X(2) else if ((nb) == 3) X(3)                          \
  else if ((nb) == 4) X(4) else if ((nb) == 5) X(5) else if ((nb) == 6) X(6)                     \
  else if ((nb) == 7) X(7) else if ((nb) == 8) X(8) else if ((nb) <= 12) X(12)                   \
  else if ((nb) <= 16) X(16) else if ((nb) <= 24) X(24) else if ((nb) <= 32) X(32)

// Symmetric thin products (Hf, the word iterate): column-lane kernel plus
// the ordered chunk sum.
template <typename MT>
static hipError_t symthin_dispatch(const MT* M, int64_t ldm, int64_t ps, int d, const double* V,
                                   int64_t ldv, int nb, double* Y, int64_t ldy, double* work,
                                   hipStream_t st) {
  const int64_t wld = d;
#define REFL_STHIN(NBV)                                                                          \
  {                                                                                              \
    const dim3 grid(nblocks(d, 256), nblocks(d, symthin_chunk<NBV>()));                          \
    hipLaunchKernelGGL((k_symthin<MT, NBV>), grid, dim3(256 * symthin_ks<NBV>()), 0, st, M, ldm, \
                       ps, d, V, ldv, nb, work, wld);                                            \
    hipLaunchKernelGGL((k_thin_finish<NBV, true>), dim3(nblocks(d, 256), nb), dim3(256), 0, st,   \
                       work, wld, (int)grid.y, d, nb, Y, ldy);                                   \
  }
  if (nb <= 0) return hipSuccess;
  REFL_NB_DISPATCH(nb, REFL_STHIN)
  else return hipErrorInvalidValue;
#undef REFL_STHIN
  return hipGetLastError();
}

hipError_t symthin_f64(const double* M, int64_t ldm, int d, const double* V, int64_t ldv, int nb,
                       double* Y, int64_t ldy, double* work, hipStream_t st) {
  return symthin_dispatch<double>(M, ldm, 0, d, V, ldv, nb, Y, ldy, work, st);
}
hipError_t symthin_words(int words, const uint16_t* X, int ld, int64_t ps, int d, const double* V,
                         int64_t ldv, int nb, double* Y, int64_t ldy, double* work,
                         hipStream_t st) {
  switch (words) {
    case 1: return symthin_dispatch<WordsM<1>>(reinterpret_cast<const WordsM<1>*>(X), ld, ps, d, V, ldv, nb, Y, ldy, work, st);
    case 2: return symthin_dispatch<WordsM<2>>(reinterpret_cast<const WordsM<2>*>(X), ld, ps, d, V, ldv, nb, Y, ldy, work, st);
    case 3: return symthin_dispatch<WordsM<3>>(reinterpret_cast<const WordsM<3>*>(X), ld, ps, d, V, ldv, nb, Y, ldy, work, st);
    default: return hipErrorInvalidValue;
  }
}

// One pipelined CG launch pair (see above); `it` counts from 0 within a
// solve; it = 0 also forms U = M V and the partials of r_0.
hipError_t cg_pipe_iteration(const double* M, const float* M32, int64_t ldm, int d, int nb, int k,
                             const double* V, int64_t ldv, const CgBufs& bufs, void* state,
                             double* work, double* part, int it, int max_iter, hipStream_t st) {
  if (k < 0 || k > nb || nb > 32 || (k > 0 && !bufs.U)) return hipErrorInvalidValue;
  CgState* s = reinterpret_cast<CgState*>(state);
  const int64_t wld = d;
  const int nrg = nblocks(d, 64);
  const size_t half = (size_t)nrg * 32 * 66;
  double* pin = part + (size_t)((it + 1) & 1) * half;
  double* pout = part + (size_t)(it & 1) * half;
  if (it == 0) {
    // U = M V (k columns), with the matrix the passes read.
    if (k > 0) {
      const hipError_t e =
          M32 ? symthin_dispatch<float>(M32, ldm, 0, d, V, ldv, k, bufs.U, ldv, work, st)
              : symthin_dispatch<double>(M, ldm, 0, d, V, ldv, k, bufs.U, ldv, work, st);
      if (e != hipSuccess) return e;
    }
  }
#define REFL_CGP_PASS(MT, MP, NBV)                                                               \
  {                                                                                              \
    constexpr int CH = cg_chunk<MT, NBV>();                                                      \
    nchunk = nblocks(d, CH);                                                                     \
    hipLaunchKernelGGL((k_cg_pass<MT, NBV>), dim3(nblocks(d, 256), nchunk),                      \
                       dim3(256 * cg_ks<MT, NBV>()), 0, st, MP, ldm, d,                          \
                       it == 0 ? bufs.R[0] : bufs.HR, ldv, s, work, wld);                        \
  }
#define REFL_CGP(NBV)                                                                            \
  {                                                                                              \
    if (it == 0)                                                                                 \
      hipLaunchKernelGGL((k_cg_init<NBV>), dim3(nrg, nb), dim3(256), 0, st, d, V, bufs.U, ldv,   \
                         bufs.R[0], s, pin);                                                     \
    int nchunk = 0;                                                                              \
    if (M32) REFL_CGP_PASS(float, M32, NBV)                                                      \
    else REFL_CGP_PASS(double, M, NBV)                                                           \
    hipLaunchKernelGGL((k_cg_update<NBV>), dim3(nrg, nb), dim3(256), 0, st, work, wld, nchunk, d, \
                       V, bufs.U, ldv, bufs, s, pin, pout, it, max_iter);                        \
  }
  REFL_NB_DISPATCH(nb, REFL_CGP)
  else return hipErrorInvalidValue;
#undef REFL_CGP
#undef REFL_CGP_PASS
  return hipGetLastError();
}

// One CG iteration (two launches); `it` counts from 0 within a solve.// One CG iteration (two launches); `it` counts from 0 within a solve.
hipError_t cg_iteration(const double* M, const float* M32, int64_t ldm, int d, int nb,
                        const double* V, int64_t ldv, const CgBufs& bufs, void* state,
                        double* work, double* part, int it, int max_iter, hipStream_t st) {
  CgState* s = reinterpret_cast<CgState*>(state);
  // The step's set-up loads row pairs with 16-byte loads: the vector blocks
  // need an even leading dimension and 16-byte aligned columns.
  if ((ldv & 1) || (reinterpret_cast<uintptr_t>(V) | reinterpret_cast<uintptr_t>(bufs.HR) |
                    reinterpret_cast<uintptr_t>(bufs.Z) | reinterpret_cast<uintptr_t>(bufs.R[0]) |
                    reinterpret_cast<uintptr_t>(bufs.R[1]) | reinterpret_cast<uintptr_t>(bufs.P[0]) |
                    reinterpret_cast<uintptr_t>(bufs.P[1]) | reinterpret_cast<uintptr_t>(bufs.S[0]) |
                    reinterpret_cast<uintptr_t>(bufs.S[1])) & 15)
    return hipErrorInvalidValue;
  const int64_t wld = d;
  const int nrb = nblocks(d, 64);
#define REFL_CG_STEP(MT, MP, NBV)                                                                \
  {                                                                                              \
    constexpr int CH = cg_chunk<MT, NBV>();                                                      \
    nchunk = nblocks(d, CH);                                                                     \
    hipLaunchKernelGGL((k_cg_step<MT, NBV>), dim3(nblocks(d, 256), nchunk),                      \
                       dim3(256 * cg_ks<MT, NBV>()), 0, st, MP, ldm, d, V, ldv, bufs, s, part,   \
                       nrb, work, wld, it, max_iter);                                            \
  }
#define REFL_CG(NBV)                                                                             \
  {                                                                                              \
    int nchunk = 0;                                                                              \
    if (M32) REFL_CG_STEP(float, M32, NBV)                                                       \
    else REFL_CG_STEP(double, M, NBV)                                                            \
    hipLaunchKernelGGL((k_cg_apply<NBV>), dim3(nrb, nb), dim3(256), 0, st, work, wld, nchunk, d, \
                       V, ldv, bufs.R[it & 1], bufs.HR, s, part);                                \
  }
  REFL_NB_DISPATCH(nb, REFL_CG)
  else return hipErrorInvalidValue;
#undef REFL_CG
#undef REFL_CG_STEP
  return hipGetLastError();
}

}  // namespace refl
