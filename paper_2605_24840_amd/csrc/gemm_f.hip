// Symmetric FP64 / FP32 products of the Newton-Schulz step (section 3.3,
// eq. NS) on 16x16x4 MFMA, with the step's elementwise work fused into the
// epilogue.
//
// One Newton-Schulz step X <- X (3I - X^2)/2 is written as two products,
//   GEMM_RESIDUAL:  T = X X,  N = I - T            (and ||N||_F^2 = ||X^2 - I||_F^2)
//   GEMM_UPDATE:    P = X N,  X_new = X + P/2      (and trace X_new)
// which equals X (3I - X^2)/2 exactly in real arithmetic.  X and N are
// symmetric and commute, so both products are symmetric: only the tiles
// (I, J) with I <= J are multiplied, and each result tile is stored twice,
// at (I, J) and transposed at (J, I).  Because X = X^T and N = N^T, the
// (i, j) entry of either product is the dot product of row i of the left
// factor with row j of the right factor, so both operands stream row panels
// with K contiguous.
//
// Work-group: 256 threads = 4 waves, output tile 128 x 128, each wave a
// 64 x 64 quadrant = 4 x 4 MFMA blocks of 16 x 16.  K advances 16 at a time
// through two LDS buffers (global loads of step k+1 overlap the MFMAs of
// step k).  The epilogue stages the tile in LDS, so that the direct and the
// transposed stores are both row-contiguous.
#include "common.h"
#include "dbg.h"
#include "launch.h"
#include "rule.h"

namespace refl {

REFL_DBG_UNIT(gemm_f)

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct FMfma;
template <>
struct FMfma<double> {
  typedef f64x4_t acc_t;
  // 16x16 result block: lane l, register r holds row 4r + l/16, column l%16.
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct FMfma<float> {
  typedef f32x4_t acc_t;
  // 16x16 result block: lane l, register r holds row 4(l/16) + r, column l%16.
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Tile edge TS in {32, 64, 96, 128}: 4 waves in 2 x 2, each a (TS/2)^2
// quadrant of MB x MB MFMA blocks of 16 x 16 (one block at TS = 32, which
// spreads orders of a few hundred to a thousand over all compute units).
template <typename T, int TS>
struct FCfg {
  static_assert(TS == 32 || TS == 64 || TS == 96 || TS == 128, "tile edge");
  static constexpr int BK = 16;
  static constexpr int LDA = BK + 16 / (int)sizeof(T);  // 16 B pad per LDS row
  static constexpr int OPER = 2 * 2 * TS * LDA;         // 2 buffers x 2 operands
  static constexpr int SLD = TS + 1;                    // staging row stride
  static constexpr int STG = TS * SLD;
  static constexpr int LDS = OPER > STG ? OPER : STG;
  static constexpr int NV = 8 * (int)sizeof(T) / 16;    // 16 B vectors per thread per operand
  static constexpr int VE = 16 / (int)sizeof(T);        // elements per 16 B
  static constexpr int MB = TS / 32;                    // MFMA blocks per wave and dimension
  static_assert(MB >= 1, "one block per wave at least");
  static constexpr int LPR = TS / VE;                   // 16 B vectors per tile row
  static constexpr int NIT = TS * TS / VE / 256;        // epilogue vectors per thread
  static_assert(NIT * VE * 256 == TS * TS, "epilogue split");
};

// Operand pairs of one tile product: the tile accumulates
// sum_p (rows I of A[p]) (rows J of B[p])^T over the NP pairs, i.e. a product
// whose K runs over the NP pairs one after the other.
template <typename T, int NP>
struct Pairs {
  const T* A[NP];
  const T* B[NP];
};

// One output tile (I, J).  Symmetric modes (RESIDUAL, UPDATE, ADJOINT) take
// I <= J and store the tile twice; GEMM_PLAIN_NEG takes any (I, J) and
// stores -C once.  The tile's partial (||N||_F^2 or trace contribution; 0
// for the other modes) goes to *partial.
template <typename T, int MODE, int NP, int TS>
__device__ __forceinline__ void sym_gemm_f_tile(const Pairs<T, NP>& op, const T* __restrict__ Xold,
                                                T* __restrict__ out, int ld, int d, int dp, int I,
                                                int J, T* lds, double* red,
                                                double* __restrict__ partial) {
  typedef FCfg<T, TS> C;
  typedef FMfma<T> M;
  typedef typename M::acc_t acc_t;
  constexpr bool SYM = MODE != GEMM_PLAIN_NEG;
  constexpr int MB = C::MB;
  const int i0 = I * TS, j0 = J * TS;
  const bool diag = SYM && (I == J);
  REFL_GUARD(I >= 0 && J >= 0 && (!SYM || I <= J) && i0 + TS <= dp && j0 + TS <= dp && d <= dp &&
                 dp <= ld && dp % C::BK == 0,
             DBG_GEMM_F_TILE);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;

  // Loader: thread -> row (tid >> 1), 8 consecutive k at (tid & 1) * 8; the
  // first 2 TS threads load.
  const bool loader = tid < 2 * TS;
  const int lrow = loader ? tid >> 1 : 0, lk = (tid & 1) * 8;
  const int64_t rA = (int64_t)(i0 + lrow) * ld + lk, rB = (int64_t)(j0 + lrow) * ld + lk;
  u32x4_t ra[C::NV], rb[C::NV];

  acc_t acc[MB][MB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][b][r] = 0;

  const int nk = dp / C::BK;
  auto gload = [&](int t) {
    // Slice t of the concatenated K: pair t / nk, slice t % nk (wave-uniform).
    const int p = NP == 1 ? 0 : t / nk;
    const int kt = NP == 1 ? t : t - p * nk;
    const T* A = op.A[0];
    const T* B = op.B[0];
#pragma unroll
    for (int q = 1; q < NP; ++q)
      if (p == q) {
        A = op.A[q];
        B = op.B[q];
      }
    if (!loader) return;
    const u32x4_t* pa = reinterpret_cast<const u32x4_t*>(A + rA + (int64_t)kt * C::BK);
    const u32x4_t* pb = reinterpret_cast<const u32x4_t*>(B + rB + (int64_t)kt * C::BK);
#pragma unroll
    for (int v = 0; v < C::NV; ++v) {
      ra[v] = pa[v];
      rb[v] = pb[v];
    }
  };
  auto sstore = [&](int buf) {
    if (!loader) return;
    T* sa = lds + buf * (2 * TS * C::LDA);
    T* sb = sa + TS * C::LDA;
    u32x4_t* da = reinterpret_cast<u32x4_t*>(sa + lrow * C::LDA + lk);
    u32x4_t* db = reinterpret_cast<u32x4_t*>(sb + lrow * C::LDA + lk);
#pragma unroll
    for (int v = 0; v < C::NV; ++v) {
      da[v] = ra[v];
      db[v] = rb[v];
    }
  };

  const int nkt = NP * nk;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nkt; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nkt) gload(kt + 1);
    const T* sa = lds + cur * (2 * TS * C::LDA);
    const T* sb = sa + TS * C::LDA;
#pragma unroll
    for (int kk = 0; kk < C::BK / 4; ++kk) {
      T av[MB], bv[MB];
      const int kof = kk * 4 + (lane >> 4);
#pragma unroll
      for (int a = 0; a < MB; ++a) av[a] = sa[(wr * (TS / 2) + a * 16 + (lane & 15)) * C::LDA + kof];
#pragma unroll
      for (int b = 0; b < MB; ++b) bv[b] = sb[(wc * (TS / 2) + b * 16 + (lane & 15)) * C::LDA + kof];
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < MB; ++b) acc[a][b] = M::op(av[a], bv[b], acc[a][b]);
    }
    if (kt + 1 < nkt) sstore(cur ^ 1);
    __syncthreads();
  }

  // ---- epilogue: stage the TS x TS result tile ----
  T* stg = lds;
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr * (TS / 2) + a * 16 + M::row(lane, r);
        const int col = wc * (TS / 2) + b * 16 + (lane & 15);
        stg[row * C::SLD + col] = acc[a][b][r];
      }
  __syncthreads();

  // Direct pass: row-contiguous 16 B stores, vector v = it * 256 + tid of the
  // tile (row v / LPR, columns (v % LPR) * VE ..).  In a diagonal tile entry
  // (r, c) takes the value computed at (min, max) so the stored tile is
  // exactly symmetric.
  constexpr int LPR = C::LPR;
  double part = 0.0;
  alignas(16) T vals[C::NIT][C::VE];
#pragma unroll
  for (int it = 0; it < C::NIT; ++it) {
    const int v = it * 256 + tid;
    const int r = v / LPR, cofs = (v % LPR) * C::VE;
    const int gi = i0 + r;
    alignas(16) T xo[C::VE];
    if (MODE == GEMM_UPDATE || MODE == GEMM_ADJOINT) {
      const u32x4_t v = *reinterpret_cast<const u32x4_t*>(Xold + (int64_t)gi * ld + j0 + cofs);
      *reinterpret_cast<u32x4_t*>(xo) = v;
    }
#pragma unroll
    for (int e = 0; e < C::VE; ++e) {
      const int c = cofs + e;
      const int rr = (diag && r > c) ? c : r, cc = (diag && r > c) ? r : c;
      const T v = stg[rr * C::SLD + cc];
      const int gj = j0 + c;
      T n;
      if (MODE == GEMM_RESIDUAL) {
        n = ((gi == gj && gi < d) ? T(1) : T(0)) - v;
        part += (diag ? 1.0 : 2.0) * (double)n * (double)n;
      } else if (MODE == GEMM_UPDATE) {
        n = xo[e] + T(0.5) * v;
        if (gi == gj) part += (double)n;
      } else if (MODE == GEMM_ADJOINT) {
        n = T(0.5) * (xo[e] + v);
      } else {
        n = -v;
      }
      vals[it][e] = n;
    }
    *reinterpret_cast<u32x4_t*>(out + (int64_t)gi * ld + j0 + cofs) =
        *reinterpret_cast<const u32x4_t*>(&vals[it][0]);
  }
  __syncthreads();
  if (SYM && !diag) {
    // Write the final values back to staging, then store the transposed tile.
#pragma unroll
    for (int it = 0; it < C::NIT; ++it) {
      const int v = it * 256 + tid;
      const int r = v / LPR, cofs = (v % LPR) * C::VE;
#pragma unroll
      for (int e = 0; e < C::VE; ++e) stg[r * C::SLD + cofs + e] = vals[it][e];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < C::NIT; ++it) {
      const int v = it * 256 + tid;
      const int c = v / LPR, rofs = (v % LPR) * C::VE;   // output row j0 + c
      alignas(16) T w[C::VE];
#pragma unroll
      for (int e = 0; e < C::VE; ++e) w[e] = stg[(rofs + e) * C::SLD + c];
      *reinterpret_cast<u32x4_t*>(out + (int64_t)(j0 + c) * ld + i0 + rofs) =
          *reinterpret_cast<const u32x4_t*>(w);
    }
  }
  const double tot = block_sum_256(part, red);
  if (tid == 0) *partial = tot;
}

// With live != null and *live == 0 the launch does nothing (a step enqueued
// ahead of the device-side stopping decision of an iteration that stopped).
template <typename T, int MODE, int TS>
__global__ __launch_bounds__(256) void k_sym_gemm_f(const T* __restrict__ A,
                                                    const T* __restrict__ B,
                                                    const T* __restrict__ Xold,
                                                    T* __restrict__ out, int ld, int d, int dp,
                                                    const int2* __restrict__ tiles,
                                                    double* __restrict__ partials,
                                                    const int* __restrict__ live) {
  if (live && *live == 0) return;
  __shared__ T lds[FCfg<T, TS>::LDS];
  __shared__ double red[4];
  const int2 tl = tiles[blockIdx.x];
  Pairs<T, 1> op;
  op.A[0] = A;
  op.B[0] = B;
  sym_gemm_f_tile<T, MODE, 1, TS>(op, Xold, out, ld, d, dp, tl.x, tl.y, lds, red,
                                  partials + blockIdx.x);
}

// Adjoint step of eq. NS (see launch.h): out = (Gb + Gb N + N Gb + Pn X)/2
// with Pn = -X Gb, all operands symmetric except Pn.
template <typename T, int TS>
__global__ __launch_bounds__(256) void k_adjoint_step(const T* __restrict__ Gb,
                                                      const T* __restrict__ N,
                                                      const T* __restrict__ Pn,
                                                      const T* __restrict__ X,
                                                      T* __restrict__ out, int ld, int d, int dp,
                                                      const int2* __restrict__ tiles,
                                                      double* __restrict__ partials) {
  __shared__ T lds[FCfg<T, TS>::LDS];
  __shared__ double red[4];
  const int2 tl = tiles[blockIdx.x];
  Pairs<T, 3> op;
  op.A[0] = Gb;
  op.B[0] = N;
  op.A[1] = N;
  op.B[1] = Gb;
  op.A[2] = Pn;
  op.B[2] = X;
  sym_gemm_f_tile<T, GEMM_ADJOINT, 3, TS>(op, Gb, out, ld, d, dp, tl.x, tl.y, lds, red,
                                          partials + blockIdx.x);
}

// Grouped launch over the tiles of many problems of one tile edge TS: tile
// (p, I, J, slot) reads the problem's iterate pair and N from its descriptor
// and writes its partial to partials[slot]; `parity` selects which of the
// pair holds the current iterate (every problem still iterating has taken
// the same number of steps).
template <typename T, int MODE, int TS>
__global__ __launch_bounds__(256) void k_sym_gemm_f_grouped(const GemmProblem* __restrict__ probs,
                                                            const int4* __restrict__ tiles,
                                                            int parity,
                                                            double* __restrict__ partials,
                                                            const int* __restrict__ live) {
  __shared__ T lds[FCfg<T, TS>::LDS];
  __shared__ double red[4];
  const int4 tl = tiles[blockIdx.x];
  // A problem that has stopped keeps its iterates: its tiles do nothing.
  if (live && !live[tl.x]) return;
  const GemmProblem pr = probs[tl.x];
  T* Xc = reinterpret_cast<T*>(pr.X[parity]);
  T* Xn = reinterpret_cast<T*>(pr.X[parity ^ 1]);
  T* N = reinterpret_cast<T*>(pr.N);
  Pairs<T, 1> op;
  op.A[0] = Xc;
  op.B[0] = MODE == GEMM_RESIDUAL ? Xc : N;
  if (MODE == GEMM_RESIDUAL)
    sym_gemm_f_tile<T, MODE, 1, TS>(op, nullptr, N, pr.ld, pr.d, pr.dp, tl.y, tl.z, lds, red,
                                    partials + tl.w);
  else
    sym_gemm_f_tile<T, MODE, 1, TS>(op, Xc, Xn, pr.ld, pr.d, pr.dp, tl.y, tl.z, lds, red,
                                    partials + tl.w);
}

template <typename T, int TS>
static hipError_t launch_f_ts(int mode, const T* A, const T* B, const T* Xold, T* out, int ld,
                              int d, int dp, const int2* tiles, int ntiles, double* partials,
                              const int* live, hipStream_t st) {
  if (mode == GEMM_RESIDUAL)
    hipLaunchKernelGGL((k_sym_gemm_f<T, GEMM_RESIDUAL, TS>), dim3(ntiles), dim3(256), 0, st, A, B,
                       Xold, out, ld, d, dp, tiles, partials, live);
  else if (mode == GEMM_UPDATE)
    hipLaunchKernelGGL((k_sym_gemm_f<T, GEMM_UPDATE, TS>), dim3(ntiles), dim3(256), 0, st, A, B,
                       Xold, out, ld, d, dp, tiles, partials, live);
  else if (mode == GEMM_PLAIN_NEG)
    hipLaunchKernelGGL((k_sym_gemm_f<T, GEMM_PLAIN_NEG, TS>), dim3(ntiles), dim3(256), 0, st, A, B,
                       Xold, out, ld, d, dp, tiles, partials, live);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_f(int ts, int mode, const T* A, const T* B, const T* Xold, T* out, int ld,
                           int d, int dp, const int2* tiles, int ntiles, double* partials,
                           const int* live, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (dp % ts != 0) return hipErrorInvalidValue;
  switch (ts) {
    case 32: return launch_f_ts<T, 32>(mode, A, B, Xold, out, ld, d, dp, tiles, ntiles, partials, live, st);
    case 64: return launch_f_ts<T, 64>(mode, A, B, Xold, out, ld, d, dp, tiles, ntiles, partials, live, st);
    case 96: return launch_f_ts<T, 96>(mode, A, B, Xold, out, ld, d, dp, tiles, ntiles, partials, live, st);
    case 128: return launch_f_ts<T, 128>(mode, A, B, Xold, out, ld, d, dp, tiles, ntiles, partials, live, st);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t launch_adj(int ts, const T* Gb, const T* N, const T* Pn, const T* X, T* out,
                             int ld, int d, int dp, const int2* tiles, int ntiles,
                             double* partials, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (dp % ts != 0) return hipErrorInvalidValue;
  switch (ts) {
    case 32:
      hipLaunchKernelGGL((k_adjoint_step<T, 32>), dim3(ntiles), dim3(256), 0, st, Gb, N, Pn, X,
                         out, ld, d, dp, tiles, partials);
      break;
    case 64:
      hipLaunchKernelGGL((k_adjoint_step<T, 64>), dim3(ntiles), dim3(256), 0, st, Gb, N, Pn, X,
                         out, ld, d, dp, tiles, partials);
      break;
    case 96:
      hipLaunchKernelGGL((k_adjoint_step<T, 96>), dim3(ntiles), dim3(256), 0, st, Gb, N, Pn, X,
                         out, ld, d, dp, tiles, partials);
      break;
    case 128:
      hipLaunchKernelGGL((k_adjoint_step<T, 128>), dim3(ntiles), dim3(256), 0, st, Gb, N, Pn, X,
                         out, ld, d, dp, tiles, partials);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_adjoint_step_f64(int ts, const double* Gb, const double* N, const double* Pn,
                                   const double* X, double* out, int ld, int d, int dp,
                                   const int2* tiles, int ntiles, double* partials,
                                   hipStream_t st) {
  return launch_adj<double>(ts, Gb, N, Pn, X, out, ld, d, dp, tiles, ntiles, partials, st);
}
hipError_t launch_adjoint_step_f32(int ts, const float* Gb, const float* N, const float* Pn,
                                   const float* X, float* out, int ld, int d, int dp,
                                   const int2* tiles, int ntiles, double* partials,
                                   hipStream_t st) {
  return launch_adj<float>(ts, Gb, N, Pn, X, out, ld, d, dp, tiles, ntiles, partials, st);
}

hipError_t launch_sym_gemm_f64(int ts, int mode, const double* A, const double* B,
                               const double* Xold, double* out, int ld, int d, int dp,
                               const int2* tiles, int ntiles, double* partials, hipStream_t st,
                               const int* live) {
  return launch_f<double>(ts, mode, A, B, Xold, out, ld, d, dp, tiles, ntiles, partials, live, st);
}
hipError_t launch_sym_gemm_f32(int ts, int mode, const float* A, const float* B, const float* Xold,
                               float* out, int ld, int d, int dp, const int2* tiles, int ntiles,
                               double* partials, hipStream_t st, const int* live) {
  return launch_f<float>(ts, mode, A, B, Xold, out, ld, d, dp, tiles, ntiles, partials, live, st);
}

// Blocks of one tile-edge choice that a compute unit holds at once (LDS).
int sym_gemm_f_blocks_per_cu(int fp64, int ts) {
  constexpr int LDS_BYTES = 160 * 1024;
  int lds = 0;
  if (fp64)
    lds = ts == 32 ? FCfg<double, 32>::LDS : ts == 64 ? FCfg<double, 64>::LDS
        : ts == 96 ? FCfg<double, 96>::LDS : FCfg<double, 128>::LDS;
  else
    lds = ts == 32 ? FCfg<float, 32>::LDS : ts == 64 ? FCfg<float, 64>::LDS
        : ts == 96 ? FCfg<float, 96>::LDS : FCfg<float, 128>::LDS;
  const int per = LDS_BYTES / (lds * (fp64 ? 8 : 4) + 64);
  return per < 1 ? 1 : (per > 8 ? 8 : per);
}

template <typename T, int TS>
static void launch_grouped_ts(int mode, const GemmProblem* probs, const int4* tiles, int ntiles,
                              int parity, double* partials, const int* live, hipStream_t st) {
  if (mode == GEMM_RESIDUAL)
    hipLaunchKernelGGL((k_sym_gemm_f_grouped<T, GEMM_RESIDUAL, TS>), dim3(ntiles), dim3(256), 0,
                       st, probs, tiles, parity, partials, live);
  else
    hipLaunchKernelGGL((k_sym_gemm_f_grouped<T, GEMM_UPDATE, TS>), dim3(ntiles), dim3(256), 0, st,
                       probs, tiles, parity, partials, live);
}

hipError_t launch_sym_gemm_grouped(int fp64, int mode, int ts, const GemmProblem* probs,
                                   const int4* tiles, int ntiles, int parity, double* partials,
                                   const int* live, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (mode != GEMM_RESIDUAL && mode != GEMM_UPDATE) return hipErrorInvalidValue;
  switch (ts) {
    case 32:
      if (fp64) launch_grouped_ts<double, 32>(mode, probs, tiles, ntiles, parity, partials, live, st);
      else launch_grouped_ts<float, 32>(mode, probs, tiles, ntiles, parity, partials, live, st);
      break;
    case 64:
      if (fp64) launch_grouped_ts<double, 64>(mode, probs, tiles, ntiles, parity, partials, live, st);
      else launch_grouped_ts<float, 64>(mode, probs, tiles, ntiles, parity, partials, live, st);
      break;
    case 96:
      if (fp64) launch_grouped_ts<double, 96>(mode, probs, tiles, ntiles, parity, partials, live, st);
      else launch_grouped_ts<float, 96>(mode, probs, tiles, ntiles, parity, partials, live, st);
      break;
    case 128:
      if (fp64) launch_grouped_ts<double, 128>(mode, probs, tiles, ntiles, parity, partials, live, st);
      else launch_grouped_ts<float, 128>(mode, probs, tiles, ntiles, parity, partials, live, st);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- small orders
// The whole iteration of one small problem in one work-group (eq. NS with the
// stopping rule of section 3.3): X and N live in LDS for every step, so a
// step costs two in-LDS products and no launch, and the only HBM traffic is
// X_0 in and X_m out.  512 threads = 8 waves; the order is padded to dp, a
// multiple of 16, and the (dp/16)(dp/16 + 1)/2 upper 16 x 16 blocks of each
// product are dealt round-robin to the waves.  Both products are symmetric
// (X and N commute), so each block is computed once and stored with its
// transpose; in a diagonal block the entry (r, c), r > c, takes the value
// computed at (c, r), so both matrices stay exactly symmetric.
//
// Fragments: for a K chunk of 4 VE entries (VE = 16 B / element), lane
// (i + 16 q) reads VE consecutive entries k = k0 + q VE .. of row i of each
// operand in one 16 B LDS load, and MFMA number kk of the chunk takes entry
// kk of it: MFMA input slot q stands for k = k0 + q VE + kk, the same
// permutation of K on both operands, so the chunk's four (FP32) or two (FP64)
// MFMAs sum the products over all 4 VE entries.
template <typename T>
struct SmallCfg {
  static constexpr int VE = 16 / (int)sizeof(T);
  static constexpr int KC = 4 * VE;
  static constexpr int DMAX = sizeof(T) == 8 ? SMALL_MAX_F64 : SMALL_MAX_F32;
  static constexpr int NBMAX = DMAX / 16;
  static constexpr int NW = 8;
  static constexpr int MAXB = (NBMAX * (NBMAX + 1) / 2 + NW - 1) / NW;
  static constexpr int LDS = 2 * DMAX * (DMAX + VE);  // elements: X and N, padded rows
  static_assert(LDS * (int)sizeof(T) <= 160 * 1024 - 256, "two matrices in LDS");
  static_assert(DMAX % 16 == 0, "order padding");
};

// Sum over the 512 threads, returned in every thread (the same value: the
// butterfly gives each lane the same sum, and the wave sums are added in a
// fixed order).
__device__ __forceinline__ double small_all_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < SmallCfg<float>::NW; ++w) t += red[w];
  return t;
}

// acc[t] = (rows 16 bi[t] .. of A) (rows 16 bj[t] .. of B)^T over k < dp,
// for the wave's NBK blocks.  NBK is a template argument so that the MFMAs of
// a chunk issue back to back with no branch between them (a per-block test
// would make each MFMA wait for the previous one's result).  Consecutive
// blocks of a wave mostly share their row block bi, whose fragment is then
// loaded once.
template <typename T, int NBK>
__device__ __forceinline__ void small_products(const T* A, const T* B, int ldx, int dp,
                                               const int (&bi)[SmallCfg<T>::MAXB],
                                               const int (&bj)[SmallCfg<T>::MAXB],
                                               typename FMfma<T>::acc_t (&acc)[SmallCfg<T>::MAXB],
                                               int lane) {
  typedef SmallCfg<T> C;
  typedef FMfma<T> M;
  typedef T vec_t __attribute__((ext_vector_type(C::VE)));
#pragma unroll
  for (int t = 0; t < NBK; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[t][r] = 0;
  const int row = lane & 15, q = lane >> 4;
  for (int k0 = 0; k0 < dp; k0 += C::KC) {
    vec_t a[NBK], b[NBK];
#pragma unroll
    for (int t = 0; t < NBK; ++t) {
      if (t == 0 || bi[t] != bi[t - 1])
        a[t] = *reinterpret_cast<const vec_t*>(A + (bi[t] * 16 + row) * ldx + k0 + q * C::VE);
      else
        a[t] = a[t - 1];
      b[t] = *reinterpret_cast<const vec_t*>(B + (bj[t] * 16 + row) * ldx + k0 + q * C::VE);
    }
#pragma unroll
    for (int kk = 0; kk < C::VE; ++kk)
#pragma unroll
      for (int t = 0; t < NBK; ++t) acc[t] = M::op(a[t][kk], b[t][kk], acc[t]);
  }
}

// small_products for a wave-uniform block count nblk <= MAXB.
template <typename T, int NBK = 1>
__device__ __forceinline__ void small_products_n(int nblk, const T* A, const T* B, int ldx, int dp,
                                                 const int (&bi)[SmallCfg<T>::MAXB],
                                                 const int (&bj)[SmallCfg<T>::MAXB],
                                                 typename FMfma<T>::acc_t (&acc)[SmallCfg<T>::MAXB],
                                                 int lane) {
  if (nblk == NBK) {
    small_products<T, NBK>(A, B, ldx, dp, bi, bj, acc, lane);
  } else if constexpr (NBK < SmallCfg<T>::MAXB) {
    small_products_n<T, NBK + 1>(nblk, A, B, ldx, dp, bi, bj, acc, lane);
  }
}

template <typename T>
__global__ __launch_bounds__(512) void k_ns_small(const SmallProb* __restrict__ probs,
                                                  const BatchRule* __restrict__ rules,
                                                  BatchStep* __restrict__ stp) {
  typedef SmallCfg<T> C;
  typedef FMfma<T> M;
  typedef typename M::acc_t acc_t;
  __shared__ __attribute__((aligned(16))) T lds[C::LDS];
  __shared__ double red[2][C::NW];
  const SmallProb pr = probs[blockIdx.x];
  const int d = pr.d, dp = (d + 15) & ~15, ldx = dp + C::VE;
  // The host sends only orders 1 .. DMAX (and pr.dp >= d); anything else
  // leaves the step record untouched (state BATCH_LIVE) and no memory read.
  if (d < 1 || dp > C::DMAX || pr.dp < d) return;
  T* Xs = lds;
  T* Ns = lds + dp * ldx;
  // wave is uniform across the wave; readfirstlane lets the block bookkeeping
  // below live in scalar registers.
  const int tid = threadIdx.x, lane = tid & (WAVE - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);

  // This wave's upper blocks (I, J), I <= J: a contiguous piece of the
  // row-major list of the upper triangle (so that its blocks mostly share a
  // row block), the nbu % NW longer pieces to the first waves, which sit on
  // different SIMDs.
  const int nb = dp / 16, nbu = nb * (nb + 1) / 2;
  const int qn = nbu / C::NW, rn = nbu % C::NW;
  const int nblk = qn + (wave < rn ? 1 : 0);
  const int first = wave * qn + min(wave, rn);
  int bi[C::MAXB], bj[C::MAXB];
  {
    int idx = first, I = 0;
    while (I < nb && idx >= nb - I) {
      idx -= nb - I;
      ++I;
    }
    int J = I + idx;
#pragma unroll
    for (int t = 0; t < C::MAXB; ++t) {
      bi[t] = t < nblk ? I : 0;
      bj[t] = t < nblk ? J : 0;
      if (++J == nb) {
        ++I;
        J = I;
      }
    }
  }

  const T* X0 = reinterpret_cast<const T*>(pr.X[0]);
  for (int e = tid; e < dp * dp; e += 512) {
    const int i = e / dp, j = e - i * dp;
    Xs[i * ldx + j] = (i < d && j < d) ? X0[(int64_t)i * pr.dp + j] : T(0);
  }
  BatchStep s = stp[pr.slot];
  const BatchRule ru = rules[pr.slot];
  // The rule stops by the step cap at the latest; the bound below only
  // guards the loop itself.
  const int hard = max(max(ru.fixed_steps, ru.max_iter), 0);
  __syncthreads();

  acc_t acc[C::MAXB];
  int m = 0;
  for (;; ++m) {
    // GEMM_RESIDUAL: N = I - X X, ||N||_F^2.
    small_products_n<T>(nblk, Xs, Xs, ldx, dp, bi, bj, acc, lane);
    double part = 0.0;
#pragma unroll
    for (int t = 0; t < C::MAXB; ++t)
      if (t < nblk) {
        const bool dg = bi[t] == bj[t];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = bi[t] * 16 + M::row(lane, r), gj = bj[t] * 16 + (lane & 15);
          if (dg && gi > gj) continue;
          const T n = ((gi == gj && gi < d) ? T(1) : T(0)) - acc[t][r];
          Ns[gi * ldx + gj] = n;
          Ns[gj * ldx + gi] = n;
          part += (gi == gj ? 1.0 : 2.0) * (double)n * (double)n;
        }
      }
    const double r2 = small_all_sum(part, red[0]);
    if (batch_rule(s, ru, sqrt(fmax(r2, 0.0)), m, m & 1)) break;
    if (m >= hard) {
      s.state = BATCH_STOPPED;
      s.par = m & 1;
      break;
    }
    // GEMM_UPDATE: X <- X + (X N)/2, trace of the new iterate.
    small_products_n<T>(nblk, Xs, Ns, ldx, dp, bi, bj, acc, lane);
    double tp = 0.0;
#pragma unroll
    for (int t = 0; t < C::MAXB; ++t)
      if (t < nblk)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = bi[t] * 16 + M::row(lane, r), gj = bj[t] * 16 + (lane & 15);
          const T n = Xs[gi * ldx + gj] + T(0.5) * acc[t][r];
          acc[t][r] = n;
          if (gi == gj) tp += (double)n;
        }
    __syncthreads();  // every product has read X and N
#pragma unroll
    for (int t = 0; t < C::MAXB; ++t)
      if (t < nblk) {
        const bool dg = bi[t] == bj[t];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = bi[t] * 16 + M::row(lane, r), gj = bj[t] * 16 + (lane & 15);
          if (dg && gi > gj) continue;
          Xs[gi * ldx + gj] = acc[t][r];
          Xs[gj * ldx + gi] = acc[t][r];
        }
      }
    s.trace = small_all_sum(tp, red[1]);
  }

  // X_m to X[m & 1], the whole dp x dp buffer (zero outside d x d).
  T* Xo = reinterpret_cast<T*>((m & 1) ? pr.X[1] : pr.X[0]);
  const int gdp = pr.dp;
  for (int e = tid; e < gdp * gdp; e += 512) {
    const int i = e / gdp, j = e - i * gdp;
    Xo[(int64_t)i * gdp + j] = (i < dp && j < dp) ? Xs[i * ldx + j] : T(0);
  }
  if (tid == 0) stp[pr.slot] = s;
}

hipError_t launch_ns_small(int fp64, const SmallProb* probs, int nprob, const BatchRule* rules,
                           BatchStep* stp, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(k_ns_small<double>, dim3(nprob), dim3(512), 0, st, probs, rules, stp);
  else
    hipLaunchKernelGGL(k_ns_small<float>, dim3(nprob), dim3(512), 0, st, probs, rules, stp);
  return hipGetLastError();
}

}  // namespace refl
