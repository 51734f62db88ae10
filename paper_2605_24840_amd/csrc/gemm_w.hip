// Symmetric products of the Newton-Schulz step (section 3.2, eq. NS) on
// BF16 MFMA with FP32 accumulation, for matrices held as W BF16 words per
// entry (x ~= w0 + w1 + w2, each word the round-to-nearest-even BF16 of the
// remainder left by the words before it).  The product of two such matrices
// keeps the word products whose combined weight is at least 2^-16 (W = 2:
// w0w0 + w0w1 + w1w0, "bf16x3") or 2^-24 (W = 3: six products, "bf16x6");
// the split-BF16 technique of Henry, Tang and Heinecke (ARITH 2019).
//
// The two products of one step and their fused epilogues are the same as in
// gemm_f.hip (GEMM_RESIDUAL: N = I - X X; GEMM_UPDATE: X_new = X + X N / 2),
// with the result re-split into W words on store.  X enters the update as
// the exact FP32 sum of its words.
//
// Work-group: 256 threads = 4 waves, output tile 128 x 128, each wave a
// 64 x 64 quadrant = 2 x 2 blocks of the 32x32x16 BF16 MFMA.  K advances 32
// at a time through two LDS buffers.  LDS rows are 32 BF16 + 16 B of pad
// (80 B), so the 16-byte fragment reads of 16 consecutive rows hit distinct
// banks.
#include "common.h"
#include "launch.h"

namespace refl {

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

template <int W>
struct WCfg {
  static constexpr int BK = 32;
  static constexpr int LDA = BK + 8;                    // BF16 elements per LDS row (80 B)
  static constexpr int PLANE = TILE * LDA;              // one operand word plane in LDS
  static constexpr int BUF = 2 * W * PLANE;             // both operands, all words
  static constexpr int OPER_BYTES = 2 * BUF * 2;        // 2 buffers, 2 B per element
  static constexpr int SLD = TILE + 1;                  // FP32 staging row stride
  static constexpr int STG_BYTES = TILE * SLD * 4;
  static constexpr int LDS_BYTES = OPER_BYTES > STG_BYTES ? OPER_BYTES : STG_BYTES;
  // Word products (a, b) kept: weight 2^-8(a+b) >= 2^-8(W-1).
  static constexpr int NPROD = W == 1 ? 1 : (W == 2 ? 3 : 6);
};

__device__ __forceinline__ constexpr int prod_a(int W, int p) {
  return W == 1 ? 0 : (W == 2 ? (p == 2 ? 1 : 0) : (p < 3 ? (p == 2 ? 1 : 0) : (p == 3 ? 0 : (p == 4 ? 1 : 2))));
}
__device__ __forceinline__ constexpr int prod_b(int W, int p) {
  return W == 1 ? 0 : (W == 2 ? (p == 1 ? 1 : 0) : (p < 3 ? (p == 1 ? 1 : 0) : (p == 3 ? 2 : (p == 4 ? 1 : 0))));
}

template <int W, int MODE>
__global__ __launch_bounds__(256) void k_sym_gemm_w(const uint16_t* __restrict__ A,
                                                    const uint16_t* __restrict__ B,
                                                    const uint16_t* __restrict__ Xold,
                                                    uint16_t* __restrict__ out, int ld, int64_t ps,
                                                    int d, int dp, const int2* __restrict__ tiles,
                                                    double* __restrict__ partials) {
  typedef WCfg<W> C;
  __shared__ __attribute__((aligned(16))) unsigned char lds_raw[C::LDS_BYTES];
  __shared__ double red[4];
  uint16_t* lds = reinterpret_cast<uint16_t*>(lds_raw);

  const int2 tl = tiles[blockIdx.x];
  const int i0 = tl.x * TILE, j0 = tl.y * TILE;
  const bool diag = (tl.x == tl.y);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;

  // Loader: thread -> row (tid >> 1), 16 consecutive k at (tid & 1) * 16:
  // two 16 B vectors per word plane per operand.
  const int lrow = tid >> 1, lk = (tid & 1) * 16;
  const int64_t goffA = (int64_t)(i0 + lrow) * ld + lk;
  const int64_t goffB = (int64_t)(j0 + lrow) * ld + lk;
  u32x4_t ra[W][2], rb[W][2];

  f32x16_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  const int nk = dp / C::BK;
  auto gload = [&](int kt) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const u32x4_t* pa = reinterpret_cast<const u32x4_t*>(A + w * ps + goffA + kt * C::BK);
      const u32x4_t* pb = reinterpret_cast<const u32x4_t*>(B + w * ps + goffB + kt * C::BK);
      ra[w][0] = pa[0];
      ra[w][1] = pa[1];
      rb[w][0] = pb[0];
      rb[w][1] = pb[1];
    }
  };
  auto sstore = [&](int buf) {
    uint16_t* base = lds + buf * C::BUF;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      u32x4_t* da = reinterpret_cast<u32x4_t*>(base + w * C::PLANE + lrow * C::LDA + lk);
      u32x4_t* db = reinterpret_cast<u32x4_t*>(base + (W + w) * C::PLANE + lrow * C::LDA + lk);
      da[0] = ra[w][0];
      da[1] = ra[w][1];
      db[0] = rb[w][0];
      db[1] = rb[w][1];
    }
  };

  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload(kt + 1);
    const uint16_t* base = lds + cur * C::BUF;
#pragma unroll
    for (int kk = 0; kk < C::BK / 16; ++kk) {
      bf16x8_t af[W][2], bfr[W][2];
      const int kof = kk * 16 + (lane >> 5) * 8;
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          af[w][a] = *reinterpret_cast<const bf16x8_t*>(
              base + w * C::PLANE + (wr * 64 + a * 32 + (lane & 31)) * C::LDA + kof);
          bfr[w][a] = *reinterpret_cast<const bf16x8_t*>(
              base + (W + w) * C::PLANE + (wc * 64 + a * 32 + (lane & 31)) * C::LDA + kof);
        }
      // Smaller word products first.
#pragma unroll
      for (int p = C::NPROD - 1; p >= 0; --p)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[prod_a(W, p)][a],
                                                               bfr[prod_b(W, p)][b], acc[a][b],
                                                               0, 0, 0);
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }

  // ---- epilogue: stage the FP32 tile.  32x32 block layout: lane holds
  // column lane&31, rows 8*(r>>2) + 4*(lane>>5) + (r&3), r = 0..15. ----
  float* stg = reinterpret_cast<float*>(lds_raw);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = wc * 64 + b * 32 + (lane & 31);
        stg[row * C::SLD + col] = acc[a][b][r];
      }
  __syncthreads();

  // Direct pass: 8 consecutive entries (one 16 B vector per word plane) per
  // thread; 16 threads per tile row, 16 rows per iteration.
  constexpr int VE = 8, LPR = TILE / VE, RPI = 256 / LPR, NIT = TILE / RPI;
  const int cofs = (tid % LPR) * VE;
  double part = 0.0;
  float vals[NIT][VE];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int r = it * RPI + tid / LPR;
    const int gi = i0 + r;
    float xo[VE];
    if (MODE == GEMM_UPDATE) {
#pragma unroll
      for (int e = 0; e < VE; ++e) xo[e] = 0.f;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        alignas(16) uint16_t xw[VE];
        *reinterpret_cast<u32x4_t*>(xw) =
            *reinterpret_cast<const u32x4_t*>(Xold + w * ps + (int64_t)gi * ld + j0 + cofs);
#pragma unroll
        for (int e = 0; e < VE; ++e) xo[e] += bf16_to_f32(xw[e]);
      }
    }
    alignas(16) uint16_t ow[W][VE];
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      const int c = cofs + e;
      const int rr = (diag && r > c) ? c : r, cc = (diag && r > c) ? r : c;
      const float v = stg[rr * C::SLD + cc];
      const int gj = j0 + c;
      float n;
      if (MODE == GEMM_RESIDUAL) {
        n = ((gi == gj && gi < d) ? 1.f : 0.f) - v;
        part += (diag ? 1.0 : 2.0) * (double)n * (double)n;
      } else {
        n = xo[e] + 0.5f * v;
        if (gi == gj) part += (double)n;
      }
      vals[it][e] = n;
      uint16_t wv[W];
      split_words<W>(n, wv);
#pragma unroll
      for (int w = 0; w < W; ++w) ow[w][e] = wv[w];
    }
#pragma unroll
    for (int w = 0; w < W; ++w)
      *reinterpret_cast<u32x4_t*>(out + w * ps + (int64_t)gi * ld + j0 + cofs) =
          *reinterpret_cast<const u32x4_t*>(ow[w]);
  }
  __syncthreads();
  if (!diag) {
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int r = it * RPI + tid / LPR;
#pragma unroll
      for (int e = 0; e < VE; ++e) stg[r * C::SLD + cofs + e] = vals[it][e];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int c = it * RPI + tid / LPR;  // output row j0 + c
      alignas(16) uint16_t ow[W][VE];
#pragma unroll
      for (int e = 0; e < VE; ++e) {
        uint16_t wv[W];
        split_words<W>(stg[(cofs + e) * C::SLD + c], wv);
#pragma unroll
        for (int w = 0; w < W; ++w) ow[w][e] = wv[w];
      }
#pragma unroll
      for (int w = 0; w < W; ++w)
        *reinterpret_cast<u32x4_t*>(out + w * ps + (int64_t)(j0 + c) * ld + i0 + cofs) =
            *reinterpret_cast<const u32x4_t*>(ow[w]);
    }
  }
  const double tot = block_sum_256(part, red);
  if (tid == 0) partials[blockIdx.x] = tot;
}

template <int W>
static hipError_t launch_w(int mode, const uint16_t* A, const uint16_t* B, const uint16_t* Xold,
                           uint16_t* out, int ld, int64_t ps, int d, int dp, const int2* tiles,
                           int ntiles, double* partials, hipStream_t st) {
  if (mode == GEMM_RESIDUAL)
    hipLaunchKernelGGL((k_sym_gemm_w<W, GEMM_RESIDUAL>), dim3(ntiles), dim3(256), 0, st, A, B,
                       Xold, out, ld, ps, d, dp, tiles, partials);
  else
    hipLaunchKernelGGL((k_sym_gemm_w<W, GEMM_UPDATE>), dim3(ntiles), dim3(256), 0, st, A, B, Xold,
                       out, ld, ps, d, dp, tiles, partials);
  return hipGetLastError();
}

hipError_t launch_sym_gemm_words(int words, int mode, const uint16_t* A, const uint16_t* B,
                                 const uint16_t* Xold, uint16_t* out, int ld, int64_t ps, int d,
                                 int dp, const int2* tiles, int ntiles, double* partials,
                                 hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  switch (words) {
    case 1: return launch_w<1>(mode, A, B, Xold, out, ld, ps, d, dp, tiles, ntiles, partials, st);
    case 2: return launch_w<2>(mode, A, B, Xold, out, ld, ps, d, dp, tiles, ntiles, partials, st);
    case 3: return launch_w<3>(mode, A, B, Xold, out, ld, ps, d, dp, tiles, ntiles, partials, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace refl
