// Symmetric products of the Newton-Schulz step (section 3.3, eq. NS) on
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
// Work-group: 256 threads = 4 waves in a 2 x 2 arrangement; output tile
// TS x TS (TS = 128 or 192), each wave a (TS/2)^2 quadrant of 32x32x16 MFMA
// blocks.  Larger wave quadrants cut the LDS fragment reads per MFMA
// (192: 6 fragment reads of 1 KB feed 27 MFMAs per word pair and K-slice of
// 16, against 4 for 12 at 128), and 192 x 192 tiles cover the upper triangle
// of a 4096 x 4096 matrix with 253 tiles: one work-group per compute unit of
// a 256-CU device, with no split of K and no fix-up pass.
//
// K advances 32 at a time through two LDS buffers; global loads run two
// K-steps ahead in two register sets (one K-step for the 192 tiles, whose
// accumulators take the registers a second set would need).  LDS rows are 32 BF16 + 16 B of pad
// (80 B): the 16-byte fragment reads of 16 consecutive rows then fall in
// distinct bank groups whether the LDS serves 8 or 16 lanes per cycle.
#include <cstdlib>

#include <type_traits>

#include "common.h"
#include "dbg.h"
#include "launch.h"

namespace refl {

REFL_DBG_UNIT(gemm_w)

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

template <int W, int TS>
struct WCfg {
  static constexpr int BK = 32;
  static constexpr int LDA = BK + 8;                    // BF16 elements per LDS row (80 B)
  static constexpr int PLANE = TS * LDA;                // one operand word plane in LDS
  static constexpr int BUF = 2 * W * PLANE;             // both operands, all words
  static constexpr int OPER_BYTES = 2 * BUF * 2;        // 2 buffers, 2 B per element
  static constexpr int SLD = TS + 1;                    // FP32 staging row stride
  static constexpr int STG_BYTES = TS * SLD * 4;
  static constexpr int LDS_BYTES = OPER_BYTES > STG_BYTES ? OPER_BYTES : STG_BYTES;
  static constexpr int NB = TS / 64;                    // 32x32 blocks per wave dimension
  static constexpr int CHUNKS = TS * (BK / 8);          // 16-byte chunks per operand word plane
  static constexpr int CPT = CHUNKS / 256;              // chunks per thread
  // Word products (a, b) kept: weight 2^-8(a+b) >= 2^-8(W-1).
  static constexpr int NPROD = W == 1 ? 1 : (W == 2 ? 3 : 6);
  // Register sets for the global-load prefetch: two (loads run two K-steps
  // ahead) unless the accumulators of a 192 tile leave no room.
  static constexpr int DEPTH = (TS == 192 && W >= 2) ? 1 : 2;
  static_assert(CHUNKS % 256 == 0, "tile rows must split evenly over the work-group");
};

__device__ __forceinline__ constexpr int prod_a(int W, int p) {
  return W == 1 ? 0 : (W == 2 ? (p == 2 ? 1 : 0) : (p < 3 ? (p == 2 ? 1 : 0) : (p == 3 ? 0 : (p == 4 ? 1 : 2))));
}
__device__ __forceinline__ constexpr int prod_b(int W, int p) {
  return W == 1 ? 0 : (W == 2 ? (p == 1 ? 1 : 0) : (p < 3 ? (p == 1 ? 1 : 0) : (p == 3 ? 2 : (p == 4 ? 1 : 0))));
}

template <int W, int MODE, int TS>
__global__ __launch_bounds__(256) void k_sym_gemm_w(const uint16_t* __restrict__ A,
                                                    const uint16_t* __restrict__ B,
                                                    const uint16_t* __restrict__ Xold,
                                                    uint16_t* __restrict__ out, int ld, int64_t ps,
                                                    int d, int dk, const int2* __restrict__ tiles,
                                                    double* __restrict__ partials,
                                                    const int* __restrict__ live) {
  if (live && *live == 0) return;
  typedef WCfg<W, TS> C;
  constexpr int NB = C::NB;
  __shared__ __attribute__((aligned(16))) unsigned char lds_raw[C::LDS_BYTES];
  __shared__ double red[4];
  uint16_t* lds = reinterpret_cast<uint16_t*>(lds_raw);

  const int2 tl = tiles[blockIdx.x];
  const int i0 = tl.x * TS, j0 = tl.y * TS;
  const bool diag = (tl.x == tl.y);
  REFL_GUARD(tl.x >= 0 && tl.x <= tl.y && j0 + TS <= ld && d <= dk && dk <= ld && dk % 32 == 0 &&
                 ps >= (int64_t)ld * ld,
             DBG_GEMM_W_TILE);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;

  // Loader: chunk q = tid + 256 i -> row q / 4, 16-byte chunk q % 4 of the
  // K-slice (consecutive threads read consecutive 16 B of a row).
  int64_t goffA[C::CPT], goffB[C::CPT];
  int soff[C::CPT];
#pragma unroll
  for (int i = 0; i < C::CPT; ++i) {
    const int q = tid + 256 * i, row = q >> 2, ch = q & 3;
    goffA[i] = (int64_t)(i0 + row) * ld + ch * 8;
    goffB[i] = (int64_t)(j0 + row) * ld + ch * 8;
    soff[i] = row * C::LDA + ch * 8;
  }
  u32x4_t ra[W][C::DEPTH][C::CPT], rb[W][C::DEPTH][C::CPT];

  f32x16_t acc[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  const int nk = dk / C::BK;
  auto gload = [&](int kt, int set) {
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int i = 0; i < C::CPT; ++i) {
        ra[w][set][i] = *reinterpret_cast<const u32x4_t*>(A + w * ps + goffA[i] + kt * C::BK);
        rb[w][set][i] = *reinterpret_cast<const u32x4_t*>(B + w * ps + goffB[i] + kt * C::BK);
      }
  };
  auto sstore = [&](int buf, int set) {
    uint16_t* base = lds + buf * C::BUF;
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int i = 0; i < C::CPT; ++i) {
        *reinterpret_cast<u32x4_t*>(base + w * C::PLANE + soff[i]) = ra[w][set][i];
        *reinterpret_cast<u32x4_t*>(base + (W + w) * C::PLANE + soff[i]) = rb[w][set][i];
      }
  };
  auto compute = [&](int buf) {
    const uint16_t* base = lds + buf * C::BUF;
#pragma unroll
    for (int kk = 0; kk < C::BK / 16; ++kk) {
      bf16x8_t af[W][NB], bfr[W][NB];
      const int kof = kk * 16 + (lane >> 5) * 8;
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int a = 0; a < NB; ++a) {
          af[w][a] = *reinterpret_cast<const bf16x8_t*>(
              base + w * C::PLANE + (wr * (TS / 2) + a * 32 + (lane & 31)) * C::LDA + kof);
          bfr[w][a] = *reinterpret_cast<const bf16x8_t*>(
              base + (W + w) * C::PLANE + (wc * (TS / 2) + a * 32 + (lane & 31)) * C::LDA + kof);
        }
      // Smaller word products first.
#pragma unroll
      for (int p = C::NPROD - 1; p >= 0; --p)
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[prod_a(W, p)][a],
                                                               bfr[prod_b(W, p)][b], acc[a][b],
                                                               0, 0, 0);
    }
  };

  if constexpr (C::DEPTH == 2) {
    // LDS buffer kt & 1 holds K-slice kt; register set (kt + 1) & 1 holds or
    // receives slice kt + 1 while slice kt + 2 is fetched into the other set.
    gload(0, 0);
    if (nk > 1) gload(1, 1 % C::DEPTH);
    sstore(0, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; kt += 2) {
      // even step: register set 1 holds slice kt + 1, set 0 is free
      if (kt + 2 < nk) gload(kt + 2, 0);
      compute(0);
      if (kt + 1 < nk) sstore(1, 1 % C::DEPTH);
      __syncthreads();
      if (kt + 1 >= nk) break;
      // odd step: set 0 holds slice kt + 2, set 1 is free
      if (kt + 3 < nk) gload(kt + 3, 1 % C::DEPTH);
      compute(1);
      if (kt + 2 < nk) sstore(0, 0);
      __syncthreads();
    }
  } else {
    // One register set: slice kt + 1 is fetched while slice kt is multiplied.
    gload(0, 0);
    sstore(0, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      if (kt + 1 < nk) gload(kt + 1, 0);
      compute(kt & 1);
      if (kt + 1 < nk) sstore((kt + 1) & 1, 0);
      __syncthreads();
    }
  }

  // ---- epilogue: stage the FP32 tile.  32x32 block layout: lane holds
  // column lane&31, rows 8*(r>>2) + 4*(lane>>5) + (r&3), r = 0..15. ----
  float* stg = reinterpret_cast<float*>(lds_raw);
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * (TS / 2) + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = wc * (TS / 2) + b * 32 + (lane & 31);
        stg[row * C::SLD + col] = acc[a][b][r];
      }
  __syncthreads();

  // Direct pass: 8 consecutive entries (one 16 B vector per word plane) per
  // thread and iteration, row-contiguous.  In a diagonal tile entry (r, c)
  // takes the value computed at (min, max), so the stored tile is exactly
  // symmetric; off-diagonal tiles write their final values back in place for
  // the transposed pass.
  constexpr int VE = 8, CPR = TS / VE;
  double part = 0.0;
  for (int e = tid; e < TS * CPR; e += 256) {
    const int r = e / CPR, cofs = (e % CPR) * VE;
    const int gi = i0 + r;
    float xo[VE];
    if (MODE == GEMM_UPDATE) {
#pragma unroll
      for (int q = 0; q < VE; ++q) xo[q] = 0.f;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        alignas(16) uint16_t xw[VE];
        *reinterpret_cast<u32x4_t*>(xw) =
            *reinterpret_cast<const u32x4_t*>(Xold + w * ps + (int64_t)gi * ld + j0 + cofs);
#pragma unroll
        for (int q = 0; q < VE; ++q) xo[q] += bf16_to_f32(xw[q]);
      }
    }
    alignas(16) uint16_t ow[W][VE];
    float nv[VE];
#pragma unroll
    for (int q = 0; q < VE; ++q) {
      const int c = cofs + q;
      const int rr = (diag && r > c) ? c : r, cc = (diag && r > c) ? r : c;
      const float v = stg[rr * C::SLD + cc];
      const int gj = j0 + c;
      float n;
      if (MODE == GEMM_RESIDUAL) {
        n = ((gi == gj && gi < d) ? 1.f : 0.f) - v;
        part += (diag ? 1.0 : 2.0) * (double)n * (double)n;
      } else {
        n = xo[q] + 0.5f * v;
        if (gi == gj) part += (double)n;
      }
      nv[q] = n;
      uint16_t wv[W];
      split_words<W>(n, wv);
#pragma unroll
      for (int w = 0; w < W; ++w) ow[w][q] = wv[w];
    }
    if (!diag) {
#pragma unroll
      for (int q = 0; q < VE; ++q) stg[r * C::SLD + cofs + q] = nv[q];
    }
#pragma unroll
    for (int w = 0; w < W; ++w)
      *reinterpret_cast<u32x4_t*>(out + w * ps + (int64_t)gi * ld + j0 + cofs) =
          *reinterpret_cast<const u32x4_t*>(ow[w]);
  }
  if (!diag) {
    __syncthreads();
    // Transposed pass: output row j0 + c, columns i0 + rofs .. + 7.
    for (int e = tid; e < TS * CPR; e += 256) {
      const int c = e / CPR, rofs = (e % CPR) * VE;
      alignas(16) uint16_t ow[W][VE];
#pragma unroll
      for (int q = 0; q < VE; ++q) {
        uint16_t wv[W];
        split_words<W>(stg[(rofs + q) * C::SLD + c], wv);
#pragma unroll
        for (int w = 0; w < W; ++w) ow[w][q] = wv[w];
      }
#pragma unroll
      for (int w = 0; w < W; ++w)
        *reinterpret_cast<u32x4_t*>(out + w * ps + (int64_t)(j0 + c) * ld + i0 + rofs) =
            *reinterpret_cast<const u32x4_t*>(ow[w]);
    }
  }
  const double tot = block_sum_256(part, red);
  if (tid == 0) partials[blockIdx.x] = tot;
}

// ---------------------------------------------------------------------
// Direct-to-LDS variant: K-slices reach LDS by global_load_lds_dwordx4 (each
// lane's 16 B land at the wave's LDS base + 16 * lane, so a wave writes 1 KB
// = 16 rows of 64 B), through a ring of three stages: the loads of slice
// kt + 2 are issued while slice kt is multiplied, with no staging registers.
// Rows are 64 B without padding; the 16-byte chunk c of row r is stored at
// position c ^ swz(r), swz(r) = ((r >> 1) ^ (r >> 2)) & 3, which keeps the
// fragment reads of 16 consecutive rows on distinct bank groups whether the
// LDS serves 8 or 16 lanes per cycle.
__device__ __forceinline__ int swz(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

template <int W, int TS>
struct DCfg {
  static constexpr int BK = 32;
  static constexpr int ROWB = 64;                       // bytes per LDS row (BK BF16)
  static constexpr int NS = 3;                          // ring stages
  static constexpr int PLANE_B = TS * ROWB;
  static constexpr int STAGE_B = 2 * W * PLANE_B;
  static constexpr int NINST = 2 * W * (TS / 16);       // 1 KB load instructions per stage
  static constexpr int NLW = NINST / 4;                 // per wave
  static constexpr int NB = TS / 64;
  static constexpr int NPROD = W == 1 ? 1 : (W == 2 ? 3 : 6);
  static_assert(NINST % 4 == 0, "load instructions must split over 4 waves");
  static_assert(NS * STAGE_B <= 160 * 1024, "ring exceeds LDS");
};

// Work-group barrier that orders LDS only.  __syncthreads() would also wait
// for every outstanding vector-memory operation, which includes the
// direct-to-LDS loads of the slices still in flight; here each wave first
// waits (vmcnt) for the slice about to be read, then the barrier makes all
// waves' copies of it visible.  The memory clobber keeps the compiler from
// moving LDS accesses across the barrier.
#define REFL_LDS_BARRIER() asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory")

// s_waitcnt with vmcnt = n (0..63) and no wait on the other counters.
#define REFL_WAIT_VMCNT(n) \
  __builtin_amdgcn_s_waitcnt(((n) & 15) | (((n) >> 4) << 14) | (7 << 4) | (15 << 8))

// Scheduling hints for the two-register-set schedule: N LDS fragment reads
// and NG global-to-LDS loads spread evenly through NMF MFMAs (groups of
// MFMA, then one DS read, then at most one global load).
template <int I, int N, int NMF, int NG>
__device__ __forceinline__ void interleave_hints() {
  if constexpr (I < N) {
    constexpr int m = (NMF * (I + 1)) / N - (NMF * I) / N;
    constexpr int g = (NG * (I + 1)) / N - (NG * I) / N;
    if constexpr (m > 0) __builtin_amdgcn_sched_group_barrier(0x008, m, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    if constexpr (g > 0) __builtin_amdgcn_sched_group_barrier(0x020, g, 0);
    interleave_hints<I + 1, N, NMF, NG>();
  }
}

// One wave per SIMD (the ring fills the LDS); telling the compiler so lets it
// keep a whole K-slice of fragments in registers instead of re-reading LDS.
template <int W, int MODE, int TS, int PIPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_sym_gemm_wd(const uint16_t* __restrict__ A,
                                                     const uint16_t* __restrict__ B,
                                                     const uint16_t* __restrict__ Xold,
                                                     uint16_t* __restrict__ out, int ld,
                                                     int64_t ps, int d, int dk,
                                                     const int2* __restrict__ tiles,
                                                     double* __restrict__ partials,
                                                     const int* __restrict__ live) {
  // A stopped iteration (device-side stopping rule): nothing to do.
  if (live && *live == 0) return;
  typedef DCfg<W, TS> C;
  constexpr int NB = C::NB;
  // Three separate arrays: the compiler's per-variable alias scopes then let
  // LDS reads of one stage proceed while direct loads into another are in
  // flight (one array would make it wait for every outstanding load).
  __shared__ __attribute__((aligned(1024))) unsigned char ring0[C::STAGE_B];
  __shared__ __attribute__((aligned(1024))) unsigned char ring1[C::STAGE_B];
  __shared__ __attribute__((aligned(1024))) unsigned char ring2[C::STAGE_B];
  __shared__ double red[4];

  const int2 tl = tiles[blockIdx.x];
  const int i0 = tl.x * TS, j0 = tl.y * TS;
  const bool diag = (tl.x == tl.y);
  REFL_GUARD(tl.x >= 0 && tl.x <= tl.y && j0 + TS <= ld && d <= dk && dk <= ld && dk % 32 == 0 &&
                 ps >= (int64_t)ld * ld,
             DBG_GEMM_WD_TILE);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;

  // Load descriptors.  Instruction m (of this wave's NLW) covers 16 rows of
  // one word plane of one operand; lane l loads row 16 rb + l/4, logical
  // chunk (l & 3) ^ swz(l/4) (the swizzle only involves row bits 0..3, so it
  // is the same for every 16-row block).  The per-instruction part of the
  // address is wave-uniform; the per-lane part is one offset.
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  const int lane_goff = (lane >> 2) * ld + 8 * ((lane & 3) ^ swz(lane >> 2));
  auto issue = [&](int kt, unsigned char* stage) {
#pragma unroll
    for (int j = 0; j < C::NLW; ++j) {
      const int m = wave_u * C::NLW + j;
      const int op = m / (W * (TS / 16));
      const int rem = m % (W * (TS / 16));
      const int word = rem / (TS / 16), rb = rem % (TS / 16);
      const uint16_t* gbase = (op == 0 ? A : B) + word * ps +
                              (int64_t)((op == 0 ? i0 : j0) + rb * 16) * ld + kt * C::BK;
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)(gbase + lane_goff),
          (__attribute__((address_space(3))) void*)(stage + ((op * W + word) * TS + rb * 16) * C::ROWB),
          16, 0, 0);
    }
  };

  f32x16_t acc[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  // Fragments of one K-slice in two halves: H[0] for k 0..15, H[1] for
  // k 16..31 of the slice, all word planes.
  constexpr int KH = C::BK / 16;
  static_assert(KH == 2, "two 16-wide halves per K-slice");
  bf16x8_t fa[KH][W][NB], fb[KH][W][NB];
  // Fragment reads: lane l reads row (block row) + l % 32, logical chunk
  // 2 kk + l / 32; block rows are multiples of 32, so the swizzle is swz(l % 32)
  // and every read is one lane offset plus an immediate.
  const int frag_lane[KH] = {
      (lane & 31) * C::ROWB + 16 * ((0 + (lane >> 5)) ^ swz(lane & 31)),
      (lane & 31) * C::ROWB + 16 * ((2 + (lane >> 5)) ^ swz(lane & 31))};
  auto load_half = [&](const unsigned char* sb, int kk) {
    const unsigned char* p = sb + frag_lane[kk];
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        fa[kk][w][a] = *reinterpret_cast<const bf16x8_t*>(
            p + (w * TS + wr * (TS / 2) + a * 32) * C::ROWB);
        fb[kk][w][a] = *reinterpret_cast<const bf16x8_t*>(
            p + ((W + w) * TS + wc * (TS / 2) + a * 32) * C::ROWB);
      }
  };
  auto mfma_half = [&](int kk) {
#pragma unroll
    for (int p = C::NPROD - 1; p >= 0; --p)
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              fa[kk][prod_a(W, p)][a], fb[kk][prod_b(W, p)][b], acc[a][b], 0, 0, 0);
  };

  // Pipeline.  Slice j lives in stage j % 3.  Step kt: issue the loads of
  // slice kt + 2; MFMAs of the first half of slice kt; wait for slice kt + 1
  // (this wave's loads, then the barrier for everyone's); read its first
  // half while the second half of slice kt is multiplied; then read its
  // second half.  The stage written by the loads of slice kt + 2 held slice
  // kt - 1, whose last reads every wave completed before the barrier of
  // step kt - 1.  The steady-state loop is unconditional (the compiler then
  // keeps track of which stage each in-flight load writes); the last two
  // steps are peeled.
  const int nk = dk / C::BK;
  if constexpr (PIPE == 1) {
    auto step = [&](int kt, unsigned char* dma, const unsigned char* nxt) {
      issue(kt + 2, dma);
      mfma_half(0);
      REFL_WAIT_VMCNT(C::NLW);
      REFL_LDS_BARRIER();
      load_half(nxt, 0);
      mfma_half(1);
      load_half(nxt, 1);
    };
    // Slice 1 is fetched even when nk == 1: the matrices are at least 128
    // columns wide, so the read stays in bounds, and an unconditional
    // prologue keeps the in-flight-load bookkeeping exact.
    issue(0, ring0);
    issue(1, ring1);
    REFL_WAIT_VMCNT(C::NLW);
    REFL_LDS_BARRIER();
    load_half(ring0, 0);
    load_half(ring0, 1);
    int kt = 0;
    for (; kt + 4 < nk; kt += 3) {
      step(kt, ring2, ring1);
      step(kt + 1, ring0, ring2);
      step(kt + 2, ring1, ring0);
    }
    // Tail: slices kt .. nk - 1, stages continuing from ring0 (kt % 3 == 0).
    for (int t = 0; kt + t < nk; ++t) {
      const int j = kt + t;
      unsigned char* dma = (t % 3 == 0) ? ring2 : ((t % 3 == 1) ? ring0 : ring1);
      const unsigned char* nxt = (t % 3 == 0) ? ring1 : ((t % 3 == 1) ? ring2 : ring0);
      if (j + 2 < nk) issue(j + 2, dma);
      mfma_half(0);
      if (j + 1 < nk) {
        if (j + 2 < nk) {
          REFL_WAIT_VMCNT(C::NLW);
        } else {
          REFL_WAIT_VMCNT(0);
        }
        REFL_LDS_BARRIER();
        load_half(nxt, 0);
        mfma_half(1);
        load_half(nxt, 1);
      } else {
        mfma_half(1);
      }
    }
  } else if constexpr (PIPE == 2) {
    // Two fragment register sets.  Step kt: wait for slice kt + 1 (own
    // loads, then the barrier for everyone's); the stage of slice kt, whose
    // fragments every wave already holds in registers, is then free and
    // takes the loads of slice kt + 3; then the fragment reads of slice
    // kt + 1 into the other set run interleaved with the MFMAs of slice kt.
    // The LDS reads of the next slice overlap the matrix work of this one,
    // and two slices beyond the one being read stay in flight.  Slice j sits
    // in stage j % 3 and in register set j % 2: six steps form one static
    // pattern.
    struct Frag {
      bf16x8_t a[KH][W][NB], b[KH][W][NB];
    };
    Frag F0, F1;
    auto fset = [&](auto ci) -> Frag& {
      if constexpr (decltype(ci)::value == 0) return F0;
      else return F1;
    };
    auto read_frag = [&](Frag& f, const unsigned char* sb) {
#pragma unroll
      for (int kk = 0; kk < KH; ++kk) {
        const unsigned char* p = sb + frag_lane[kk];
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int a = 0; a < NB; ++a) {
            f.a[kk][w][a] = *reinterpret_cast<const bf16x8_t*>(
                p + (w * TS + wr * (TS / 2) + a * 32) * C::ROWB);
            f.b[kk][w][a] = *reinterpret_cast<const bf16x8_t*>(
                p + ((W + w) * TS + wc * (TS / 2) + a * 32) * C::ROWB);
          }
      }
    };
    auto mfma_frag = [&](const Frag& f) {
#pragma unroll
      for (int kk = 0; kk < KH; ++kk)
#pragma unroll
        for (int p = C::NPROD - 1; p >= 0; --p)
#pragma unroll
          for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  f.a[kk][prod_a(W, p)][a], f.b[kk][prod_b(W, p)][b], acc[a][b], 0, 0, 0);
    };
    auto ring_at = [&](auto si) -> unsigned char* {
      constexpr int S = decltype(si)::value % 3;
      if constexpr (S == 0) return ring0;
      else if constexpr (S == 1) return ring1;
      else return ring2;
    };
    constexpr int NDSR = 2 * KH * W * NB;
    constexpr int NMF = KH * C::NPROD * NB * NB;
    auto stepP = [&](auto ci, auto si, int kt, bool dma, bool more) {
      constexpr int CI = decltype(ci)::value;
      constexpr int SI = decltype(si)::value;
      if (more) {
        // Slices kt + 1 and kt + 2 were issued; kt + 2 may stay in flight.
        if (kt + 2 < nk) {
          REFL_WAIT_VMCNT(C::NLW);
        } else {
          REFL_WAIT_VMCNT(0);
        }
        REFL_LDS_BARRIER();
        __builtin_amdgcn_sched_barrier(0);
        if (dma) issue(kt + 3, ring_at(std::integral_constant<int, SI>()));
        read_frag(fset(std::integral_constant<int, CI ^ 1>()), ring_at(std::integral_constant<int, SI + 1>()));
        mfma_frag(fset(std::integral_constant<int, CI>()));
        interleave_hints<0, NDSR, NMF, C::NLW>();
        __builtin_amdgcn_sched_barrier(0);
      } else {
        mfma_frag(fset(std::integral_constant<int, CI>()));
      }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    // Prologue: slices 0, 1, 2 (slice 1 and 2 may be beyond K: the matrices
    // are at least one tile wide, so the reads stay in bounds).
    issue(0, ring0);
    issue(1, ring1);
    issue(2, ring2);
    REFL_WAIT_VMCNT(2 * C::NLW);
    REFL_LDS_BARRIER();
    read_frag(F0, ring0);
    int kt = 0;
    for (; kt + 9 <= nk; kt += 6) {
      stepP(I0(), I0(), kt, true, true);
      stepP(I1(), I1(), kt + 1, true, true);
      stepP(I0(), I2(), kt + 2, true, true);
      stepP(I1(), I0(), kt + 3, true, true);
      stepP(I0(), I1(), kt + 4, true, true);
      stepP(I1(), I2(), kt + 5, true, true);
    }
    // Tail (at most 8 slices, entered at phase 0 with slice kt in F0 and
    // slices kt + 1, kt + 2 in flight): one register set, reads after the
    // MFMAs.
    for (; kt < nk; ++kt) {
      auto stage = [&](int j) -> unsigned char* {
        const int m = j % 3;
        return m == 0 ? ring0 : (m == 1 ? ring1 : ring2);
      };
      mfma_frag(F0);
      if (kt + 1 < nk) {
        if (kt + 2 < nk) {
          REFL_WAIT_VMCNT(C::NLW);
        } else {
          REFL_WAIT_VMCNT(0);
        }
        REFL_LDS_BARRIER();
        if (kt + 3 < nk) issue(kt + 3, stage(kt));
        read_frag(F0, stage(kt + 1));
      }
    }
  } else {
    // Barrier at the start of each slice, then all of its fragment reads,
    // the loads of slice kt + 2, and the MFMAs.
    auto step = [&](int kt, const unsigned char* cur, unsigned char* next2) {
      REFL_WAIT_VMCNT(C::NLW);
      REFL_LDS_BARRIER();
      load_half(cur, 0);
      load_half(cur, 1);
      __builtin_amdgcn_sched_barrier(0);
      issue(kt + 2, next2);
      mfma_half(0);
      mfma_half(1);
    };
    issue(0, ring0);
    issue(1, ring1);
    int kt = 0;
    for (; kt + 4 < nk; kt += 3) {
      step(kt, ring0, ring2);
      step(kt + 1, ring1, ring0);
      step(kt + 2, ring2, ring1);
    }
    for (int t = 0; kt + t < nk; ++t) {
      const int j = kt + t;
      const unsigned char* cur = (t % 3 == 0) ? ring0 : ((t % 3 == 1) ? ring1 : ring2);
      unsigned char* nx = (t % 3 == 0) ? ring2 : ((t % 3 == 1) ? ring0 : ring1);
      if (j + 1 < nk) {
        REFL_WAIT_VMCNT(C::NLW);
      } else {
        REFL_WAIT_VMCNT(0);
      }
      REFL_LDS_BARRIER();
      load_half(cur, 0);
      load_half(cur, 1);
      if (j + 2 < nk) issue(j + 2, nx);
      mfma_half(0);
      mfma_half(1);
    }
  }
  REFL_WAIT_VMCNT(0);
  __syncthreads();

  // ---- epilogue.  The FP32 tile is staged across the three ring arrays,
  // RPA rows per array, row-major without padding; entry (r, c) sits at
  // column c ^ ((r >> 3) & 31) of its row, so the transposed pass (eight
  // consecutive rows of one column per lane, 24 lanes per column) reads
  // distinct banks. ----
  constexpr int RPA = C::STAGE_B / (TS * 4);
  static_assert(3 * RPA >= TS, "staging must fit in the ring");
  auto stg = [&](int r, int c) -> float& {
    unsigned char* base = r < RPA ? ring0 : (r < 2 * RPA ? ring1 : ring2);
    const int rr = r % RPA;
    return reinterpret_cast<float*>(base)[rr * TS + (c ^ ((r >> 3) & 31))];
  };
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * (TS / 2) + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = wc * (TS / 2) + b * 32 + (lane & 31);
        stg(row, col) = acc[a][b][r];
      }
  __syncthreads();
  constexpr int VE = 8, CPR = TS / VE;
  double part = 0.0;
  for (int e = tid; e < TS * CPR; e += 256) {
    const int r = e / CPR, cofs = (e % CPR) * VE;
    const int gi = i0 + r;
    float xo[VE];
    if (MODE == GEMM_UPDATE) {
#pragma unroll
      for (int q = 0; q < VE; ++q) xo[q] = 0.f;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        alignas(16) uint16_t xw[VE];
        *reinterpret_cast<u32x4_t*>(xw) =
            *reinterpret_cast<const u32x4_t*>(Xold + w * ps + (int64_t)gi * ld + j0 + cofs);
#pragma unroll
        for (int q = 0; q < VE; ++q) xo[q] += bf16_to_f32(xw[q]);
      }
    }
    alignas(16) uint16_t ow[W][VE];
    float nv[VE];
#pragma unroll
    for (int q = 0; q < VE; ++q) {
      const int c = cofs + q;
      const int rr = (diag && r > c) ? c : r, cc = (diag && r > c) ? r : c;
      const float v = stg(rr, cc);
      const int gj = j0 + c;
      float n;
      if (MODE == GEMM_RESIDUAL) {
        n = ((gi == gj && gi < d) ? 1.f : 0.f) - v;
        part += (diag ? 1.0 : 2.0) * (double)n * (double)n;
      } else {
        n = xo[q] + 0.5f * v;
        if (gi == gj) part += (double)n;
      }
      nv[q] = n;
      uint16_t wv[W];
      split_words<W>(n, wv);
#pragma unroll
      for (int w = 0; w < W; ++w) ow[w][q] = wv[w];
    }
    if (!diag) {
#pragma unroll
      for (int q = 0; q < VE; ++q) stg(r, cofs + q) = nv[q];
    }
#pragma unroll
    for (int w = 0; w < W; ++w)
      *reinterpret_cast<u32x4_t*>(out + w * ps + (int64_t)gi * ld + j0 + cofs) =
          *reinterpret_cast<const u32x4_t*>(ow[w]);
  }
  if (!diag) {
    __syncthreads();
    for (int e = tid; e < TS * CPR; e += 256) {
      const int c = e / CPR, rofs = (e % CPR) * VE;
      alignas(16) uint16_t ow[W][VE];
#pragma unroll
      for (int q = 0; q < VE; ++q) {
        uint16_t wv[W];
        split_words<W>(stg(rofs + q, c), wv);
#pragma unroll
        for (int w = 0; w < W; ++w) ow[w][q] = wv[w];
      }
#pragma unroll
      for (int w = 0; w < W; ++w)
        *reinterpret_cast<u32x4_t*>(out + w * ps + (int64_t)(j0 + c) * ld + i0 + rofs) =
            *reinterpret_cast<const u32x4_t*>(ow[w]);
    }
  }
  const double tot = block_sum_256(part, red);
  if (tid == 0) partials[blockIdx.x] = tot;
}

static int gemm_pipe() {
  static const int v = [] {
    const char* e = std::getenv("REFL_GEMM_PIPE");
    return (e && (e[0] == '0' || e[0] == '1' || e[0] == '2')) ? e[0] - '0' : 2;
  }();
  return v;
}

static bool use_register_staging() {
  static const int v = [] {
    const char* e = std::getenv("REFL_GEMM_STAGING");
    return (e && e[0] == 'r') ? 1 : 0;
  }();
  return v != 0;
}

template <int W, int TS>
static hipError_t launch_w(int mode, const uint16_t* A, const uint16_t* B, const uint16_t* Xold,
                           uint16_t* out, int ld, int64_t ps, int d, int dk, const int2* tiles,
                           int ntiles, double* partials, hipStream_t st, const int* live) {
  if constexpr (W >= 2) {
    if (!use_register_staging()) {
      const int pipe = gemm_pipe();
#define REFL_WD(MODEV, PIPEV)                                                                \
  hipLaunchKernelGGL((k_sym_gemm_wd<W, MODEV, TS, PIPEV>), dim3(ntiles), dim3(256), 0, st, A, B, \
                     Xold, out, ld, ps, d, dk, tiles, partials, live)
      if (mode == GEMM_RESIDUAL) {
        if (pipe == 2) REFL_WD(GEMM_RESIDUAL, 2);
        else if (pipe == 1) REFL_WD(GEMM_RESIDUAL, 1);
        else REFL_WD(GEMM_RESIDUAL, 0);
      } else {
        if (pipe == 2) REFL_WD(GEMM_UPDATE, 2);
        else if (pipe == 1) REFL_WD(GEMM_UPDATE, 1);
        else REFL_WD(GEMM_UPDATE, 0);
      }
#undef REFL_WD
      return hipGetLastError();
    }
  }
  if (mode == GEMM_RESIDUAL)
    hipLaunchKernelGGL((k_sym_gemm_w<W, GEMM_RESIDUAL, TS>), dim3(ntiles), dim3(256), 0, st, A, B,
                       Xold, out, ld, ps, d, dk, tiles, partials, live);
  else
    hipLaunchKernelGGL((k_sym_gemm_w<W, GEMM_UPDATE, TS>), dim3(ntiles), dim3(256), 0, st, A, B,
                       Xold, out, ld, ps, d, dk, tiles, partials, live);
  return hipGetLastError();
}

template <int TS>
static hipError_t launch_ts_impl(int words, int mode, const uint16_t* A, const uint16_t* B,
                            const uint16_t* Xold, uint16_t* out, int ld, int64_t ps, int d, int dk,
                            const int2* tiles, int ntiles, double* partials, hipStream_t st,
                            const int* live) {
  switch (words) {
    case 1: return launch_w<1, TS>(mode, A, B, Xold, out, ld, ps, d, dk, tiles, ntiles, partials, st, live);
    case 2: return launch_w<2, TS>(mode, A, B, Xold, out, ld, ps, d, dk, tiles, ntiles, partials, st, live);
    default: return hipErrorInvalidValue;
  }
}
template <>
hipError_t launch_ts_impl<128>(int words, int mode, const uint16_t* A, const uint16_t* B,
                               const uint16_t* Xold, uint16_t* out, int ld, int64_t ps, int d,
                               int dk, const int2* tiles, int ntiles, double* partials,
                               hipStream_t st, const int* live) {
  switch (words) {
    case 1: return launch_w<1, 128>(mode, A, B, Xold, out, ld, ps, d, dk, tiles, ntiles, partials, st, live);
    case 2: return launch_w<2, 128>(mode, A, B, Xold, out, ld, ps, d, dk, tiles, ntiles, partials, st, live);
    case 3: return launch_w<3, 128>(mode, A, B, Xold, out, ld, ps, d, dk, tiles, ntiles, partials, st, live);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sym_gemm_words(int words, int tile, int mode, const uint16_t* A,
                                 const uint16_t* B, const uint16_t* Xold, uint16_t* out, int ld,
                                 int64_t ps, int d, int dk, const int2* tiles, int ntiles,
                                 double* partials, hipStream_t st, const int* live) {
  if (ntiles <= 0) return hipSuccess;
  if (tile == 128)
    return launch_ts_impl<128>(words, mode, A, B, Xold, out, ld, ps, d, dk, tiles, ntiles, partials, st,
                               live);
  // 192-row tiles need 4 * 192 * 80 B of operand LDS per word: W <= 2 only.
  if (tile == 192 && words <= 2)
    return launch_ts_impl<192>(words, mode, A, B, Xold, out, ld, ps, d, dk, tiles, ntiles, partials, st,
                               live);
  return hipErrorInvalidValue;
}

}  // namespace refl
