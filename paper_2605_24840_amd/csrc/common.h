// Device-side helpers shared by the reflector kernels (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace refl {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4_t;

// Square output tile of the symmetric products, and the padding unit of the
// workspace matrices: every workspace matrix is dp x dp with dp a multiple of
// TILE, zero outside the leading d x d block.
constexpr int TILE = 128;
constexpr int WAVE = 64;

// Slots of the small FP64 scalar array the kernels and the host share.
enum ScalarSlot {
  SC_ALPHA = 0,      // scale: X_0 = (H - sI)/alpha
  SC_NONFINITE = 1,  // > 0 if a non-finite entry of H was seen
  SC_RESID2 = 2,     // ||X^2 - I||_F^2 of the iterate entering the last GEMM-1
  SC_TRACE = 3,      // trace of the newest iterate
  SC_SCRATCH = 4,    // first free slot
  SC_SYM = 60,       // two slots: the symmetry check's maxima
  SC_COUNT = 64
};

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}

// Split x into W BF16 words, x ~= w0 + w1 (+ w2), each the RNE rounding of
// the remainder left by the words before it (the remainders are exact in FP32).
template <int W>
__device__ __forceinline__ void split_words(float x, uint16_t (&w)[W]) {
  float r = x;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    w[i] = f32_to_bf16_rne(r);
    r = r - bf16_to_f32(w[i]);
  }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
  return v;
}

// Sum over a 256-thread block in a fixed order (deterministic).
__device__ __forceinline__ double block_sum_256(double v, double* red /* >= 4 */) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
  return r;  // valid in thread 0 only
}

}  // namespace refl
