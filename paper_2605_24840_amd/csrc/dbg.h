// Launch-extent guards of the debug build (compiled with -DREFL_DEBUG).
//
// A guarded kernel checks, on entry and for its own block, that the rows,
// columns, tiles and K-slices it is about to touch lie inside the extents it
// was launched with (the order d, the leading dimension, the padded order,
// the tile edge).  Every condition is uniform over the block, so a failing
// block returns as a whole before its first memory access or barrier; no
// kernel of the library waits on another block, so an early return cannot
// stall the grid.  The failing block records the guard's site code in a
// device word of its translation unit (first failure wins); the host reads
// and clears every unit's word at the end of each entry point and returns
// REFL_ERR_BOUNDS naming the site.  Release builds compile the guards and
// the words away.
#pragma once
#include <hip/hip_runtime.h>

namespace refl {

enum DbgSite {
  DBG_NONE = 0,
  DBG_GEMM_W_TILE,      // word product: tile or K range outside the padded order
  DBG_GEMM_WD_TILE,     // word product (direct-to-LDS): the same
  DBG_GEMM_F_TILE,      // FP64/FP32 product (single, grouped, adjoint): the same
  DBG_MIRROR,           // mirror of the upper triangle: tile outside d
  DBG_ROWABS,           // row sums: rows outside d
  DBG_INIT_X0,          // X_0 = (H - sI)/alpha: rows or columns outside the padded order
  DBG_FORM_R,           // R from the iterate: rows outside d
  DBG_SYMTHIN,          // thin product: chunk or rows outside d
  DBG_THIN_FINISH,      // thin product's chunk sums: rows outside d
  DBG_CG_PASS,          // inner solve's pass: chunk outside d, more columns than instantiated
  DBG_CG_UPDATE,        // inner solve's update: row group or column outside the block
  DBG_CG_INIT,          // inner solve's first partials: the same
  DBG_LZ,               // block-Lanczos kernels: block or rows outside the basis
  DBG_CG_STEP,          // FP64 inner solve's step: chunk outside d, block wider than instantiated
  DBG_CG_APPLY,         // FP64 inner solve's apply: row group or column outside the block
  DBG_GRAM,             // Gram partials: more than 32 columns, rows outside d
  DBG_THIN_PARTIAL,     // thin product (column form): chunk or block width
  DBG_COPY_OUT,         // word planes to FP64: row outside d, planes overlapping
  DBG_TRACE,            // trace of the word planes: d above the padded order
  DBG_SHIFTED_F32,      // FP32 copy of H - sI: d above the padded order
  DBG_SITES
};

// Site names for the host's error message, in DbgSite order.
inline const char* dbg_site_name(int s) {
  static const char* const names[DBG_SITES] = {
      "none", "k_sym_gemm_w tile", "k_sym_gemm_wd tile", "k_sym_gemm_f* tile",
      "k_mirror_upper tile", "k_rowabs rows",
      "k_init_x0 extent", "k_form_reflector rows", "k_symthin chunk", "k_thin_finish rows",
      "k_cg_pass chunk/columns", "k_cg_update rows/column", "k_cg_init rows/column",
      "block-Lanczos kernel extent", "k_cg_step chunk/columns", "k_cg_apply rows/column",
      "k_gram_partial columns/rows", "k_thin_partial chunk/columns", "k_copy_out_w rows",
      "k_trace_w extent", "k_shifted_f32 extent"};
  return (s > 0 && s < DBG_SITES) ? names[s] : "unknown";
}

}  // namespace refl

#ifdef REFL_DEBUG
// One word per translation unit (internal linkage) and a host function,
// refl_dbg_take_<unit>(), that returns and clears it.  Expanded once at file
// scope in each unit that guards kernels.
#define REFL_DBG_UNIT(unit)                                                    \
  static __device__ int refl_dbg_word = 0;                                     \
  int refl_dbg_take_##unit() {                                                 \
    int v = 0, z = 0;                                                          \
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(refl_dbg_word), sizeof(int)) != hipSuccess) return -1; \
    if (v != 0 && hipMemcpyToSymbol(HIP_SYMBOL(refl_dbg_word), &z, sizeof(int)) != hipSuccess) \
      return -1;                                                               \
    return v;                                                                  \
  }
// Block-uniform condition only.  The record is an ordinary vector atomic.
#define REFL_GUARD(cond, site)                                                 \
  do {                                                                         \
    if (!(cond)) {                                                             \
      if (threadIdx.x == 0 && threadIdx.y == 0) atomicCAS(&refl_dbg_word, 0, (int)(site)); \
      return;                                                                  \
    }                                                                          \
  } while (0)
#else
#define REFL_DBG_UNIT(unit)
#define REFL_GUARD(cond, site) \
  do {                         \
  } while (0)
#endif
