// Block-level synchronisation helpers shared by the kernel sources.
#pragma once
#include <hip/hip_runtime.h>

namespace refl {

// A barrier that orders only LDS: global loads in flight stay in flight
// (__syncthreads waits for every outstanding memory access of the wave).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace refl
