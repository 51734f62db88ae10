// Fixed device scratch of the allocation-free entry point (refl_sign_noalloc).
//
// The array below is the workspace of every refl_sign_noalloc call on a
// device: each device the library runs on holds its own copy, from module
// load until the process ends.  In host code its name is only a stand-in;
// the device address comes from hipGetSymbolAddress, resolved once per
// device (with that device current) by refl_create through
// noalloc_scratch() and cached here, and only that address is ever passed
// to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.h"

static __device__ __align__(256) unsigned char scratch[refl::NOALLOC_SCRATCH_BYTES];

namespace refl {

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || ((uintptr_t)p % 256) != 0) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

}  // namespace refl
