// The fixed device array behind pp_apply_noalloc (include/pp.h): the chain's
// temporaries and the CSR check's flag for callers that cannot allocate.
//
// `scratch` is a file-scope device array: each GPU the library runs on holds its
// own copy, at its own address, from the library's load until the process ends.
// In host code the name stands for a host-side shadow, not a device address, so
// host code never passes it to a kernel or a copy: noalloc_scratch() looks up
// the current device's address once (hipGetSymbolAddress, with that device
// current) and every caller uses that pointer.
#include <hip/hip_runtime.h>

#include "noalloc.h"

namespace {

static __device__ __align__(256) double scratch[ppx::kNoAllocScratchBytes / sizeof(double)];

// device address of `scratch` per device (nullptr until the first lookup);
// written under the library lock that every entry point takes
void *g_scratch_ptr[ppx::kNoAllocMaxDevices] = {};

}  // namespace

namespace ppx {

hipError_t noalloc_scratch(void **ptr, size_t *bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  *bytes = kNoAllocScratchBytes;
  return hipSuccess;
}

}  // namespace ppx
