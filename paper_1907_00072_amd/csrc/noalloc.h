// The fixed scratch array of pp_apply_noalloc (defined in noalloc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ppx {

// Size of the array on each GPU: three FP64 vectors of 2^21 rows (the chain's
// temporaries) plus 4 KiB for the CSR check's flag and alignment.
constexpr int64_t kNoAllocMaxRowsF64 = int64_t(1) << 21;
constexpr size_t kNoAllocScratchBytes = 3 * size_t(kNoAllocMaxRowsF64) * sizeof(double) + 4096;
// devices whose array address is kept
constexpr int kNoAllocMaxDevices = 64;

// The current device's copy of the array: its device address and size.  The
// address is looked up with hipGetSymbolAddress on the first call on each
// device (that device current) and kept; later calls only return it.  Not
// thread-safe on its own: the caller holds the library lock.
hipError_t noalloc_scratch(void **ptr, size_t *bytes);

}  // namespace ppx
