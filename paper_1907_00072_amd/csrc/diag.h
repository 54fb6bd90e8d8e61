// Failure diagnostics shared by the library's translation units.
//
// Every HIP call the library checks goes through PPD_TRY_HIP: on failure it
// records where (source file and line), which call and the runtime's error name
// in a per-thread buffer that pp_last_error() returns, and prints the same line
// to stderr when PP_LOG >= 1.  Entry points that touch the device call
// ppd::enter() first: it takes any error left pending by an earlier runtime
// call of the process (the kernel-launch checks read the pending error, so a
// stale one would otherwise be reported by the library's first launch) and
// clears the record.
#pragma once

#include <hip/hip_runtime.h>

namespace ppd {

// Record a failed HIP call; returns e.
hipError_t note(hipError_t e, const char *expr, const char *file, int line);
// Record an argument error's explanation (printf format), for pp_last_error().
void note_msg(const char *fmt, ...);
// Start of a device entry point: clear the record and any pending runtime error.
void enter(const char *entry);
// The record of this thread's last failed HIP call or explained argument error
// ("" if none since the thread's last entry point).
const char *last_detail();
// PP_LOG level (0 if unset), read once.
int log_level();

}  // namespace ppd

#define PPD_TRY_HIP(expr, fail)                                            \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) {                                                \
      (void)ppd::note(e_, #expr, __FILE__, __LINE__);                      \
      return (fail);                                                       \
    }                                                                      \
  } while (0)
