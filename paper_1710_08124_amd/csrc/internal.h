// Host-side helpers shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "fepll.h"

namespace fepll {

// Records the message returned by fepll_last_error() and passes s through.
fepll_status fail(fepll_status s, const std::string& msg);
void clear_error();

template <class T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) return hipSuccess;
  return hipMalloc((void**)p, n * sizeof(T));
}

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

}  // namespace fepll

#define HIPX(call)                                                                        \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return ::fepll::fail(e_ == hipErrorOutOfMemory ? FEPLL_ENOMEM : FEPLL_EDEVICE,      \
                           std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)
