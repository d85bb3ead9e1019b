// Host-side helpers shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "fepll.h"

namespace fepll {

// Records the message returned by fepll_last_error() and passes s through.
fepll_status fail(fepll_status s, const std::string& msg);
void clear_error();

// Every device buffer of the library goes through these two: the bytes held
// are counted, and an allocation that would take them past the limit set by
// fepll_set_memory_limit fails with hipErrorOutOfMemory, as a full device.
hipError_t dev_alloc(void** p, size_t bytes);
void dev_free(void* p);

template <class T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) return hipSuccess;
  return dev_alloc((void**)p, n * sizeof(T));
}

template <class T>
void dfree(T*& p) {
  if (p) dev_free(p);
  p = nullptr;
}

// What an entry point outside the handle's own translation unit may read of
// a handle: its size, its device and its float64 mixture (device copies made
// at creation, the spectra in use).
struct GmmView {
  int K;
  int device;
  const double* U64;
  const double* lam64;
  const double* w64;
};
GmmView gmm_view(const fepll_gmm* g);

}  // namespace fepll

#define HIPX(call)                                                                        \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return ::fepll::fail(e_ == hipErrorOutOfMemory ? FEPLL_ENOMEM : FEPLL_EDEVICE,      \
                           std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)
