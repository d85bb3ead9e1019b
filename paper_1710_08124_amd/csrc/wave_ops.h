// Small wave-level helpers shared by the reduced-precision selection kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace fepll {

// best / second smallest cost and the argmin (first k on ties), branch-free
__device__ __forceinline__ void keep_best(float cost, int k, float& best, float& second,
                                          int& bk) {
  const bool better = cost < best;
  second = better ? best : fminf(second, cost);
  bk = better ? k : bk;
  best = better ? cost : best;
}

// Exchange between lane halves (v_permlane32_swap: lanes 32..63 of a with
// lanes 0..31 of b) and between 16-lane rows of each half
// (v_permlane16_swap: rows 1 and 3 of a with rows 0 and 2 of b).  After
// swap(a, b), a + b is, in lanes of the lower half (row), the pair sum of a
// and, in the upper half (row), the pair sum of b.
__device__ __forceinline__ float pair_sum32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float pair_sum16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

}  // namespace fepll
