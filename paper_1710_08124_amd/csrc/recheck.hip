// Float64 re-selection of the patches the float32 E-step could not certify
// (Alg. 1, Gaussian selection, eigenspace form of Sec. 2.1, all in float64):
// z~ = patch - mean, c = U_k^t z~, cost_k = L_k + sum_j c_j^2 / nu_kj,
// k* = first k of minimal cost.
//
// Each list entry carries the components that can still hold the patch's
// exact minimum (at most 4, in ascending order) or asks for all K; the
// float32 bound guarantees every other component has a larger exact cost,
// so the minimum over the candidates is the minimum over all K.
//
// The list length lives on the device, so the kernel is launched with a
// fixed grid and each wave strides over the list; every wave exits once its
// stride passes the length.  Lane j owns eigen-direction j.
#include "common.h"

namespace fepll {

namespace {
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}
}  // namespace

__global__ __launch_bounds__(256) void recheck_f64_kernel(
    const float* __restrict__ x, int H, int W, const double* __restrict__ U64,
    const double* __restrict__ invnu, const double* __restrict__ L64, int K,
    const int32_t* __restrict__ list_count, const int4* __restrict__ list,
    int32_t* __restrict__ labels) {
  __shared__ double zsh[4][kP];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double* zs = zsh[wave];
  const int Wp = W - 7;
  const int n = *list_count;
  const int nwaves = gridDim.x * 4;
  for (int e = blockIdx.x * 4 + wave; e < n; e += nwaves) {
    const int4 ent = list[e];
    const int idx = ent.x;
    const int r = idx / Wp, c = idx - (idx / Wp) * Wp;
    const double v = (double)x[(size_t)(r + (lane >> 3)) * W + c + (lane & 7)];
    const double m = wave_sum(v) * (1.0 / 64.0);
    zs[lane] = v - m;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    const bool all = ent.y > 4;
    const int ncand = all ? K : ent.y;
    double best = INFINITY;
    int bk = 0;
    for (int i = 0; i < ncand; ++i) {
      int k = i;
      if (!all) {
        const int word = (i < 2) ? ent.z : ent.w;
        k = (i & 1) ? ((word >> 16) & 0xffff) : (word & 0xffff);
      }
      const double* uk = U64 + (size_t)k * kP * kP + lane;
      double cj = 0.0;
#pragma unroll 16
      for (int p = 0; p < kP; ++p) cj = fma(uk[p * kP], zs[p], cj);
      const double cost = L64[k] + wave_sum(cj * cj * invnu[k * kP + lane]);
      if (cost < best) {
        best = cost;
        bk = k;
      }
    }
    if (lane == 0) labels[idx] = bk;
    __builtin_amdgcn_wave_barrier();
  }
}

hipError_t launch_recheck_f64(const float* x, int H, int W, const double* U64,
                              const double* invnu64_t, const double* L64_t, int K,
                              const int32_t* list_count, const int32_t* list, int32_t* labels,
                              int max_list, hipStream_t st) {
  int blocks = (max_list + 3) / 4;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(recheck_f64_kernel, dim3(blocks), dim3(256), 0, st, x, H, W, U64, invnu64_t,
                     L64_t, K, list_count, reinterpret_cast<const int4*>(list), labels);
  return hipGetLastError();
}

}  // namespace fepll
