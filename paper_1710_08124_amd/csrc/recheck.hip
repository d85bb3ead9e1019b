// Float64 re-selection of the patches the float32 E-step could not certify
// (Alg. 1, Gaussian selection, eigenspace form of Sec. 2.1, all in float64):
// z~ = patch - mean, c = U_k^t z~, cost_k = L_k + sum_j c_j^2 / nu_kj,
// k* = first k of minimal cost.
//
// The flagged list has a device-side length, so the kernel is launched with
// a fixed grid and each workgroup strides over the list; every workgroup
// exits once its stride passes the length.  One wave handles a batch of
// kBatch patches: lane j owns eigen-direction j and reuses each U_k[p][j]
// it loads for the whole batch.
#include "common.h"

namespace fepll {

namespace {
constexpr int kBatch = 16;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}
}  // namespace

__global__ __launch_bounds__(64) void recheck_f64_kernel(
    const float* __restrict__ x, int H, int W, const double* __restrict__ U64,
    const double* __restrict__ invnu, const double* __restrict__ L64, int K,
    const int32_t* __restrict__ list_count, const int32_t* __restrict__ list,
    int32_t* __restrict__ labels) {
  const int lane = threadIdx.x;
  const int Wp = W - 7;
  const int n = *list_count;
  __shared__ double zs[kBatch][kP];
  for (int base = blockIdx.x * kBatch; base < n; base += gridDim.x * kBatch) {
    const int nb = min(kBatch, n - base);
    for (int b = 0; b < kBatch; ++b) {
      double v = 0.0;
      if (b < nb) {
        const int idx = list[base + b];
        const int r = idx / Wp, c = idx - (idx / Wp) * Wp;
        v = (double)x[(size_t)(r + (lane >> 3)) * W + c + (lane & 7)];
      }
      const double m = wave_sum(v) * (1.0 / 64.0);
      zs[b][lane] = (b < nb) ? v - m : 0.0;
    }
    __syncthreads();
    double best[kBatch];
    int bk[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      best[b] = INFINITY;
      bk[b] = 0;
    }
    for (int k = 0; k < K; ++k) {
      double c[kBatch];
#pragma unroll
      for (int b = 0; b < kBatch; ++b) c[b] = 0.0;
      const double* uk = U64 + (size_t)k * kP * kP + lane;
      for (int p = 0; p < kP; ++p) {
        const double u = uk[p * kP];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) c[b] = fma(u, zs[b][p], c[b]);
      }
      const double in = invnu[k * kP + lane];
      const double Lk = L64[k];
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const double cost = Lk + wave_sum(c[b] * c[b] * in);
        if (cost < best[b]) {
          best[b] = cost;
          bk[b] = k;
        }
      }
    }
    if (lane < nb) {
      int lab = bk[0];
#pragma unroll
      for (int b = 1; b < kBatch; ++b)
        if (lane == b) lab = bk[b];
      labels[list[base + lane]] = lab;
    }
    __syncthreads();
  }
}

hipError_t launch_recheck_f64(const float* x, int H, int W, const double* U64,
                              const double* invnu64_t, const double* L64_t, int K,
                              const int32_t* list_count, const int32_t* list, int32_t* labels,
                              int max_list, hipStream_t st) {
  int blocks = (max_list + kBatch - 1) / kBatch;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(recheck_f64_kernel, dim3(blocks), dim3(64), 0, st, x, H, W, U64, invnu64_t,
                     L64_t, K, list_count, list, labels);
  return hipGetLastError();
}

}  // namespace fepll
