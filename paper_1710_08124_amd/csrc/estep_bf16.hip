// Gaussian selection with bfloat16 projections (same step as estep.hip:
// Alg. 1 patch extraction + Gaussian selection in the eigenspace form of
// Sec. 2.1), for the reduced-precision mode: the DC-removed patches and the
// scaled eigenbases Ut_k = U_k diag(nu_k)^-1/2 are rounded to bfloat16, the
// products accumulate in float32 on v_mfma_f32_32x32x16_bf16, and the
// squared norms, the log-determinant terms L_k and the argmin stay float32.
// Labels are not certified in this mode: they are an approximation whose
// agreement with the exact selection is measured, not assumed.
//
// One MFMA consumes 16 pixels of 32 patches: lane l supplies the 8 pixels
// 16 t + 8 (l >> 5) + e (e = 0..7) of patch (l & 31) -- exactly one 8-pixel
// row, dy = 2 t + (l >> 5), of the patch -- and the A operand supplies the
// same 8 pixels of eigen-direction j = 32 jb + (l & 31).  A wave holds 128
// patches (four blocks of 32 along a patch row) as B operands for the whole
// K loop; per component it issues 2 (eigen blocks) x 4 (depth steps) x 4
// (patch blocks) MFMAs and 128 float32 FMAs of squares.
#include "common.h"

namespace fepll {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {
constexpr int CB = 4;  // blocks of 32 patches per wave

__device__ __forceinline__ uint32_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ uint32_t pack2(float a, float b) {
  return bf16_rne(a) | (bf16_rne(b) << 16);
}
__device__ __forceinline__ f32x16 mfma_bf16(uint4 a, uint4 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
__device__ __forceinline__ void keep_best(float cost, int k, float& best, float& second,
                                          int& bk) {
  if (cost < best) {
    second = best;
    best = cost;
    bk = k;
  } else if (cost < second) {
    second = cost;
  }
}
}  // namespace

__global__ __launch_bounds__(256, 2) void estep_bf16_kernel(
    const float* __restrict__ x, int H, int W, const uint4* __restrict__ Ub,
    const float* __restrict__ L, int K, int32_t* __restrict__ labels,
    float* __restrict__ best_out, float* __restrict__ second_out) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int Hp = H - 7, Wp = W - 7;
  const int r = blockIdx.y * 4 + wave;
  const int c0 = blockIdx.x * (32 * CB);
  const int rr = min(r, Hp - 1);

  // ---- B operands: DC-removed patches, bfloat16
  uint4 zb[CB][4];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int cc = min(c0 + 32 * cb + col, Wp - 1);
    float v[4][8];
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float* row = x + (size_t)(rr + 2 * t + half) * W + cc;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        v[t][e] = row[e];
        s += (double)v[t][e];
      }
    }
    s += __shfl_xor(s, 32);
    const double m = s * (1.0 / 64.0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float d[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) d[e] = (float)((double)v[t][e] - m);
      zb[cb][t] = make_uint4(pack2(d[0], d[1]), pack2(d[2], d[3]), pack2(d[4], d[5]),
                             pack2(d[6], d[7]));
    }
  }

  float bA = INFINITY, sA = INFINITY, bB = INFINITY, sB = INFINITY;
  int kA = 0, kB = 0;
  const uint4* up = Ub + lane;  // [K][2][4][64] uint4
  for (int k = 0; k < K; ++k) {
    uint4 A[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) A[i] = up[(size_t)k * 512 + i * 64];
    float q[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) q[cb] = 0.f;
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      f32x16 acc[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
        acc[cb] = (f32x16){0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                           0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[cb] = mfma_bf16(A[jb * 4 + t], zb[cb][t], acc[cb]);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int i = 0; i < 16; ++i) q[cb] = fmaf(acc[cb][i], acc[cb][i], q[cb]);
      // keep the two eigen blocks in sequence: one set of accumulators live
      __builtin_amdgcn_sched_barrier(0);
    }
    // lanes < 32 finish blocks 0 and 2, lanes >= 32 blocks 1 and 3
    const float s0 = half ? q[0] : q[1];
    const float s1 = half ? q[2] : q[3];
    const float r0 = __shfl_xor(s0, 32);
    const float r1 = __shfl_xor(s1, 32);
    const float Lk = L[k];
    keep_best(Lk + ((half ? q[1] : q[0]) + r0), k, bA, sA, kA);
    keep_best(Lk + ((half ? q[3] : q[2]) + r1), k, bB, sB, kB);
  }
  if (r < Hp) {
    const int ca = c0 + 32 * half + col;
    const int cb2 = c0 + 64 + 32 * half + col;
    if (ca < Wp) {
      const int idx = r * Wp + ca;
      labels[idx] = kA;
      if (best_out) best_out[idx] = bA;
      if (second_out) second_out[idx] = sA;
    }
    if (cb2 < Wp) {
      const int idx = r * Wp + cb2;
      labels[idx] = kB;
      if (best_out) best_out[idx] = bB;
      if (second_out) second_out[idx] = sB;
    }
  }
}

hipError_t launch_estep_bf16(const float* x, int H, int W, const uint16_t* Ub_t,
                             const float* L32_t, int K, int32_t* labels, float* best,
                             float* second, hipStream_t st) {
  const int Hp = H - 7, Wp = W - 7;
  dim3 grid((Wp + 32 * CB - 1) / (32 * CB), (Hp + 3) / 4);
  hipLaunchKernelGGL(estep_bf16_kernel, grid, dim3(256), 0, st, x, H, W,
                     reinterpret_cast<const uint4*>(Ub_t), L32_t, K, labels, best, second);
  return hipGetLastError();
}

}  // namespace fepll
