// Patch estimation (Alg. 1, "Patch estimation", eigenspace form of Sec. 2.1):
// z^_i = U_k* diag(gamma_k*) U_k*^t z~_i + m_i = W_k* z~_i + m_i, with the
// patch mean m_i added back unshrunk.  W_k is formed once per beta in
// float64 (prep.hip); here it is applied as a grouped GEMM over the patches
// bucketed by component (bucket.hip): one wave takes a tile of up to 64
// patches that share a component, recomputes their DC-removed pixels from
// the current image, multiplies by W_k on MFMA and writes z^ in row planes:
// Zhat[dy][patch][dx] (8 planes of Np x 8 floats), so that each patch row
// is one 32-byte sector and the reprojection reads every plane row once.
//
// The tile count depends on the labels, so the grid is fixed and waves
// stride over the device-side tile list; a wave exits once its stride passes
// the total.
#include "common.h"

namespace fepll {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void wiener_f32_kernel(const float* __restrict__ x, int H,
                                                         int W, const float4* __restrict__ Wt,
                                                         int K, const int32_t* __restrict__ seg,
                                                         const int32_t* __restrict__ perm,
                                                         float* __restrict__ Zhat) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int Wp = W - 7;
  const int32_t* start = seg;
  const int32_t* count = seg + (K + 1);
  const int32_t* tpre = seg + (2 * K + 1);
  const int total = seg[3 * K + 2];
  const size_t Np8 = (size_t)(H - 7) * Wp * 8;  // floats per row plane of z^
  const int nwaves = gridDim.x * (blockDim.x >> 6);
  for (int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t < total; t += nwaves) {
    // component of tile t: last k with tpre[k] <= t
    int lo = 0, hi = K - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tpre[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const int k = lo;
    const int first = (t - tpre[k]) * kWienerTile;
    const int n = min(kWienerTile, count[k] - first);
    const int32_t* ids = perm + start[k] + first;

    // patches: lane holds pixels p = 2s + half of patches col and 32 + col
    const bool v0 = col < n, v1 = 32 + col < n;
    const int id0 = v0 ? ids[col] : ids[0];
    const int id1 = v1 ? ids[32 + col] : ids[0];
    const int r0 = id0 / Wp, c0 = id0 - r0 * Wp;
    const int r1 = id1 / Wp, c1 = id1 - r1 * Wp;
    float z0[32], z1[32];
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int s = 0; s < 32; ++s) {
      const int dy = s >> 2;
      const int dx = 2 * (s & 3) + half;
      z0[s] = x[(size_t)(r0 + dy) * W + c0 + dx];
      z1[s] = x[(size_t)(r1 + dy) * W + c1 + dx];
      s0 += (double)z0[s];
      s1 += (double)z1[s];
    }
    s0 += __shfl_xor(s0, 32);
    s1 += __shfl_xor(s1, 32);
    const double m0 = s0 * (1.0 / 64.0), m1 = s1 * (1.0 / 64.0);
#pragma unroll
    for (int s = 0; s < 32; ++s) {
      z0[s] = (float)((double)z0[s] - m0);
      z1[s] = (float)((double)z1[s] - m1);
    }
    const float fm0 = (float)m0, fm1 = (float)m1;
    // one 32-row block of W_k at a time (rows q = 32 qb + ...)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
      const float4* wp = Wt + (size_t)k * 1024 + qb * 512 + lane;
      float4 A[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) A[i] = wp[i * 64];
      f32x16 a0 = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      f32x16 a1 = a0;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
#define STEP(E, S)                                                            \
  a0 = __builtin_amdgcn_mfma_f32_32x32x2f32(A[i].E, z0[S], a0, 0, 0, 0);      \
  a1 = __builtin_amdgcn_mfma_f32_32x32x2f32(A[i].E, z1[S], a1, 0, 0, 0);
        STEP(x, 4 * i + 0)
        STEP(y, 4 * i + 1)
        STEP(z, 4 * i + 2)
        STEP(w, 4 * i + 3)
#undef STEP
      }
      // accumulator 4 g + e of lane l is pixel q = 32 qb + 8 g + 4 half + e:
      // row dy = 4 qb + g, columns dx = 4 half + e (one float4 of the row)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const size_t plane = (size_t)(4 * qb + g) * Np8;
        if (v0)
          *reinterpret_cast<float4*>(Zhat + plane + (size_t)id0 * 8 + 4 * half) =
              make_float4(a0[4 * g] + fm0, a0[4 * g + 1] + fm0, a0[4 * g + 2] + fm0,
                          a0[4 * g + 3] + fm0);
        if (v1)
          *reinterpret_cast<float4*>(Zhat + plane + (size_t)id1 * 8 + 4 * half) =
              make_float4(a1[4 * g] + fm1, a1[4 * g + 1] + fm1, a1[4 * g + 2] + fm1,
                          a1[4 * g + 3] + fm1);
      }
    }
  }
}

hipError_t launch_wiener_f32(const float* x, int H, int W, const float* Wt_t, int K,
                             const int32_t* seg, const int32_t* perm, float* Zhat,
                             hipStream_t st) {
  const int Np = (H - 7) * (W - 7);
  const int max_tiles = Np / kWienerTile + K;
  int blocks = (max_tiles + 3) / 4;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(wiener_f32_kernel, dim3(blocks), dim3(256), 0, st, x, H, W,
                     reinterpret_cast<const float4*>(Wt_t), K, seg, perm, Zhat);
  return hipGetLastError();
}

}  // namespace fepll
