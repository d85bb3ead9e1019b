// Per-beta constants of the eigenspace formulation (Sec. 2.1, the terms
// defined after eq:selection_eigenspace): nu_kj = lambda_kj + 1/beta,
// gamma_kj = lambda_kj / nu_kj, iota_k = -2 log w_k.  Computed in float64
// from the float64 eigendecomposition, then rounded once to float32 in the
// operand layouts the MFMA kernels read (see common.h).
#include "common.h"

namespace fepll {

__global__ __launch_bounds__(256) void prep_kernel(const double* __restrict__ U64,
                                                   const double* __restrict__ lam,
                                                   const double* __restrict__ w, int K,
                                                   Schedule sch, float* __restrict__ Ut,
                                                   uint16_t* __restrict__ Ub,
                                                   float* __restrict__ Wt,
                                                   float* __restrict__ L32,
                                                   double* __restrict__ L64,
                                                   double* __restrict__ invnu64,
                                                   uint8_t* __restrict__ Uf,
                                                   int32_t* __restrict__ Ue) {
  const int k = blockIdx.x;
  const int t = blockIdx.y;
  const double beta = sch.beta[t];
  __shared__ double Us[kP * kP];  // U_k[p][j]
  __shared__ double nu[kP], gam[kP], rs[kP];
  for (int i = threadIdx.x; i < kP * kP; i += blockDim.x) Us[i] = U64[(size_t)k * kP * kP + i];
  if (threadIdx.x < kP) {
    const int j = threadIdx.x;
    const double l = lam[k * kP + j];
    const double n = l + 1.0 / beta;
    nu[j] = n;
    gam[j] = l / n;
    rs[j] = 1.0 / sqrt(n);
    invnu64[((size_t)t * K + k) * kP + j] = 1.0 / n;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = -2.0 * log(w[k]);
    for (int j = 0; j < kP; ++j) s += log(nu[j]);
    L64[t * K + k] = s;
    L32[t * K + k] = (float)s;
  }
  float* ut = Ut + ((size_t)t * K + k) * kTileStride;
  float* wt = Wt + ((size_t)t * K + k) * kTileStride;
  uint16_t* ub = Ub + ((size_t)t * K + k) * kTileStride;
  for (int idx = threadIdx.x; idx < kTileStride; idx += blockDim.x) {
    const int e = idx & 3, l = (idx >> 2) & 63, i = (idx >> 8) & 7, jb = idx >> 11;
    const int s = 4 * i + e;
    const int p = 2 * s + (l >> 5);
    const int j = 32 * jb + (l & 31);
    ut[idx] = (float)(Us[p * kP + j] * rs[j]);
    {
      // bfloat16 table: same entries, MFMA 16x16x32 operand order
      const int eb = idx & 7, lb = (idx >> 3) & 63, tb = (idx >> 9) & 1, rb = idx >> 10;
      const int pb = 32 * tb + 8 * (lb >> 4) + eb;
      const int jb2 = 16 * rb + (lb & 15);
      uint32_t u = __float_as_uint((float)(Us[pb * kP + jb2] * rs[jb2]));
      u += 0x7fffu + ((u >> 16) & 1u);
      ub[idx] = (uint16_t)(u >> 16);
    }
    // Wiener operand: row q of W_k = U_k diag(gamma) U_k^t, column pw;
    // depth step s pairs pixel s (lanes 0..31) with pixel 32 + s (lanes
    // 32..63), so each lane's patch operand is 32 consecutive pixels
    const int q = j;
    const int pw = 32 * (l >> 5) + s;
    double acc = 0.0;
    for (int jj = 0; jj < kP; ++jj) acc += Us[q * kP + jj] * gam[jj] * Us[pw * kP + jj];
    wt[idx] = (float)acc;
  }

  // e4m3 table: Ut_k scaled by 2^-e, e the smallest exponent that brings
  // max |Ut_k| to at most 448 (the largest finite e4m3), rounded float64 ->
  // float32 -> e4m3 (nearest even); the scale's E8M0 code is e + 127
  __shared__ double red[256];
  double mx = 0.0;
  for (int i = threadIdx.x; i < kP * kP; i += blockDim.x)
    mx = fmax(mx, fabs(Us[i] * rs[i & (kP - 1)]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  mx = red[0];
  int e = 0;
  if (mx > 0.0) {
    int ex;
    const double f = frexp(mx, &ex);
    e = (f <= 0.875) ? ex - 9 : ex - 8;
    e = max(-127, min(e, 127));
  }
  if (threadIdx.x == 0) Ue[t * K + k] = e + 127;
  uint8_t* uf = Uf + ((size_t)t * K + k) * kTileStride;
  for (int bi = threadIdx.x; bi < kTileStride; bi += blockDim.x) {
    // byte bb of uint4 u = (2 rb + part) * 64 + l: row j = 32 rb + (l & 31),
    // pixel p = 32 (l >> 5) + 16 part + bb
    const int bb = bi & 15, u = bi >> 4;
    const int l = u & 63, part = (u >> 6) & 1, rb = u >> 7;
    const int j = 32 * rb + (l & 31);
    const int p = 32 * (l >> 5) + 16 * part + bb;
    const float q = (float)ldexp(Us[p * kP + j] * rs[j], -e);
    uf[bi] = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(q, 0.f, 0, false) & 0xff);
  }
}

hipError_t launch_prep(const double* U64, const double* lam64, const double* w64, int K,
                       const Schedule& sch, float* Ut, uint16_t* Ub, float* Wt, float* L32,
                       double* L64, double* invnu64, uint8_t* Uf, int32_t* Ue, hipStream_t st) {
  dim3 grid(K, sch.T);
  hipLaunchKernelGGL(prep_kernel, grid, dim3(256), 0, st, U64, lam64, w64, K, sch, Ut, Ub, Wt,
                     L32, L64, invnu64, Uf, Ue);
  return hipGetLastError();
}

}  // namespace fepll
