// Per-beta constants of the eigenspace formulation (Sec. 2.1, the terms
// defined after Eq. (8)): nu_kj = lambda_kj + 1/beta,
// gamma_kj = lambda_kj / nu_kj, iota_k = -2 log w_k.  Computed in float64
// from the float64 eigendecomposition, then rounded once to the operand
// layouts the kernels read (see common.h).  One workgroup per (component,
// beta slot); the slots are a list of betas (the T iterations of one image,
// or of every image of a batch).
#include "common.h"

namespace fepll {

namespace {
constexpr int UP = kP + 1;  // LDS pitch of U_k rows (doubles): conflict-free column reads
}

__global__ __launch_bounds__(256) void prep_kernel(const double* __restrict__ U64,
                                                   const double* __restrict__ lam,
                                                   const double* __restrict__ w, int K,
                                                   const double* __restrict__ betas, int mask,
                                                   ConstTables tb) {
  const int k = blockIdx.x;
  const int t = blockIdx.y;  // beta slot
  const double beta = betas[t];
  __shared__ double Us[kP * UP];  // U_k[p][j] at p * UP + j
  __shared__ double Ws[kP * UP];  // W_k[q][p]
  __shared__ double nu[kP], gam[kP], rs[kP], rsf[kP];
  __shared__ double red[256];
  for (int i = threadIdx.x; i < kP * kP; i += blockDim.x)
    Us[(i >> 6) * UP + (i & 63)] = U64[(size_t)k * kP * kP + i];
  if (threadIdx.x < kP) {
    const int j = threadIdx.x;
    const double l = lam[k * kP + j];
    const double n = l + 1.0 / beta;
    nu[j] = n;
    gam[j] = l / n;
    rs[j] = 1.0 / sqrt(n);
    if (mask & kTabF32) tb.invnu64[((size_t)t * K + k) * kP + j] = 1.0 / n;
  }
  __syncthreads();
  // flat-tail form of the reduced-precision operands (Sec. 3.1): with a
  // tail (r_k < 64), cost = L_k + |z~|^2 / nu_P - sum_{j < r_k} c_j^2
  // (1/nu_P - 1/nu_j), so the kept columns carry sqrt(1/nu_P - 1/nu_j) (>= 0:
  // the tail average is at most every kept eigenvalue) and the others
  // vanish; without a tail, the plain nu^-1/2
  const int rk = tb.rk ? tb.rk[k] : kP;
  if (threadIdx.x < kP) {
    const int j = threadIdx.x;
    if (rk >= kP) rsf[j] = rs[j];
    else rsf[j] = (j < rk) ? sqrt(fmax(1.0 / nu[rk] - 1.0 / nu[j], 0.0)) : 0.0;
  }
  if (threadIdx.x == 0 && (mask & (kTabBF16 | kTabF8)))
    tb.Pinv[t * K + k] = (rk >= kP) ? 0.f : (float)(1.0 / nu[rk]);
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = -2.0 * log(w[k]);
    for (int j = 0; j < kP; ++j) s += log(nu[j]);
    if (mask & kTabF32) tb.L64[t * K + k] = s;
    tb.L32[t * K + k] = (float)s;
  }
  // W_k = U_k diag(gamma) U_k^t, a 4 x 4 block of it per thread
  {
    const int q0 = 4 * (threadIdx.x >> 4), p0 = 4 * (threadIdx.x & 15);
    double acc[4][4] = {};
    for (int jj = 0; jj < kP; ++jj) {
      const double gj = gam[jj];
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = Us[(q0 + i) * UP + jj] * gj;
        b[i] = Us[(p0 + i) * UP + jj];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) Ws[(q0 + i) * UP + p0 + j] = acc[i][j];
  }
  // largest |Ut_k| for the e4m3 scale
  double mx = 0.0;
  if (mask & kTabF8)
    for (int i = threadIdx.x; i < kP * kP; i += blockDim.x)
      mx = fmax(mx, fabs(Us[(i >> 6) * UP + (i & 63)] * rsf[i & 63]));
  red[threadIdx.x] = mx;
  __syncthreads();
  const size_t tk = (size_t)t * K + k;
  float* wt = tb.Wt + tk * kTileStride;
  float* ut = (mask & kTabF32) ? tb.Ut + tk * kTileStride : nullptr;
  uint16_t* ub = (mask & kTabBF16) ? tb.Ub + tk * kTileStride : nullptr;
  uint16_t* wh = (tb.Wh && (mask & (kTabBF16 | kTabF8))) ? tb.Wh + tk * kTileStride : nullptr;
  for (int idx = threadIdx.x; idx < kTileStride; idx += blockDim.x) {
    const int e = idx & 3, l = (idx >> 2) & 63, i = (idx >> 8) & 7, jb = idx >> 11;
    const int s = 4 * i + e;
    const int j = 32 * jb + (l & 31);
    if (ut) {
      const int p = 2 * s + (l >> 5);
      ut[idx] = (float)(Us[p * UP + j] * rs[j]);
    }
    if (ub) {
      // bfloat16 table: MFMA 16x16x32 operand order
      const int eb = idx & 7, lb = (idx >> 3) & 63, tbk = (idx >> 9) & 1, rb = idx >> 10;
      const int pb = 32 * tbk + 8 * (lb >> 4) + eb;
      const int jb2 = 16 * rb + (lb & 15);
      uint32_t u = __float_as_uint((float)(Us[pb * UP + jb2] * rsf[jb2]));
      u += 0x7fffu + ((u >> 16) & 1u);
      ub[idx] = (uint16_t)(u >> 16);
    }
    // Wiener operand: row q of W_k, column pw; depth step s pairs pixel s
    // (lanes 0..31) with pixel 32 + s (lanes 32..63), so each lane's patch
    // operand is 32 consecutive pixels
    wt[idx] = (float)Ws[j * UP + 32 * (l >> 5) + s];
    if (wh) {
      // binary16 Wiener operand: MFMA 32x32x16 order, rounded via float32
      const int eh = idx & 7, lh = (idx >> 3) & 63, sh = (idx >> 9) & 3, qb = idx >> 11;
      const float f = (float)Ws[(32 * qb + (lh & 31)) * UP + 16 * sh + 8 * (lh >> 5) + eh];
      const _Float16 h = (_Float16)fresh(f);  // (two roundings: not fused)
      wh[idx] = __builtin_bit_cast(uint16_t, h);
    }
  }
  if (!(mask & kTabF8)) return;

  // e4m3 table: Ut_k scaled by 2^-e, e the smallest exponent that brings
  // max |Ut_k| to at most 448 (the largest finite e4m3), rounded float64 ->
  // float32 -> e4m3 (nearest even); the scale's E8M0 code is e + 127
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  mx = red[0];
  int ee = 0;
  if (mx > 0.0) {
    int ex;
    const double f = frexp(mx, &ex);
    ee = (f <= 0.875) ? ex - 9 : ex - 8;
    ee = max(-127, min(ee, 127));
  }
  if (threadIdx.x == 0) tb.Ue[tk] = ee + 127;
  uint8_t* uf = tb.Uf + tk * kTileStride;
  for (int bi = threadIdx.x; bi < kTileStride; bi += blockDim.x) {
    // byte bb of uint4 u = (2 rb + part) * 64 + l: row j = 32 rb + (l & 31),
    // pixel p = 32 (l >> 5) + 16 part + bb
    const int bb = bi & 15, u = bi >> 4;
    const int l = u & 63, part = (u >> 6) & 1, rb = u >> 7;
    const int j = 32 * rb + (l & 31);
    const int p = 32 * (l >> 5) + 16 * part + bb;
    const float q = (float)ldexp(Us[p * UP + j] * rsf[j], -ee);
    uf[bi] = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(q, 0.f, 0, false) & 0xff);
  }
}

hipError_t launch_prep(const double* U64, const double* lam64, const double* w64, int K,
                       const double* betas, int S, int mask, const ConstTables& tb,
                       hipStream_t st) {
  dim3 grid(K, S);
  hipLaunchKernelGGL(prep_kernel, grid, dim3(256), 0, st, U64, lam64, w64, K, betas, mask, tb);
  return hipGetLastError();
}

}  // namespace fepll
