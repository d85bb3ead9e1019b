// Gaussian selection for every patch (Alg. 1, patch extraction + Gaussian
// selection, in the eigenspace form of Sec. 2.1): per patch i and component
// k the projection c = U_k^t z~_i (Eq. (7)) and the cost
// L_k + sum_j c_j^2 / nu_kj (Eq. (8)), argmin over k.
//
// Float32 MFMA kernel for gfx950.  The contraction is
//   C[(k, j), i] = sum_p Ut_k[p][j] * z~_i[p],   Ut_k = U_k diag(nu_k)^-1/2,
// an Np x 64 by 64 x 64K product that is never stored: each 32x32 block of
// C lives in MFMA accumulators just long enough for its squares to be
// summed.  v_mfma_f32_32x32x2_f32 puts 32 eigen-directions on the rows and
// 32 patches on the columns, so after a 64-deep chain lane l holds 16 of the
// 32 coefficients of patch (l & 31) and lane l ^ 32 the other 16: the
// squared norm needs one cross-lane add.
//
// Work split: a workgroup of 4 waves covers 4 patch rows x 64 patch
// columns; each wave keeps its 64 DC-removed patches in registers (the MFMA
// B operand) for the whole K loop and streams the per-component A operand
// (16 KB per k, shared by every wave of the chip through L2) with one
// component of software prefetch.
//
// Certification: the float32 costs carry a forward rounding-error bound
// (derivation below); a patch whose best cost is not separated from the
// others by the bound is appended to a list with the few components that
// can still hold its exact minimum, and re-selected in float64 by
// recheck.hip.  Labels then equal an exact evaluation of the selection rule.
#include "common.h"

namespace fepll {

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {
constexpr float kU = 5.9604644775390625e-8f;  // 2^-24: float32 unit roundoff
constexpr float kKappa = 2.0f;                // safety factor on the bound

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
}  // namespace

// Error bound of one float32 cost (Higham-style forward bounds,
// gamma_n = n u / (1 - n u)):
//  * z~ is rounded once from a float64 difference, Ut once from float64, and
//    each coefficient is a 64-term dot product, so
//    |dc_j| <= gamma_66 * sum_p |Ut_pj| |z~_p| <= gamma_66 * ||Ut_:j|| ||z~||
//           <= gamma_66 * sqrt(beta) * ||z~|| =: a      (||Ut_:j|| = nu^-1/2)
//  * Q = sum_j c_j^2 over 64 terms:
//    |dQ| <= gamma_64 Q + 2 a sum_j |c_j| + 64 a^2
//         <= gamma_64 Q + 16 a sqrt(Q) + 64 a^2
//  * cost = fl(L32 + Q), L32 rounded once from float64: + u (|L| + |cost|).
// With Q <= cost - min_k L_k this gives one bound E(cost) for every k of the
// patch (kappa = 2 on top); E grows much slower than its argument, so
// c - E(c) is increasing and:
//  * the float32 argmin is exact when best + E(best) < second - E(second);
//  * otherwise only components with cost <= best + 3 E(best) can hold the
//    exact minimum.  The kernel keeps up to kCand of them (pruned whenever
//    the running best improves) and hands them to the float64 re-selection;
//    more than kCand at once marks the patch for a full-K re-selection.
namespace {
constexpr int kCand = 4;
}

__global__ __launch_bounds__(256, 2) void estep_f32_kernel(
    const float* __restrict__ x, int H, int W, const float4* __restrict__ Ut,
    const float* __restrict__ L, int K, float sqrt_beta, int32_t* __restrict__ labels,
    float* __restrict__ best_out, float* __restrict__ second_out, int32_t* __restrict__ flags,
    int32_t* __restrict__ list_count, int4* __restrict__ list) {
  __shared__ float cand_v[256 * kCand];
  __shared__ int cand_k[256 * kCand];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int Hp = H - 7;
  const int Wp = W - 7;
  const int r = blockIdx.y * 4 + wave;
  const int c0 = blockIdx.x * 64;
  const int rr = min(r, Hp - 1);

  // smallest L_k and largest |L_k| (wave-uniform)
  float Lmin = INFINITY, Labs = 0.f;
  for (int k = lane; k < K; k += 64) {
    Lmin = fminf(Lmin, L[k]);
    Labs = fmaxf(Labs, fabsf(L[k]));
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    Lmin = fminf(Lmin, __shfl_xor(Lmin, m));
    Labs = fmaxf(Labs, __shfl_xor(Labs, m));
  }

  // ---- patch extraction: lane holds pixels p = 2s + half of its patches
  float z0[32], z1[32];
  double s0 = 0.0, s1 = 0.0;
  {
    const int ca = min(c0 + col, Wp - 1);
    const int cb = min(c0 + 32 + col, Wp - 1);
#pragma unroll
    for (int s = 0; s < 32; ++s) {
      const int dy = s >> 2;
      const int dx = 2 * (s & 3) + half;
      const float* row = x + (size_t)(rr + dy) * W;
      z0[s] = row[ca + dx];
      z1[s] = row[cb + dx];
      s0 += (double)z0[s];
      s1 += (double)z1[s];
    }
  }
  s0 += __shfl_xor(s0, 32);
  s1 += __shfl_xor(s1, 32);
  const double m0 = s0 * (1.0 / 64.0);
  const double m1 = s1 * (1.0 / 64.0);
  float n0 = 0.f, n1 = 0.f;
#pragma unroll
  for (int s = 0; s < 32; ++s) {
    z0[s] = (float)((double)z0[s] - m0);
    z1[s] = (float)((double)z1[s] - m1);
    n0 = fmaf(z0[s], z0[s], n0);
    n1 = fmaf(z1[s], z1[s], n1);
  }
  n0 += __shfl_xor(n0, 32);
  n1 += __shfl_xor(n1, 32);
  // after the cross-lane combine below, lane l owns patch (col, block half)
  const float g66 = 66.f * kU / (1.f - 66.f * kU);
  const float g64 = 64.f * kU / (1.f - 64.f * kU);
  const float a = g66 * sqrt_beta * sqrtf((half ? n1 : n0) * (1.f + 64.f * kU));
  auto Ebound = [&](float c) {
    const float q = fmaxf(c - Lmin, 0.f);
    return kKappa * (g64 * q + 16.f * a * sqrtf(q) + 64.f * a * a + kU * (Labs + fabsf(c)));
  };

  float best_c = INFINITY, second_c = INFINITY, thr = INFINITY;
  int best_k = 0, nc = 0;
  float* my_v = cand_v + threadIdx.x * kCand;
  int* my_k = cand_k + threadIdx.x * kCand;

  const float4* up = Ut + lane;  // [K][2][8][64] float4
  float4 A[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) A[i] = up[i * 64];
  float q0 = 0.f, q1 = 0.f;
  const int nkk = 2 * K;
  for (int kk = 0; kk < nkk; ++kk) {
    const int nk = (kk + 1 < nkk) ? kk + 1 : kk;
    float4 B[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) B[i] = up[(size_t)nk * 512 + i * 64];
    f32x16 acc0 = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    f32x16 acc1 = acc0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      acc0 = mfma32(A[i].x, z0[4 * i + 0], acc0);
      acc1 = mfma32(A[i].x, z1[4 * i + 0], acc1);
      acc0 = mfma32(A[i].y, z0[4 * i + 1], acc0);
      acc1 = mfma32(A[i].y, z1[4 * i + 1], acc1);
      acc0 = mfma32(A[i].z, z0[4 * i + 2], acc0);
      acc1 = mfma32(A[i].z, z1[4 * i + 2], acc1);
      acc0 = mfma32(A[i].w, z0[4 * i + 3], acc0);
      acc1 = mfma32(A[i].w, z1[4 * i + 3], acc1);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      q0 = fmaf(acc0[i], acc0[i], q0);
      q1 = fmaf(acc1[i], acc1[i], q1);
    }
    if (kk & 1) {
      const int k = kk >> 1;
      // lanes < 32 finish patch block 0, lanes >= 32 patch block 1
      const float send = half ? q0 : q1;
      const float recv = __shfl_xor(send, 32);
      const float Q = (half ? q1 : q0) + recv;
      const float cost = L[k] + Q;
      if (cost < best_c) {
        second_c = best_c;
        best_c = cost;
        best_k = k;
        thr = cost + 3.f * Ebound(cost);
        int n2 = 0;
        const int nold = min(nc, kCand);
        for (int i = 0; i < nold; ++i) {
          const float v = my_v[i];
          if (v <= thr) {
            my_v[n2] = v;
            my_k[n2] = my_k[i];
            ++n2;
          }
        }
        nc = (nc > kCand) ? nc : n2;  // an overflow stays an overflow
      } else if (cost < second_c) {
        second_c = cost;
      }
      if (cost <= thr) {
        if (nc < kCand) {
          my_v[nc] = cost;
          my_k[nc] = k;
        }
        ++nc;
      }
      q0 = 0.f;
      q1 = 0.f;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) A[i] = B[i];
  }

  const int c = c0 + 32 * half + col;
  if (r < Hp && c < Wp) {
    const int idx = r * Wp + c;
    labels[idx] = best_k;
    if (best_out) best_out[idx] = best_c;
    if (second_out) second_out[idx] = second_c;
    const int unsure = !(best_c + Ebound(best_c) < second_c - Ebound(second_c));
    if (flags) flags[idx] = unsure;
    if (unsure && list) {
      // entry: patch, candidate count (kCand + 1 = all K), candidates packed
      // two per int in ascending k order of discovery
      int4 ent;
      ent.x = idx;
      int kk4[kCand];
      int n2 = 0;
      if (nc <= kCand) {
        for (int i = 0; i < nc; ++i)
          if (my_v[i] <= thr) kk4[n2++] = my_k[i];
      }
      for (int i = n2; i < kCand; ++i) kk4[i] = 0;
      ent.y = (nc <= kCand) ? n2 : kCand + 1;
      ent.z = kk4[0] | (kk4[1] << 16);
      ent.w = kk4[2] | (kk4[3] << 16);
      const int slot = atomicAdd(list_count, 1);
      list[slot] = ent;
    }
  }
}

hipError_t launch_estep_f32(const float* x, int H, int W, const float* Ut_t, const float* L32_t,
                            int K, double beta, int32_t* labels, float* best, float* second,
                            int32_t* flags, int32_t* list_count, int32_t* list, hipStream_t st) {
  // list holds int4 entries (see the kernel)
  const int Hp = H - 7, Wp = W - 7;
  dim3 grid((Wp + 63) / 64, (Hp + 3) / 4);
  hipLaunchKernelGGL(estep_f32_kernel, grid, dim3(256), 0, st, x, H, W,
                     reinterpret_cast<const float4*>(Ut_t), L32_t, K, (float)sqrt(beta), labels,
                     best, second, flags, list_count, reinterpret_cast<int4*>(list));
  return hipGetLastError();
}

}  // namespace fepll
