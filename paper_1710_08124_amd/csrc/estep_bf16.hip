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
// patches (four blocks of 32) as B operands for its whole component loop;
// per component it issues 2 (eigen blocks) x 4 (depth steps) x 4 (patch
// blocks) MFMAs and 128 float32 FMAs of squares.
//
// Three modes share the kernel:
//  * spatial, all K: a wave takes 128 consecutive patches of one row;
//  * spatial, candidates: each patch carries the components proposed for it;
//    the wave scores the union of its patches' candidates (sorted, built in
//    LDS) and each patch keeps the best and second best of its own
//    candidates -- the exact rescoring of the proposal.  A patch whose half
//    gap (in nats) between the two is below the margin is appended to a
//    fallback list;
//  * list, all K: the fallback patches, 128 list entries per wave, with a
//    device-side list length (fixed grid, waves stride over the list and
//    exit past its end).
#include "common.h"
#include "propose.h"

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
__device__ __forceinline__ bool has(const uint4& c, int k) {
  const uint32_t w[4] = {c.x, c.y, c.z, c.w};
  bool r = false;
#pragma unroll
  for (int i = 0; i < 4; ++i) r |= ((int)(w[i] & 0xffffu) == k) | ((int)(w[i] >> 16) == k);
  return r;
}

// DC-removed bfloat16 B operands of one 32-patch block; (r, c) top-left.
__device__ __forceinline__ void load_patch(const float* __restrict__ x, int W, int r, int c,
                                           int half, uint4 zb[4]) {
  float v[4][8];
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float* row = x + (size_t)(r + 2 * t + half) * W + c;
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
    zb[t] = make_uint4(pack2(d[0], d[1]), pack2(d[2], d[3]), pack2(d[4], d[5]),
                       pack2(d[6], d[7]));
  }
}

// Squared norms of the 4 x 32 patches for component k; returns the two
// costs this lane owns (blocks half and 2 + half).
__device__ __forceinline__ void score(const uint4* __restrict__ up, int k, const uint4 zb[CB][4],
                                      float Lk, int half, float& cA, float& cB) {
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
    __builtin_amdgcn_sched_barrier(0);
  }
  // lanes < 32 finish blocks 0 and 2, lanes >= 32 blocks 1 and 3
  const float r0 = __shfl_xor(half ? q[0] : q[1], 32);
  const float r1 = __shfl_xor(half ? q[2] : q[3], 32);
  cA = Lk + ((half ? q[1] : q[0]) + r0);
  cB = Lk + ((half ? q[3] : q[2]) + r1);
}
}  // namespace

template <int MODE>
__global__ __launch_bounds__(256, 2) void estep_bf16_kernel(BF16Args a) {
  __shared__ uint32_t bm[4][32];
  __shared__ uint16_t ul[4][kMaxK];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int Hp = a.H - 7, Wp = a.W - 7;
  const uint4* up = reinterpret_cast<const uint4*>(a.Ub) + lane;  // [K][2][4][64] uint4

  const int nlist = (MODE == kModeListFull) ? *a.list_count : 0;
  const int nwaves = gridDim.x * gridDim.y * 4;
  int chunk = (blockIdx.y * gridDim.x + blockIdx.x) * 4 + wave;
  for (;;) {
    // ---- this wave's 128 patches
    int idx[CB];
    bool valid[CB];
    if (MODE == kModeListFull) {
      if (chunk * 128 >= nlist) break;
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int e = chunk * 128 + 32 * cb + col;
        valid[cb] = e < nlist;
        idx[cb] = a.list[valid[cb] ? e : chunk * 128];
      }
    } else {
      const int r = blockIdx.y * 4 + wave;
      const int c0 = blockIdx.x * (32 * CB);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int c = c0 + 32 * cb + col;
        valid[cb] = (r < Hp) && (c < Wp);
        idx[cb] = min(r, Hp - 1) * Wp + min(c, Wp - 1);
      }
    }
    uint4 zb[CB][4];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int pr = idx[cb] / Wp;
      load_patch(a.x, a.W, pr, idx[cb] - pr * Wp, half, zb[cb]);
    }
    // lane's own patches: blocks half and 2 + half
    const int iA = half ? idx[1] : idx[0];
    const int iB = half ? idx[3] : idx[2];
    const bool vA = half ? valid[1] : valid[0];
    const bool vB = half ? valid[3] : valid[2];

    float bA = INFINITY, sA = INFINITY, bB = INFINITY, sB = INFINITY;
    int kA = 0, kB = 0;
    if (MODE == kModeSpatialCand) {
      const uint4 candA = a.cand[iA];
      const uint4 candB = a.cand[iB];
      // union of the candidates of the wave's valid patches, ascending
      if (lane < 32) bm[wave][lane] = 0u;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      const uint32_t cw[8] = {candA.x, candA.y, candA.z, candA.w,
                              candB.x, candB.y, candB.z, candB.w};
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const bool own = (i < 4) ? vA : vB;
        const int k0 = (int)(cw[i] & 0xffffu), k1 = (int)(cw[i] >> 16);
        if (own && k0 < a.K) atomicOr(&bm[wave][k0 >> 5], 1u << (k0 & 31));
        if (own && k1 < a.K) atomicOr(&bm[wave][k1 >> 5], 1u << (k1 & 31));
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      const uint32_t word = (lane < 32) ? bm[wave][lane] : 0u;
      const int cnt = __popc(word);
      int incl = cnt;
#pragma unroll
      for (int d = 1; d < 32; d <<= 1) {
        const int o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
      }
      const int nu = __shfl(incl, 31);
      int pos = incl - cnt;
      uint32_t wv = word;
      while (wv) {
        const int b = __ffs(wv) - 1;
        ul[wave][pos++] = (uint16_t)(32 * lane + b);
        wv &= wv - 1u;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      for (int u = 0; u < nu; ++u) {
        const int k = ul[wave][u];
        float cA, cB;
        score(up, k, zb, a.L[k], half, cA, cB);
        if (has(candA, k)) keep_best(cA, k, bA, sA, kA);
        if (has(candB, k)) keep_best(cB, k, bB, sB, kB);
      }
    } else {
      for (int k = 0; k < a.K; ++k) {
        float cA, cB;
        score(up, k, zb, a.L[k], half, cA, cB);
        keep_best(cA, k, bA, sA, kA);
        keep_best(cB, k, bB, sB, kB);
      }
    }
    // ---- outputs
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const bool v = p ? vB : vA;
      if (!v) continue;
      const int i = p ? iB : iA;
      const float b = p ? bB : bA, s = p ? sB : sA;
      a.labels[i] = p ? kB : kA;
      if (a.best) a.best[i] = b;
      if (a.second) a.second[i] = s;
      if (MODE == kModeSpatialCand) {
        const float gap = (s < INFINITY) ? 0.5f * (s - b) : -INFINITY;
        if (!(gap >= a.margin)) {
          const int slot = atomicAdd(a.fb_count, 1);
          a.fb_list[slot] = i;
        }
      }
    }
    if (MODE != kModeListFull) break;
    chunk += nwaves;
  }
}

hipError_t launch_estep_bf16_mode(int mode, const BF16Args& args, hipStream_t st) {
  const int Hp = args.H - 7, Wp = args.W - 7;
  if (mode == kModeListFull) {
    const int Np = Hp * Wp;
    int blocks = (Np + 511) / 512;
    if (blocks > 512) blocks = 512;
    hipLaunchKernelGGL(estep_bf16_kernel<kModeListFull>, dim3(blocks), dim3(256), 0, st, args);
    return hipGetLastError();
  }
  dim3 grid((Wp + 32 * CB - 1) / (32 * CB), (Hp + 3) / 4);
  if (mode == kModeSpatialCand)
    hipLaunchKernelGGL(estep_bf16_kernel<kModeSpatialCand>, grid, dim3(256), 0, st, args);
  else
    hipLaunchKernelGGL(estep_bf16_kernel<kModeSpatialFull>, grid, dim3(256), 0, st, args);
  return hipGetLastError();
}

hipError_t launch_estep_bf16(const float* x, int H, int W, const uint16_t* Ub_t,
                             const float* L32_t, int K, int32_t* labels, float* best,
                             float* second, hipStream_t st) {
  BF16Args a{};
  a.x = x;
  a.H = H;
  a.W = W;
  a.Ub = Ub_t;
  a.L = L32_t;
  a.K = K;
  a.labels = labels;
  a.best = best;
  a.second = second;
  return launch_estep_bf16_mode(kModeSpatialFull, a, st);
}

}  // namespace fepll
