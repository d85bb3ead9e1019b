// Proposal network inference (bfloat16 MFMA, float32 accumulation) fused
// with the top-m selection of its logits.
//
// The three layers run in transposed form, H^t = W X^t: hidden units (or
// classes) on the MFMA rows, 32 patches on the columns.  The 32x32 output of
// v_mfma_f32_32x32x16_bf16 leaves lane l with patch (l & 31) and units
// 8 g + 4 (l >> 5) + e (g, e = 0..3); the next layer's B operand needs units
// 16 s + 8 (l >> 5) + 0..7, so one v_permlane32_swap between lanes l and
// l ^ 32 per group pair re-packs every activation in registers: no
// activation ever leaves the wave.  The layer-1 B operand is the patch itself (one 8-pixel
// patch row per depth step, as in the selection kernels) plus the
// log sigma_beta feature.
//
// A workgroup of 8 waves owns 256 patches (8 patch rows x 32 columns) and
// streams the 23 weight slabs (one slab = one 32-row block of a layer, all
// depth steps, already in MFMA operand order) through double-buffered LDS,
// so each weight byte read from L2 serves 256 patches; each slab is fetched
// from L2 two slabs ahead, and one barrier per slab (after its LDS store)
// orders the buffers.
//
// Top-m: each lane keeps the 8 largest ranking keys (logit, then lower
// class) of its 112 classes in sorted registers, then merges with lane
// l ^ 32.
#include "common.h"
#include "mlp.h"
#include "propose.h"

namespace fepll {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

__device__ __forceinline__ uint32_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
// two floats to bfloat16 (nearest, ties to even), a in the low half: one
// v_cvt_pk_bf16_f32, the same rounding as bf16_rne for finite values
__device__ __forceinline__ uint32_t pack2(float a, float b) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  typedef float f32x2_t __attribute__((ext_vector_type(2)));
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}
__device__ __forceinline__ f32x16 mfma_bf16(uint4 a, uint4 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
// GELU in the tanh form of Hendrycks & Gimpel (2016),
// x * sigmoid(2 sqrt(2/pi) (x + 0.044715 x^3)), the form the network is
// trained with: branch-free, one exp2 and one reciprocal.
__device__ __forceinline__ float gelu(float a) {
  const float t = a * fmaf(0.0713548162726f, a * a, 1.59576912161f);  // 2 sqrt(2/pi) (a + 0.044715 a^3)
  const float e = __builtin_amdgcn_exp2f(-t * 1.44269504089f);
  return a * __builtin_amdgcn_rcpf(1.f + e);
}

// Ranking key of a logit: an order-preserving map of the float to uint32,
// its 10 low bits replaced by (1023 - class).  Keys compare like
// (logit, -class) with the logit truncated to 22 significant bits of its
// order (sign, exponent, 13 mantissa bits): ties within 2^-13 relative go to
// the lower class.  Every compare-exchange is then one max and one min.
__device__ __forceinline__ uint32_t rank_key(float v, int cls) {
  const uint32_t u = __float_as_uint(v);
  const uint32_t o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return (o & ~1023u) | (uint32_t)(1023 - cls);
}
__device__ __forceinline__ int key_class(uint32_t k) { return 1023 - (int)(k & 1023u); }

struct Top8 {
  uint32_t t[8];  // descending
  __device__ void init() {
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = 0u;
  }
  __device__ void insert(uint32_t x) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t hi = max(t[i], x);
      x = min(t[i], x);
      t[i] = hi;
    }
  }
};

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kSlabU4 = 16 * 64;  // uint4 of the largest slab (16 depth steps x 64 lanes)
static_assert(kSlabU4 == 2 * kThreads, "two uint4 of a slab per thread");

// activation epilogue of one 32-row block: bias + GELU, then re-pack as
// the two depth steps (2 nt, 2 nt + 1) of the next layer's B operand
__device__ __forceinline__ void hidden_epilogue(const f32x16& acc, const float* __restrict__ bias,
                                                int nt, int half, uint4& s0, uint4& s1) {
  float h[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int unit = 32 * nt + 8 * (i >> 2) + 4 * half + (i & 3);
    h[i] = gelu(acc[i] + bias[unit]);
  }
  float lo[8], hi[8];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    // groups 0/1 -> depth step 2 nt, groups 2/3 -> depth step 2 nt + 1.
    // v_permlane32_swap(a0, a1) leaves the lower half with (own a0,
    // partner's a0) and the upper half with (partner's a1, own a1): units
    // 8 g + 0..3 and 8 g + 4..7 of the lane's column, in order.
    const auto p01 = __builtin_amdgcn_permlane32_swap(__float_as_uint(h[e]),
                                                      __float_as_uint(h[4 + e]), false, false);
    const auto p23 = __builtin_amdgcn_permlane32_swap(__float_as_uint(h[8 + e]),
                                                      __float_as_uint(h[12 + e]), false, false);
    lo[e] = __uint_as_float(p01[0]);
    lo[4 + e] = __uint_as_float(p01[1]);
    hi[e] = __uint_as_float(p23[0]);
    hi[4 + e] = __uint_as_float(p23[1]);
  }
  uint32_t w[8];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    w[i] = pack2(lo[2 * i], lo[2 * i + 1]);
    w[4 + i] = pack2(hi[2 * i], hi[2 * i + 1]);
    // keep the packed words: left alone, the compiler holds the floats and
    // converts them again at every use (twice the registers, 64 more
    // conversions per slab)
    asm volatile("" : "+v"(w[i]));
    asm volatile("" : "+v"(w[4 + i]));
  }
  s0 = make_uint4(w[0], w[1], w[2], w[3]);
  s1 = make_uint4(w[4], w[5], w[6], w[7]);
}

// Weight-slab pipeline.  Slab q's offset (uint4) in Wb: 8 layer-1 slabs of
// 5 x 64, then 8 layer-2 and n3 layer-3 slabs of 16 x 64.  Every slab moves
// as kSlabU4 uint4 (two per thread), so the number of loads in flight is
// fixed and each wait is for the older slab only; a layer-1 slab carries
// the head of the next slab along, unused and in bounds (larger slabs
// follow the last one).
// (native vectors: copies of HIP's uint4 struct lower to memcpy, which keeps
// the pair in private memory)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
struct SlabRegs {
  u32x4 a, b;
};
__device__ __forceinline__ int slab_offset(int q) {
  if (q < 8) return q * 5 * 64;
  if (q < 16) return 8 * 5 * 64 + (q - 8) * 16 * 64;
  return 8 * 5 * 64 + 8 * 16 * 64 + (q - 16) * 16 * 64;
}
__device__ __forceinline__ void fetch_slab(const uint4* __restrict__ Wb, int q, SlabRegs& p) {
  const u32x4* w = reinterpret_cast<const u32x4*>(Wb) + slab_offset(q) + threadIdx.x;
  p.a = w[0];
  p.b = w[kThreads];
}
// make slab q resident in the LDS buffer buf and start fetching slab q + 2
// into the same registers (past the last slab, the last one again: no
// branch, so every wait stays exact)
__device__ __forceinline__ void stage_slab(uint4* buf, SlabRegs& p, const uint4* __restrict__ Wb,
                                           int q, int nslab) {
  u32x4* d = reinterpret_cast<u32x4*>(buf) + threadIdx.x;
  d[0] = p.a;
  d[kThreads] = p.b;
  __syncthreads();
  fetch_slab(Wb, min(q + 2, nslab - 1), p);
}

}  // namespace

// Wb: all slabs back to back, uint4 in MFMA A-operand order:
//   layer 1: 8 slabs x 5 depth steps, layer 2: 8 x 16, layer 3: n3 x 16.
// bias: b1 (256) b2 (256) b3 (32 n3, -inf beyond K).
// zop / znz: NULL, or Np x 8 uint4 and Np floats receiving the selection
// operand of every patch and its squared norm (see the input stage).
__global__ __launch_bounds__(kThreads, 1) void propose_bf16_kernel(
    const float* __restrict__ x, int H, int W, float logsb, const uint4* __restrict__ Wb,
    const float* __restrict__ bias, int n3, int K, int m, uint16_t* __restrict__ cand,
    uint4* __restrict__ zop, float* __restrict__ znz) {
  __shared__ uint4 slab[2][kSlabU4];  // 32 KB
  __shared__ float bsh[2 * kHidden + 32 * 32];  // b1, b2, b3 (n3 <= 32 blocks of 32)
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int Hp = H - 7, Wp = W - 7;
  const int r = blockIdx.y * kWaves + wave;
  const int c = blockIdx.x * 32 + col;
  const int rr = min(r, Hp - 1), cc = min(c, Wp - 1);

  for (int i = threadIdx.x; i < 2 * kHidden + 32 * n3; i += blockDim.x) bsh[i] = bias[i];
  // (made visible by the first slab's barrier)

  // ---- layer-1 input: DC-removed patch / 128 and log sigma_beta.  The
  // mean is summed in float64 (exact in any order whenever the patch's pixel
  // magnitudes lie within 2^23 of each other) and each difference is
  // rounded once to float32, as in the selection kernels; lane half h holds
  // rows 2 t + h.  With zop, the patch is also written as the bfloat16
  // selection operand (row dy at uint4 dy of the patch's 128 bytes) with its
  // float32 squared norm, summed in the order of the bfloat16 selection
  // (rows g and 4 + g in order into q_g, then (q_0 + q_1) + (q_2 + q_3)):
  // what the rescoring of the candidates reads, bit for bit the full
  // search's operands.
  uint4 xb[5];
  {
    float v[4][8];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float* row = x + (size_t)(rr + 2 * t + half) * W + cc;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[t][e] = row[e];
    }
    double sd = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int e = 0; e < 8; ++e) sd += (double)v[t][e];
    sd += __shfl_xor(sd, 32);
    const double mean = sd * (1.0 / 64.0);
    float d[4][8];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int e = 0; e < 8; ++e) d[t][e] = (float)((double)v[t][e] - mean);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float q[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) q[e] = d[t][e] * (1.f / kScaleIn);
      xb[t] = make_uint4(pack2(q[0], q[1]), pack2(q[2], q[3]), pack2(q[4], q[5]),
                         pack2(q[6], q[7]));
    }
    xb[4] = make_uint4(half ? 0u : bf16_rne(logsb), 0u, 0u, 0u);
    if (zop) {  // (uniform: the shuffles see every lane)
      const bool ok = r < Hp && c < Wp;
      const size_t idx = (size_t)rr * Wp + cc;
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (ok)
          zop[idx * 8 + 2 * t + half] =
              make_uint4(pack2(d[t][0], d[t][1]), pack2(d[t][2], d[t][3]),
                         pack2(d[t][4], d[t][5]), pack2(d[t][6], d[t][7]));
      float qa = 0.f, qb = 0.f;  // rows h then 4 + h; rows 2 + h then 6 + h
#pragma unroll
      for (int e = 0; e < 8; ++e) qa = fmaf(d[0][e], d[0][e], qa);
#pragma unroll
      for (int e = 0; e < 8; ++e) qa = fmaf(d[2][e], d[2][e], qa);
#pragma unroll
      for (int e = 0; e < 8; ++e) qb = fmaf(d[1][e], d[1][e], qb);
#pragma unroll
      for (int e = 0; e < 8; ++e) qb = fmaf(d[3][e], d[3][e], qb);
      const float oa = __shfl_xor(qa, 32), ob = __shfl_xor(qb, 32);
      if (ok && !half) znz[idx] = (qa + oa) + (qb + ob);
    }
  }

  // slabs q + 1 and q + 2 in flight in registers (preA holds the even
  // slabs, preB the odd ones; each call below names its pair at compile
  // time, so both stay in registers)
  const int nslab = 16 + n3;
  SlabRegs preA, preB;
  fetch_slab(Wb, 0, preA);
  fetch_slab(Wb, 1, preB);
  uint4 h1[16], h2[16];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (q & 1)
      stage_slab(slab[1], preB, Wb, q, nslab);
    else
      stage_slab(slab[0], preA, Wb, q, nslab);
    const uint4* A = slab[q & 1] + lane;
    f32x16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 5; ++s) acc = mfma_bf16(A[s * 64], xb[s], acc);
    hidden_epilogue(acc, bsh, q, half, h1[2 * q], h1[2 * q + 1]);
    // (no barrier here: slab q + 1 goes to the other buffer, and slab q + 2
    // overwrites this one only after the next stage's barrier, which every
    // wave reaches after its last read of this slab -- the waves of a SIMD
    // may drift by up to one slab and overlap one's epilogue with the
    // other's matrix products)
  }
#pragma unroll
  for (int q = 8; q < 16; ++q) {
    if (q & 1)
      stage_slab(slab[1], preB, Wb, q, nslab);
    else
      stage_slab(slab[0], preA, Wb, q, nslab);
    const uint4* A = slab[q & 1] + lane;
    // two independent accumulation chains (even / odd depth steps)
    f32x16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    f32x16 acc2 = acc;
#pragma unroll
    for (int s = 0; s < 16; s += 2) {
      acc = mfma_bf16(A[s * 64], h1[s], acc);
      acc2 = mfma_bf16(A[(s + 1) * 64], h1[s + 1], acc2);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] += acc2[i];
    hidden_epilogue(acc, bsh + kHidden, q - 8, half, h2[2 * (q - 8)], h2[2 * (q - 8) + 1]);
  }
  Top8 top;
  top.init();
  const float* b3 = bsh + 2 * kHidden;
  auto layer3 = [&](int q, SlabRegs& pre) __attribute__((always_inline)) {
    stage_slab(slab[q & 1], pre, Wb, q, nslab);
    const uint4* A = slab[q & 1] + lane;
    f32x16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    f32x16 acc2 = acc;
#pragma unroll
    for (int s = 0; s < 16; s += 2) {
      acc = mfma_bf16(A[s * 64], h2[s], acc);
      acc2 = mfma_bf16(A[(s + 1) * 64], h2[s + 1], acc2);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] += acc2[i];
    const int nt = q - 16;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int cls = 32 * nt + 8 * (i >> 2) + 4 * half + (i & 3);
      const float v = acc[i] + b3[cls];
      const uint32_t key = rank_key(v, cls);
      top.insert(cls < K ? key : 0u);  // (a select: classes past K rank last)
    }
  };
  // layer-3 slabs in pairs: even ones in preA, odd ones in preB
  for (int q = 16; q < nslab; q += 2) {
    layer3(q, preA);
    if (q + 1 < nslab) layer3(q + 1, preB);
  }
  // merge the two halves' lists
  // take the partner's whole list before inserting, so no key comes back twice
  uint32_t other[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) other[i] = __shfl_xor(top.t[i], 32);
#pragma unroll
  for (int i = 0; i < 8; ++i) top.insert(other[i]);
  if (!half && r < Hp && c < Wp) {
    const size_t idx = (size_t)r * Wp + c;
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t a = (2 * i < m) ? (uint32_t)key_class(top.t[2 * i]) : 0xffffu;
      const uint32_t b = (2 * i + 1 < m) ? (uint32_t)key_class(top.t[2 * i + 1]) : 0xffffu;
      w[i] = a | (b << 16);
    }
    reinterpret_cast<uint4*>(cand)[idx] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

hipError_t launch_propose_bf16(const float* x, int H, int W, double beta, const uint16_t* Wb,
                               const float* bias, int K, int m, uint16_t* cand, uint16_t* zop,
                               float* znz, hipStream_t st) {
  const int Hp = H - 7, Wp = W - 7;
  const int n3 = (K + 31) / 32;
  dim3 grid((Wp + 31) / 32, (Hp + kWaves - 1) / kWaves);
  hipLaunchKernelGGL(propose_bf16_kernel, grid, dim3(kThreads), 0, st, x, H, W,
                     (float)(-0.5 * log(beta)), reinterpret_cast<const uint4*>(Wb), bias, n3, K,
                     m, cand, reinterpret_cast<uint4*>(zop), znz);
  return hipGetLastError();
}

}  // namespace fepll
