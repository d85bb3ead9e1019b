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
// A workgroup of 4 waves owns 128 patches (a quarter of a selection tile:
// 32 columns of each of its 4 patch rows, a wave per row), of one image or
// of any image of a planned batch, and streams the 23 weight slabs (one
// slab = one 32-row block of a layer, all depth steps, already in MFMA
// operand order) through double-buffered LDS, each slab fetched from L2
// into registers one slab ahead; one barrier per slab (after its LDS store)
// orders the buffers.  The kernel is latency-bound (neither its matrix
// cores, its vector ALUs nor its LDS saturate), so it is shaped for
// occupancy: one accumulation chain per slab, no products of the next slab
// held across an epilogue and one prefetched slab keep a wave within 168
// registers (the bf16 activations of 32 patches alone take 128), three
// workgroups per compute unit, three waves per SIMD.
//
// Top-m: each lane keeps the 8 largest ranking keys (logit, then lower
// class) of its 112 classes in sorted registers (an insertion is one max and
// seven independent medians of three), then merges with lane l ^ 32.
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
// trained with: branch-free, one exp2 and one reciprocal, the factor
// -log2(e) of the exponential folded into the two constants.
__device__ __forceinline__ float gelu(float a) {
  // -log2(e) 2 sqrt(2/pi) (a + 0.044715 a^3)
  const float t = a * fmaf(-0.10294324f, a * a, -2.3022082f);
  return a * __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(t));
}

// Ranking key of a logit: an order-preserving map of the float to uint32,
// its 10 low bits replaced by (1023 - class).  Keys compare like
// (logit, -class) with the logit truncated to 22 significant bits of its
// order (sign, exponent, 13 mantissa bits): ties within 2^-13 relative go to
// the lower class.  Every compare-exchange is then one max and one min.
__device__ __forceinline__ uint32_t rank_key(float v, int cls) {
  const uint32_t u = __float_as_uint(v);
  // negative: all bits flipped; otherwise the sign bit set
  const uint32_t o = u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
  return (o & ~1023u) | (uint32_t)(1023 - cls);
}
__device__ __forceinline__ int key_class(uint32_t k) { return 1023 - (int)(k & 1023u); }

// median of three (one v_med3_u32)
__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) {
  return max(min(a, b), min(max(a, b), c));
}

struct Top8 {
  uint32_t t[8];  // descending
  __device__ void init() {
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = 0u;
  }
  // x lands at the first position whose key it exceeds: position i > 0 then
  // holds the median of (old t[i - 1], old t[i], x), position 0 the maximum
  __device__ void insert(uint32_t x) {
    const uint32_t t0 = max(t[0], x);
#pragma unroll
    for (int i = 7; i >= 1; --i) t[i] = med3u(t[i - 1], t[i], x);
    t[0] = t0;
  }
};

constexpr int kWaves = 4;                // per workgroup, three workgroups per CU
constexpr int kThreads = 64 * kWaves;
constexpr int kWgPerTile = 16 / kWaves;  // a selection tile is 16 waves of 32 patches
constexpr int kSlabU4 = 16 * 64;  // uint4 of the largest slab (16 depth steps x 64 lanes)
constexpr int kSlabPer = kSlabU4 / kThreads;  // uint4 of a slab per thread
static_assert(kSlabU4 % kThreads == 0, "whole uint4 of a slab per thread");

// the accumulator of one 32-row block (units 32 nt + 8 (i >> 2) + 4 half +
// (i & 3) of the lane's column) started at the bias of its units: the
// matrix cores add the products to it
__device__ __forceinline__ f32x16 bias_init(const float* __restrict__ bias, int nt, int half) {
  f32x16 c;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const float4 b = *reinterpret_cast<const float4*>(bias + 32 * nt + 8 * g + 4 * half);
    c[4 * g] = b.x;
    c[4 * g + 1] = b.y;
    c[4 * g + 2] = b.z;
    c[4 * g + 3] = b.w;
  }
  return c;
}

// activation epilogue of one 32-row block (bias included): GELU, then
// re-pack as the two depth steps (2 nt, 2 nt + 1) of the next layer's B
// operand
__device__ __forceinline__ void hidden_epilogue(const f32x16& acc, int half, uint4& s0,
                                                uint4& s1) {
  float h[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) h[i] = gelu(acc[i]);
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
  u32x4 v[kSlabPer];
};
__device__ __forceinline__ int slab_offset(int q) {
  if (q < 8) return q * 5 * 64;
  if (q < 16) return 8 * 5 * 64 + (q - 8) * 16 * 64;
  return 8 * 5 * 64 + 8 * 16 * 64 + (q - 16) * 16 * 64;
}
__device__ __forceinline__ void fetch_slab(const uint4* __restrict__ Wb, int q, SlabRegs& p) {
  const u32x4* w = reinterpret_cast<const u32x4*>(Wb) + slab_offset(q) + threadIdx.x;
#pragma unroll
  for (int i = 0; i < kSlabPer; ++i) p.v[i] = w[i * kThreads];
}
// make slab q resident in the LDS buffer buf and start fetching slab q + 1
// into the same registers (past the last slab, the last one again: no
// branch, so every wait stays exact)
__device__ __forceinline__ void stage_slab(uint4* buf, SlabRegs& p, const uint4* __restrict__ Wb,
                                           int q, int nslab) {
  u32x4* d = reinterpret_cast<u32x4*>(buf) + threadIdx.x;
#pragma unroll
  for (int i = 0; i < kSlabPer; ++i) d[i * kThreads] = p.v[i];
  __syncthreads();
  fetch_slab(Wb, min(q + 1, nslab - 1), p);
}

}  // namespace

// Wb: all slabs back to back, uint4 in MFMA A-operand order:
//   layer 1: 8 slabs x 5 depth steps, layer 2: 8 x 16, layer 3: n3 x 16.
// bias: b1 (256) b2 (256) b3 (32 n3, -inf beyond K).
__global__ __launch_bounds__(kThreads, 3) void propose_bf16_kernel(ProposeArgs a) {
  __shared__ uint4 slab[2][kSlabU4];  // 32 KB
  __shared__ __align__(16) float bsh[2 * kHidden + 32 * 32];  // b1, b2, b3 (n3 <= 32 blocks of 32)
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int n3 = (a.K + 31) / 32;
  const int K = a.K, m = a.m;
  const uint4* __restrict__ Wb = reinterpret_cast<const uint4*>(a.Wb);
  // this workgroup's half selection tile
  const int item = blockIdx.x / kWgPerTile;
  const float* x = a.x;
  int H = a.H, W = a.W;
  float logsb = a.logsb;
  size_t np0 = 0;
  int tr, tc;
  if (a.d) {
    const int im = a.est_img[item];
    const ImgDesc d = a.d[im];
    H = d.H;
    W = d.W;
    x += d.px;
    np0 = (size_t)d.np;
    logsb = a.logsb_slot[d.slot0 + a.t];
    const int ntx = (W - 7 + kEstCols - 1) / kEstCols;
    const int lt = item - d.est0;
    tr = lt / ntx;
    tc = lt - tr * ntx;
  } else {
    const int ntx = (W - 7 + kEstCols - 1) / kEstCols;
    tr = item / ntx;
    tc = item - tr * ntx;
  }
  const int Hp = H - 7, Wp = W - 7;
  // wave gw of the tile's 16: patch row gw % 4, columns 32 (gw / 4) + 0..31
  const int gw = (blockIdx.x % kWgPerTile) * kWaves + wave;
  const int r = 4 * tr + (gw & 3);
  const int c = kEstCols * tc + 32 * (gw >> 2) + col;
  const int rr = min(r, Hp - 1), cc = min(c, Wp - 1);

  if (a.zero && blockIdx.x == 0)
    for (int i = threadIdx.x; i < a.n_zero; i += blockDim.x) a.zero[i] = 0;
  for (int i = threadIdx.x; i < 2 * kHidden + 32 * n3; i += blockDim.x) bsh[i] = a.bias[i];
  // (made visible by the first slab's barrier)

  // ---- layer-1 input: DC-removed patch / 128 and log sigma_beta.  The
  // mean is summed in float64 (exact in any order whenever the patch's pixel
  // magnitudes lie within 2^23 of each other) and each difference is
  // rounded once to float32, as in the selection kernels; lane half h holds
  // rows 2 t + h.
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
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float q[8];
#pragma unroll
      for (int e = 0; e < 8; ++e)
        q[e] = (float)((double)fresh(v[t][e]) - mean) * (1.f / kScaleIn);
      xb[t] = make_uint4(pack2(q[0], q[1]), pack2(q[2], q[3]), pack2(q[4], q[5]),
                         pack2(q[6], q[7]));
    }
    xb[4] = make_uint4(half ? 0u : bf16_rne(logsb), 0u, 0u, 0u);
  }

  // the next slab in flight in registers
  const int nslab = 16 + n3;
  SlabRegs pre;
  fetch_slab(Wb, 0, pre);
  uint4 h1[16], h2[16];
  // Per slab: stage it, its matrix products, its epilogue (the activations
  // or the top-m of its block); the other waves of the SIMD fill the gaps.
  // (The buffer a slab is staged into last held the slab two before, whose
  // operands every wave read before the barrier of the slab in between.)
  auto mm1 = [&](int q) __attribute__((always_inline)) {
    stage_slab(slab[q & 1], pre, Wb, q, nslab);
    const uint4* A = slab[q & 1] + lane;
    f32x16 acc = bias_init(bsh, q, half);
#pragma unroll
    for (int s = 0; s < 5; ++s) acc = mfma_bf16(A[s * 64], xb[s], acc);
    return acc;
  };
  // layers 2 and 3: one accumulation chain started at the bias
  auto mm23 = [&](int q, const float* bias, int nt, const uint4* hin)
      __attribute__((always_inline)) {
    stage_slab(slab[q & 1], pre, Wb, q, nslab);
    const uint4* A = slab[q & 1] + lane;
    f32x16 acc = bias_init(bias, nt, half);
#pragma unroll
    for (int s = 0; s < 16; ++s) acc = mfma_bf16(A[s * 64], hin[s], acc);
    return acc;
  };
  {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      f32x16 acc = mm1(q);
      hidden_epilogue(acc, half, h1[2 * q], h1[2 * q + 1]);
    }
  }
  {
#pragma unroll
    for (int q = 8; q < 16; ++q) {
      f32x16 acc = mm23(q, bsh + kHidden, q - 8, h1);
      hidden_epilogue(acc, half, h2[2 * (q - 8)], h2[2 * (q - 8) + 1]);
    }
  }
  Top8 top;
  top.init();
  const float* b3 = bsh + 2 * kHidden;
  auto top_epilogue = [&](int q, const f32x16& acc) __attribute__((always_inline)) {
    const int nt = q - 16;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      // a group of 8 classes wholly past K is skipped (a wave-uniform
      // branch); in a group that straddles K the classes past it have the
      // logit -inf from their bias, below every finite key
      if (32 * nt + 8 * g >= K) break;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int cls = 32 * nt + 8 * g + 4 * half + e;
        top.insert(rank_key(acc[4 * g + e], cls));
      }
    }
  };
  // layer 3, two slabs per pass
  {
    for (int q = 16; q < nslab; q += 2) {
      f32x16 acc = mm23(q, b3, q - 16, h2);
      top_epilogue(q, acc);
      if (q + 1 < nslab) {
        acc = mm23(q + 1, b3, q + 1 - 16, h2);
        top_epilogue(q + 1, acc);
      }
    }
  }
  // merge the two halves' lists
  // take the partner's whole list before inserting, so no key comes back twice
  uint32_t other[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) other[i] = __shfl_xor(top.t[i], 32);
#pragma unroll
  for (int i = 0; i < 8; ++i) top.insert(other[i]);
  if (!half && r < Hp && c < Wp) {
    const size_t idx = np0 + (size_t)r * Wp + c;
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t a = (2 * i < m) ? (uint32_t)key_class(top.t[2 * i]) : 0xffffu;
      const uint32_t b = (2 * i + 1 < m) ? (uint32_t)key_class(top.t[2 * i + 1]) : 0xffffu;
      w[i] = a | (b << 16);
    }
    reinterpret_cast<uint4*>(a.cand)[idx] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

hipError_t launch_propose(const ProposeArgs& a, hipStream_t st) {
  int n_est = a.n_est;
  if (!a.d) n_est = ((a.W - 7 + kEstCols - 1) / kEstCols) * ((a.H - 7 + 3) / 4);
  if (n_est < 1) return hipSuccess;
  hipLaunchKernelGGL(propose_bf16_kernel, dim3((unsigned)(kWgPerTile * n_est)), dim3(kThreads), 0,
                     st, a);
  return hipGetLastError();
}

}  // namespace fepll
