// Gaussian selection with 8-bit float projections (Alg. 1 patch extraction
// + Gaussian selection, eigenspace form of Sec. 2.1), the lowest-precision
// mode: the DC-removed patches and the scaled eigenbases
// Ut_k = U_k diag(nu_k)^-1/2 are rounded to e4m3 (OCP, largest finite 448)
// after a power-of-two scale per component (Ut_k) and per patch (z~) that
// brings their largest magnitude into (224, 448].  The matrix cores apply
// both scales (v_mfma_scale_f32_32x32x64_f8f6f4 takes one 8-bit exponent per
// operand row and column), so the accumulators hold c = Ut_k^t z~ in the
// original units; squared norms, L_k and the argmin are float32, as in the
// bfloat16 mode.  Labels are an approximation whose agreement with the
// exact selection is measured.
//
// One 32x32x64 MFMA multiplies 32 eigen-directions by 32 patches over all 64
// pixels: lane l supplies the 32 bytes of pixels 32 (l >> 5) + b (b = 0..31,
// patch rows 4 (l >> 5) .. 4 (l >> 5) + 3) of patch l & 31, and the A operand
// the same pixels of direction 32 rb + (l & 31).  A wave holds 128 patches
// (four blocks of 32) for its whole component loop; per component it issues
// 2 (eigen blocks) x 4 (patch blocks) MFMAs and 128 float32 FMAs of squares,
// then one exchange between lane halves leaves every lane owning 2 patches.
// Three workgroups per compute unit (3 waves per SIMD): the squares of one
// wave are summed while the matrix core runs another wave's MFMAs.
// The per-component operand (4 KB) is staged through double-buffered LDS
// shared by the workgroup's 4 waves.  The launch is persistent over the
// selection tiles of a batch of images, each with its own beta.
#include <algorithm>

#include "common.h"
#include "wave_ops.h"

namespace fepll {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

namespace {
constexpr int PB = 4;  // blocks of 32 patches per wave

// Power-of-two scale of a block whose largest magnitude is mx: the smallest
// e with mx * 2^-e <= 448, returned with the block's E8M0 code e + 127.
__device__ __forceinline__ int fp8_exponent(float mx) {
  if (!(mx > 0.f)) return 0;
  int ex;
  const float f = frexpf(mx, &ex);  // mx = f 2^ex, f in [0.5, 1)
  int e = (f <= 0.875f) ? ex - 9 : ex - 8;
  return max(e, -127);
}

// e4m3 B operand (32 bytes) and E8M0 scale of a patch from the lane's 32
// pixels v (rows 4 h .. 4 h + 3 of it, row-major): the mean is a float64
// sum of the 64 pixels (exact for any order whenever the patch's pixel
// magnitudes lie within 2^23 of each other), each difference rounded once to
// float32.  With NZ, nz receives the float32 squared norm of the (unrounded)
// DC-removed patch, the same in both lanes of its column.
template <bool NZ>
__device__ __forceinline__ void quantize_patch8(float (&v)[32], i32x8& zq, int& code, float& nz) {
  double s = (double)v[0];
#pragma unroll
  for (int i = 1; i < 32; ++i) s += (double)v[i];
  s += __shfl_xor(s, 32);
  const double m = s * (1.0 / 64.0);
  float mx = 0.f, q2 = 0.f;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    v[i] = (float)((double)fresh(v[i]) - m);
    mx = fmaxf(mx, fabsf(v[i]));
    if (NZ) q2 = fmaf(v[i], v[i], q2);
  }
  mx = fmaxf(mx, __shfl_xor(mx, 32));
  if (NZ) nz = q2 + __shfl_xor(q2, 32);
  const int e = fp8_exponent(mx);
  code = e + 127;
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    int p = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(v[4 * w], -e), ldexpf(v[4 * w + 1], -e), 0,
                                            false);
    p = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(v[4 * w + 2], -e), ldexpf(v[4 * w + 3], -e), p,
                                        true);
    zq[w] = p;
  }
}

// the same for the patch at (r, c) of x, lane half h, read from the image
template <bool NZ>
__device__ __forceinline__ void load_patch8(const float* __restrict__ x, int W, int r, int c,
                                            int h, i32x8& zq, int& code, float& nz) {
  float v[32];
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const float* row = x + (size_t)(r + 4 * h + rr) * W + c;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[8 * rr + e] = row[e];
  }
  quantize_patch8<NZ>(v, zq, code, nz);
}
}  // namespace

// FLAT: the flat-tail form (Sec. 3.1) -- only the eigen blocks of 32 that
// hold a component's kept directions are staged and projected on, and the
// cost is L_k + Pk |z~|^2 minus their squared projections (the operand's
// columns carry sqrt(1/nu_P - 1/nu_j), Pk = 1/nu_P); a component without a
// tail (rk = 64) takes the plain form.
template <bool FLAT>
__global__ __launch_bounds__(256, 3) void estep_fp8_kernel(
    const ImgDesc* __restrict__ dsc, const int32_t* __restrict__ est_img, int n_est, int t,
    const float* __restrict__ xb, const uint4* __restrict__ Uf_all,
    const int32_t* __restrict__ Ue_all, const float* __restrict__ L_all,
    const int32_t* __restrict__ rkt, const float* __restrict__ P_all, int K,
    int32_t* __restrict__ labels_b, float* __restrict__ best_b, float* __restrict__ second_b) {
  __shared__ uint4 Ash[2][256];
  __shared__ int Esh[kMaxK];
  __shared__ float Lsh[kMaxK];
  __shared__ float Psh[FLAT ? kMaxK : 1];
  __shared__ int Rsh[FLAT ? kMaxK : 1];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int h = lane >> 5;
  const int col = lane & 31;

  // persistent: each workgroup loops over selection tiles (4 patch rows x
  // 128 columns) of the batch; the loop is workgroup-uniform
  for (int item = blockIdx.x; item < n_est; item += gridDim.x) {
    const ImgDesc d = dsc[est_img[item]];
    const int W = d.W, Hp = d.H - 7, Wp = d.W - 7;
    const float* x = xb + d.px;
    const size_t slot = (size_t)(d.slot0 + t);
    const uint4* Uf = Uf_all + slot * K * (kTileStride / 16);
    const int32_t* Ue = Ue_all + slot * K;
    const float* L = L_all + slot * K;
    const float* Pk_t = FLAT ? P_all + slot * K : nullptr;
    // this lane's patch of block pb: index (r Wp + c) of the image and
    // whether it is a real patch (tile edge / list end otherwise)
    int pidx[PB];
    bool pval[PB];
    {
      const int ntx = (Wp + kEstCols - 1) / kEstCols;
      const int lt = item - d.est0;
      const int tr = lt / ntx, tc = lt - tr * ntx;
      const int r = tr * 4 + wave;
      const int c0 = tc * (32 * PB);
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
        const int c = c0 + 32 * pb + col;
        pval[pb] = r < Hp && c < Wp;
        pidx[pb] = min(r, Hp - 1) * Wp + min(c, Wp - 1);
      }
    }
    i32x8 zq[PB];
    int zc[PB];
    float nzA = 0.f, nzB = 0.f;  // own patches: blocks h and 2 + h
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      float nz = 0.f;
      const int pr = pidx[pb] / Wp;
      load_patch8<FLAT>(x, W, pr, pidx[pb] - pr * Wp, h, zq[pb], zc[pb], nz);
      if (FLAT) {
        nzA = (pb == h) ? nz : nzA;
        nzB = (pb == 2 + h) ? nz : nzB;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // the component scales and L_k of the tile's beta sit in LDS, read with
    // the operand (no scalar-memory wait in the component loop)
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
      Esh[k] = Ue[k];
      Lsh[k] = L[k];
      if (FLAT) {
        Psh[k] = Pk_t[k];
        Rsh[k] = rkt[k];
      }
    }
    const int kbeg = 0, kend = K;
    float bA = INFINITY, sA = INFINITY, bB = INFINITY, sB = INFINITY;
    int kA = kbeg, kB = kbeg;
    const f32x16 zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                         0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    // (flat tail: the eigen blocks of 32 beyond the kept rank are zero and
    // neither staged nor multiplied)
    const int tid = threadIdx.x;
    const int hi16 = (lane >> 4) & 1;
    // units: one component, or two consecutive flat-tailed ones with kept
    // ranks <= 16 sharing one 32-direction block (as in the list kernel
    // below: the second one's directions in the rows with bit 4 set, each
    // component's squares summed over its own 16 rows, bit for bit the
    // single-component sums); staged 256 entries: the pair's two blocks, or
    // the component's nb blocks of 128
    auto is_pair = [&](int k) { return FLAT && k + 1 < kend && rkt[k] <= 16 && rkt[k + 1] <= 16; };
    auto stage_src = [&](int k, bool pair, int nb) -> const uint4* {
      if (pair) return tid < 256 ? Uf + (size_t)(k + (tid >> 7)) * 256 + (tid & 127) : nullptr;
      return tid < 128 * nb ? Uf + (size_t)k * 256 + tid : nullptr;
    };
    int k = kbeg;
    bool pair = is_pair(k);
    int nb = pair ? 1 : ((FLAT ? rkt[k] : kP) + 31) >> 5;
    uint4 pre = make_uint4(0, 0, 0, 0);
    {
      const uint4* src = stage_src(k, pair, nb);
      if (src) pre = *src;
    }
    for (int u = 0; k < kend; ++u) {
      uint4* As = Ash[u & 1];
      const bool staged = pair ? tid < 256 : tid < 128 * nb;
      if (staged) As[tid] = pre;
      __syncthreads();
      const int kn = k + (pair ? 2 : 1);
      bool pairn = false;
      int nbn = 0;
      if (kn < kend) {
        pairn = is_pair(kn);
        nbn = pairn ? 1 : ((FLAT ? rkt[kn] : kP) + 31) >> 5;
        const uint4* src = stage_src(kn, pairn, nbn);
        if (src) pre = *src;
      }
      const int ek = Esh[pair ? k + hi16 : k];
      float q[PB], q2[PB];
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) q[pb] = q2[pb] = 0.f;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        if (FLAT && rb >= nb) break;
        const int ia = pair ? 128 * hi16 + (lane & ~16) : (2 * rb) * 64 + lane;
        const uint4 a0 = As[ia], a1 = As[ia + 64];
        const i32x8 A = {(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w,
                         (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
        f32x16 acc[PB];
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
          acc[pb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, zq[pb], zero, 0, 0, 0, ek,
                                                                    0, zc[pb]);
        // accumulator i holds direction 8 (i / 4) + 4 h + i % 4
        if (FLAT && pair) {
#pragma unroll
          for (int pb = 0; pb < PB; ++pb)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              q[pb] = fmaf(acc[pb][i], acc[pb][i], q[pb]);
              q2[pb] = fmaf(acc[pb][8 + i], acc[pb][8 + i], q2[pb]);
            }
        } else {
#pragma unroll
          for (int pb = 0; pb < PB; ++pb)
#pragma unroll
            for (int i = 0; i < 16; ++i) q[pb] = fmaf(acc[pb][i], acc[pb][i], q[pb]);
        }
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (c == 1 && !pair) break;
        const int kc = k + c;
        const float* qc = c ? q2 : q;
        const float Lk = Lsh[kc];
        const float mA = pair_sum32(qc[0], qc[1]), mB = pair_sum32(qc[2], qc[3]);
        if (FLAT) {
          const float Pk = Psh[kc], sg = (Rsh[kc] < kP) ? -1.f : 1.f;
          keep_best(fmaf(sg, mA, fmaf(Pk, nzA, Lk)), kc, bA, sA, kA);
          keep_best(fmaf(sg, mB, fmaf(Pk, nzB, Lk)), kc, bB, sB, kB);
        } else {
          keep_best(Lk + mA, kc, bA, sA, kA);
          keep_best(Lk + mB, kc, bB, sB, kB);
        }
      }
      k = kn;
      pair = pairn;
      nb = nbn;
    }
    __syncthreads();  // the staging buffers are reused by the next tile
    // lane's own patches after the half exchange: blocks h and 2 + h
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int pb = 2 * p + h;
      bool v = pval[0];
      int pi = pidx[0];
#pragma unroll
      for (int q = 1; q < PB; ++q)
        if (q == pb) {
          v = pval[q];
          pi = pidx[q];
        }
      if (!v) continue;
      const int64_t i = d.np + (int64_t)pi;
      labels_b[i] = p ? kB : kA;
      if (best_b) best_b[i] = p ? bB : bA;
      if (second_b) second_b[i] = p ? sB : sA;
    }
  }
}


// LIST: the patches of a list (a jittered subset, Sec. 3.3) of the one image
// dsc[0]: 128 list entries per workgroup of 8 waves, the list length read on
// the device (a workgroup past its end exits).
//  1. waves 0..3 each gather a block of 32 patches, one patch per load
//     instruction (lane 8 dy + dx reads pixel (dy, dx): 8 row segments of
//     32 bytes), transpose them through LDS to the operand layout of
//     load_patch8 and quantize them (quantize_patch8), once;
//  2. every wave takes 1/8 of the workgroup's component range and all 128
//     patches (operands from LDS), each component's e4m3 table read from
//     global memory one component ahead;
//  3. the 8 waves' best, second and label per patch are merged in wave
//     order, so ties stay on the lower component, as in one pass;
//  4. with hist, the workgroup counts its labels in LDS and adds the counts
//     to its sort chunk's column of the list sort's histogram (one atomic
//     per component present), which saves the sort its histogram launch.
// A short list is also split over the components across workgroups
// (blockIdx.y of nsplit takes a contiguous component range and writes its
// best, second and label per entry to part; fp8_merge_kernel combines them
// in range order).  The costs are those of the tiled kernel, bit for bit.
constexpr int kListItem = 128;
constexpr int kListWaves = 8;
constexpr int XP = 68;  // LDS pitch (floats) of a gathered patch

template <bool FLAT>
__global__ __launch_bounds__(512) void estep_fp8_list_kernel(
    const ImgDesc* __restrict__ dsc, int t, const float* __restrict__ xb,
    const uint4* __restrict__ Uf_all, const int32_t* __restrict__ Ue_all,
    const float* __restrict__ L_all, const int32_t* __restrict__ rkt,
    const float* __restrict__ P_all, int K, int32_t* __restrict__ labels_b,
    float* __restrict__ best_b, float* __restrict__ second_b, const int32_t* __restrict__ list,
    const int32_t* __restrict__ list_count, int nsplit, float4* __restrict__ part, int pcap,
    int32_t* __restrict__ hist, int nbl) {
  __shared__ float4 Xs4[PB * 32 * XP / 4];  // gathered pixels, then the waves' results
  __shared__ i32x8 Zq[PB][64];
  __shared__ int Zc[PB][64];
  __shared__ float Nz[FLAT ? PB : 1][64];
  __shared__ int Esh[kMaxK];
  __shared__ float Lsh[kMaxK];
  __shared__ float Psh[FLAT ? kMaxK : 1];
  __shared__ int Rsh[FLAT ? kMaxK : 1];
  __shared__ int Hsh[kMaxK];  // label counts of the workgroup (with hist)
  static_assert(kListWaves * kListItem <= PB * 32 * XP / 4, "results fit the pixel buffer");
  static_assert(kListChunk % kListItem == 0, "a workgroup's entries lie in one sort chunk");
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int h = lane >> 5;
  const int col = lane & 31;
  const int nlist = *list_count;
  const int base = blockIdx.x * kListItem;
  if (base >= nlist) return;  // (workgroup-uniform)
  const ImgDesc d = dsc[0];
  const int W = d.W, Wp = d.W - 7;
  const float* x = xb + d.px;
  const size_t slot = (size_t)(d.slot0 + t);
  const uint4* Uf = Uf_all + slot * K * (kTileStride / 16);
  const int32_t* Ue = Ue_all + slot * K;
  const float* L = L_all + slot * K;
  const float* Pk_t = FLAT ? P_all + slot * K : nullptr;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    Esh[k] = Ue[k];
    Lsh[k] = L[k];
    if (FLAT) {
      Psh[k] = Pk_t[k];
      Rsh[k] = rkt[k];
    }
    Hsh[k] = 0;
  }
  float* Xs = reinterpret_cast<float*>(Xs4);

  // 1. gather (entries past the list end repeat a valid one; never written)
  if (wave < PB) {
    const int pid = list[min(base + 32 * wave + col, nlist - 1)];
    const int pr = pid / Wp, pc = pid - pr * Wp;
    const int dy = lane >> 3, dx = lane & 7;
    float v[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const int ri = __builtin_amdgcn_readlane(pr, i), ci = __builtin_amdgcn_readlane(pc, i);
      v[i] = x[(size_t)(ri + dy) * W + ci + dx];
    }
    float* X = Xs + wave * 32 * XP;
#pragma unroll
    for (int i = 0; i < 32; ++i) X[i * XP + lane] = v[i];
  }
  __syncthreads();
  if (wave < PB) {
    const float4* X = reinterpret_cast<const float4*>(Xs + wave * 32 * XP + col * XP + 32 * h);
    float v[32];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float4 f = X[q];
      v[4 * q] = f.x;
      v[4 * q + 1] = f.y;
      v[4 * q + 2] = f.z;
      v[4 * q + 3] = f.w;
    }
    i32x8 zq;
    int code;
    float nz = 0.f;
    quantize_patch8<FLAT>(v, zq, code, nz);
    Zq[wave][lane] = zq;
    Zc[wave][lane] = code;
    if (FLAT) Nz[wave][lane] = nz;
  }
  __syncthreads();

  // 2. this wave's component range
  i32x8 zq[PB];
  int zc[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    zq[pb] = Zq[pb][lane];
    zc[pb] = Zc[pb][lane];
  }
  const float nzA = FLAT ? Nz[FLAT ? h : 0][lane] : 0.f;
  const float nzB = FLAT ? Nz[FLAT ? 2 + h : 0][lane] : 0.f;
  const int kb = (int)(((int64_t)K * blockIdx.y) / nsplit);
  const int ke = (int)(((int64_t)K * (blockIdx.y + 1)) / nsplit);
  const int k0 = kb + ((ke - kb) * wave) / kListWaves;
  const int k1 = kb + ((ke - kb) * (wave + 1)) / kListWaves;
  float bA = INFINITY, sA = INFINITY, bB = INFINITY, sB = INFINITY;
  int kA = k0, kB = k0;
  const f32x16 zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                       0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  // The component loop runs over units: one component, or (flat tail) two
  // consecutive components whose kept ranks are both at most 16, packed in
  // one 32-direction block (lanes with bit 4 set read the second one's
  // directions, each with its own scale), so one MFMA projects on both.  A
  // direction beyond a component's rank has a zero operand row, so each
  // component's sum of squares, taken over its own 16 rows in the same
  // order, is the one of a single-component block bit for bit.  Operands of
  // the next kPre units wait in a register queue (slot 0 is consumed, the
  // others move up, the new unit enters the last slot); eigen blocks of 32
  // beyond a kept rank are neither read nor multiplied.
  constexpr int kPre = 4;
  uint4 pre[kPre][4];
  int uk[kPre];     // first component of the unit in each slot (k1: none)
  bool up[kPre];    // the slot holds a pair
  int kf = k0;      // first component of the next unit to fetch
  const int hi16 = (lane >> 4) & 1;
  auto fetch = [&](uint4(&dst)[4], int& dk, bool& dp) __attribute__((always_inline)) {
    dk = k1;
    dp = false;
    if (kf >= k1) return;
    const int k = kf;
    const bool pair = FLAT && k + 1 < k1 && Rsh[k] <= 16 && Rsh[k + 1] <= 16;
    dk = k;
    dp = pair;
    if (pair) {
      const uint4* u = Uf + (size_t)(k + hi16) * 256 + (lane & ~16);
      dst[0] = u[0];
      dst[1] = u[64];
    } else {
      const uint4* u = Uf + (size_t)k * 256 + lane;
      dst[0] = u[0];
      dst[1] = u[64];
      if (!FLAT || Rsh[k] > 32) {
        dst[2] = u[128];
        dst[3] = u[192];
      }
    }
    kf = k + (pair ? 2 : 1);
  };
  // cost of component k from its squared projections q (per patch block)
  auto score = [&](int k, const float(&q)[PB]) __attribute__((always_inline)) {
    const float Lk = Lsh[k];
    const float mA = pair_sum32(q[0], q[1]), mB = pair_sum32(q[2], q[3]);
    if (FLAT) {
      const float Pk = Psh[k], sg = (Rsh[k] < kP) ? -1.f : 1.f;
      keep_best(fmaf(sg, mA, fmaf(Pk, nzA, Lk)), k, bA, sA, kA);
      keep_best(fmaf(sg, mB, fmaf(Pk, nzB, Lk)), k, bB, sB, kB);
    } else {
      keep_best(Lk + mA, k, bA, sA, kA);
      keep_best(Lk + mB, k, bB, sB, kB);
    }
  };
#pragma unroll
  for (int j = 0; j < kPre; ++j) fetch(pre[j], uk[j], up[j]);
  while (uk[0] < k1) {
    const int k = uk[0];
    const bool pair = up[0];
    const uint4 cur[4] = {pre[0][0], pre[0][1], pre[0][2], pre[0][3]};
#pragma unroll
    for (int j = 0; j + 1 < kPre; ++j) {
#pragma unroll
      for (int e = 0; e < 4; ++e) pre[j][e] = pre[j + 1][e];
      uk[j] = uk[j + 1];
      up[j] = up[j + 1];
    }
    fetch(pre[kPre - 1], uk[kPre - 1], up[kPre - 1]);
    const int nb = pair ? 1 : ((FLAT ? Rsh[k] : kP) + 31) >> 5;
    const int ek = Esh[pair ? k + hi16 : k];
    float q[PB], q2[PB];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) q[pb] = q2[pb] = 0.f;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      if (rb >= nb) break;
      const uint4 a0 = cur[2 * rb], a1 = cur[2 * rb + 1];
      const i32x8 A = {(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w,
                       (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
      f32x16 acc[PB];
#pragma unroll
      for (int pb = 0; pb < PB; ++pb)
        acc[pb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, zq[pb], zero, 0, 0, 0, ek, 0,
                                                                  zc[pb]);
      // accumulator i holds direction 8 (i / 4) + 4 h + i % 4: i < 8 the
      // block's first 16 directions, i >= 8 the others
      if (pair) {
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            q[pb] = fmaf(acc[pb][i], acc[pb][i], q[pb]);
            q2[pb] = fmaf(acc[pb][8 + i], acc[pb][8 + i], q2[pb]);
          }
      } else {
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
#pragma unroll
          for (int i = 0; i < 16; ++i) q[pb] = fmaf(acc[pb][i], acc[pb][i], q[pb]);
      }
    }
    score(k, q);
    if (pair) score(k + 1, q2);
  }

  // 3. merge the waves' ranges in order (the pixel buffer is free since the
  // second barrier)
  float4* M = Xs4;
  M[wave * kListItem + 32 * h + col] = make_float4(bA, sA, __int_as_float(kA), 0.f);
  M[wave * kListItem + 32 * (2 + h) + col] = make_float4(bB, sB, __int_as_float(kB), 0.f);
  __syncthreads();
  if (threadIdx.x < kListItem) {
    const int qi = threadIdx.x;
    float b = INFINITY, s2 = INFINITY;
    int k = kb;
#pragma unroll
    for (int w = 0; w < kListWaves; ++w) {
      const float4 r = M[w * kListItem + qi];
      if (r.x < b) {
        s2 = fminf(b, r.y);
        b = r.x;
        k = __float_as_int(r.z);
      } else {
        s2 = fminf(s2, r.x);
      }
    }
    const int e = base + qi;
    if (e < nlist) {
      if (nsplit > 1) {
        part[(size_t)blockIdx.y * pcap + e] = make_float4(b, s2, __int_as_float(k), 0.f);
      } else {
        const int64_t i = d.np + (int64_t)list[e];
        labels_b[i] = k;
        if (best_b) best_b[i] = b;
        if (second_b) second_b[i] = s2;
        if (hist) atomicAdd(&Hsh[k], 1);
      }
    }
  }
  // 4. (one pass) the labels' counts added to this chunk's histogram column
  if (hist) {
    __syncthreads();
    const int ch = base / kListChunk;
    for (int k = threadIdx.x; k < K; k += blockDim.x)
      if (Hsh[k]) atomicAdd(&hist[(size_t)k * nbl + ch], Hsh[k]);
  }
}

hipError_t launch_estep_fp8_batch(const Batch& b, const float* x, const uint8_t* Uf,
                                  const int32_t* Ue, const float* L32, const int32_t* rk,
                                  const float* Pinv, int K, int t, int32_t* labels, float* best,
                                  float* second, int blocks, hipStream_t st) {
  // persistent: a fixed number of workgroups looping over the tiles
  if (blocks <= 0 || blocks > b.n_est) blocks = b.n_est;
  if (blocks < 1) return hipSuccess;
  if (rk)
    hipLaunchKernelGGL((estep_fp8_kernel<true>), dim3(blocks), dim3(256), 0, st, b.d, b.est_img,
                       b.n_est, t, x, reinterpret_cast<const uint4*>(Uf), Ue, L32, rk, Pinv, K,
                       labels, best, second);
  else
    hipLaunchKernelGGL((estep_fp8_kernel<false>), dim3(blocks), dim3(256), 0, st, b.d, b.est_img,
                       b.n_est, t, x, reinterpret_cast<const uint4*>(Uf), Ue, L32, rk, Pinv, K,
                       labels, best, second);
  return hipGetLastError();
}

// Per list entry: the best, second and label over the nsplit component
// ranges, in range order (ties stay on the lower component).
__global__ __launch_bounds__(256) void fp8_merge_kernel(const ImgDesc* __restrict__ d,
                                                        const int32_t* __restrict__ count,
                                                        const int32_t* __restrict__ list,
                                                        const float4* __restrict__ part,
                                                        int pcap, int nsplit,
                                                        int32_t* __restrict__ labels_b,
                                                        float* __restrict__ best_b,
                                                        float* __restrict__ second_b) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= *count) return;
  float b = INFINITY, s = INFINITY;
  int k = 0;
  for (int j = 0; j < nsplit; ++j) {
    const float4 q = part[(size_t)j * pcap + e];
    if (q.x < b) {
      s = fminf(b, q.y);
      b = q.x;
      k = __float_as_int(q.z);
    } else {
      s = fminf(s, q.x);
    }
  }
  const int64_t i = d->np + (int64_t)list[e];
  labels_b[i] = k;
  if (best_b) best_b[i] = b;
  if (second_b) second_b[i] = s;
}

int fp8_list_split(int64_t list_max, int K) {
  // a list of at least 128 workgroups runs in one pass; a shorter one is
  // split over the components up to about 256 workgroups
  const int64_t items = (list_max + kListItem - 1) / kListItem;
  if (items >= 128) return 1;
  int64_t ns = (256 + items - 1) / std::max<int64_t>(items, 1);
  ns = std::min<int64_t>(ns, std::min(16, K));
  return (int)std::max<int64_t>(ns, 1);
}

hipError_t launch_estep_fp8_list(const ImgDesc* d, int64_t list_max, int t, const float* x,
                                 const uint8_t* Uf, const int32_t* Ue, const float* L32,
                                 const int32_t* rk, const float* Pinv, int K,
                                 const int32_t* count, const int32_t* list, int32_t* labels,
                                 float* best, float* second, float4* part, int* nsplit,
                                 int32_t* hist, int nbl, hipStream_t st) {
  *nsplit = 1;
  if (hist && part) return hipErrorInvalidValue;
  // one workgroup per 128 entries of the longest list; the actual length is
  // read on the device
  const int64_t blocks = (list_max + kListItem - 1) / kListItem;
  if (blocks < 1) return hipSuccess;
  const int ns = part ? fp8_list_split(list_max, K) : 1;
  const int pcap = (int)list_max;
  const dim3 grid((unsigned)blocks, ns);
  if (rk)
    hipLaunchKernelGGL((estep_fp8_list_kernel<true>), grid, dim3(64 * kListWaves), 0, st, d, t, x,
                       reinterpret_cast<const uint4*>(Uf), Ue, L32, rk, Pinv, K, labels, best,
                       second, list, count, ns, part, pcap, hist, nbl);
  else
    hipLaunchKernelGGL((estep_fp8_list_kernel<false>), grid, dim3(64 * kListWaves), 0, st, d, t,
                       x, reinterpret_cast<const uint4*>(Uf), Ue, L32, rk, Pinv, K, labels, best,
                       second, list, count, ns, part, pcap, hist, nbl);
  *nsplit = ns;
  return hipGetLastError();
}

hipError_t launch_fp8_merge(const ImgDesc* d, int64_t list_max, const int32_t* count,
                            const int32_t* list, const float4* part, int nsplit, int32_t* labels,
                            float* best, float* second, hipStream_t st) {
  if (nsplit <= 1) return hipSuccess;
  hipLaunchKernelGGL(fp8_merge_kernel, dim3((unsigned)((list_max + 255) / 256)), dim3(256), 0, st,
                     d, count, list, part, (int)list_max, nsplit, labels, best, second);
  return hipGetLastError();
}

}  // namespace fepll
