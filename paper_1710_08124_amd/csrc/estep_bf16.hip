// Gaussian selection with bfloat16 projections (same step as estep.hip:
// Alg. 1 patch extraction + Gaussian selection in the eigenspace form of
// Sec. 2.1), for the reduced-precision mode: the DC-removed patches and the
// scaled eigenbases Ut_k = U_k diag(nu_k)^-1/2 are rounded to bfloat16, the
// products accumulate in float32 on v_mfma_f32_32x32x16_bf16, and the
// squared norms, the log-determinant terms L_k and the argmin stay float32.
// Labels are not certified in this mode: they are an approximation whose
// agreement with the exact selection is measured, not assumed.
//
// v_mfma_f32_16x16x32_bf16 multiplies 16 eigen-directions by 16 patches
// over 32 pixels: lane l supplies the 8 pixels 32 t + 8 (l >> 4) + e
// (e = 0..7) of patch (l & 15) -- exactly one 8-pixel row,
// dy = 4 t + (l >> 4), of the patch -- and the A operand supplies the same
// pixels of eigen-direction 16 rb + (l & 15).  (On gfx950 this shape keeps
// the matrix cores busier than 32x32x16 for this loop: measured 83% against
// 64% of the bf16 peak without the epilogue.)  A wave holds 128 patches
// (eight blocks of 16) as B operands for its whole component loop; per
// component it issues 4 (eigen blocks) x 2 (depth steps) x 8 (patch blocks)
// MFMAs and 128 float32 FMAs of squares, then reduces each patch's squared
// norm over the four 16-lane groups (lanes l, l^16, l^32, l^48) with a
// transpose-reduction that leaves every lane owning 2 patches.
//
// Two modes share the kernel:
//  * spatial, all K: a wave takes 128 consecutive patches of one row;
//  * list, all K: the proposal's fallback patches, 512 list entries per
//    workgroup, with a device-side list length (fixed grid, workgroups
//    stride over the list and exit past its end); the patches' operands
//    come from the records the proposal network writes, or, without them
//    (the jittered patch subset), from the image.
// The exact rescoring of the proposal's candidates runs over (patch,
// candidate) pairs bucketed by component (pairs_bf16_kernel), each tile of
// 128 pairs sharing one operand, with the same scoring arithmetic.
// In the all-K modes the per-component operand is staged through
// double-buffered LDS shared by the workgroup's 4 waves (one barrier per
// component, the next component's operand already loading).
#include <algorithm>

#include "common.h"
#include "propose.h"
#include "wave_ops.h"

namespace fepll {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {
constexpr int PB = 8;  // blocks of 16 patches per wave

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
__device__ __forceinline__ f32x4 mfma16(uint4 a, uint4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
// DC-removed bfloat16 B operands (2 depth steps) of one 16-patch block for
// lane group g = l >> 4: patch rows g and 4 + g of the patch at (r, c).
// With NZ, nz receives the float32 squared norm of the (unrounded)
// DC-removed patch, the same in the 4 lanes of its column.
template <bool NZ>
__device__ __forceinline__ void load_patch(const float* __restrict__ x, int W, int r, int c,
                                           int g, uint4 zb[2], float& nz) {
  // the mean in float64 (exact for any order whenever the patch's pixel
  // magnitudes lie within 2^23 of each other), each difference rounded once
  // to float32
  float v[2][8];
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const float* row = x + (size_t)(r + 4 * t + g) * W + c;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      v[t][e] = row[e];
      s += (double)v[t][e];
    }
  }
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  const double m = s * (1.0 / 64.0);
  float q2 = 0.f;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    float d[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      d[e] = (float)((double)fresh(v[t][e]) - m);
      if (NZ) q2 = fmaf(d[e], d[e], q2);
    }
    zb[t] = make_uint4(pack2(d[0], d[1]), pack2(d[2], d[3]), pack2(d[4], d[5]),
                       pack2(d[6], d[7]));
  }
  if (NZ) {
    q2 += __shfl_xor(q2, 16);
    nz = q2 + __shfl_xor(q2, 32);
  }
}

// The same operands for a patch anywhere in the image, from the patch-major
// records the proposal network writes (rows dy at uint4 dy, the squared norm
// beside): lane group g takes rows g and 4 + g.  Bit for bit what
// load_patch computes (same mean and norm order).
template <bool NZ>
__device__ __forceinline__ void load_operand(const uint4* __restrict__ zop,
                                             const float* __restrict__ znz, int i, int g,
                                             uint4 zb[2], float& nz) {
  zb[0] = zop[(size_t)i * 8 + g];
  zb[1] = zop[(size_t)i * 8 + 4 + g];
  if (NZ) nz = znz[i];
}

// Squared norms of the 8 x 16 patches' projections on the first 16 NB
// directions of one component whose operand (4 eigen blocks x 2 depth steps,
// this lane's entries) starts at ap with a stride of 64 uint4.  Lane l
// (group g = l >> 4) returns the sums of the two patches it owns: blocks
// 4 (g >> 1) + 2 (g & 1) + {0, 1}, column l & 15.
// NB < 0: the block count nb (1..4) is known at run time only, and each
// block's operand is loaded in turn (the flat-tail form).
template <int NB>
__device__ __forceinline__ void project(const uint4* ap, const uint4 zb[PB][2], float& mA,
                                        float& mB, int nb = NB) {
  float q[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) q[pb] = 0.f;
  if (NB > 0) {
    uint4 A[2 * (NB > 0 ? NB : 1)];
#pragma unroll
    for (int i = 0; i < 2 * NB; ++i) A[i] = ap[i * 64];
#pragma unroll
    for (int rb = 0; rb < NB; ++rb) {
      f32x4 acc[PB];
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) acc[pb] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) acc[pb] = mfma16(A[rb * 2 + t], zb[pb][t], acc[pb]);
#pragma unroll
      for (int pb = 0; pb < PB; ++pb)
#pragma unroll
        for (int i = 0; i < 4; ++i) q[pb] = fmaf(acc[pb][i], acc[pb][i], q[pb]);
    }
  } else {
    for (int rb = 0; rb < nb; ++rb) {
      const uint4 A0 = ap[(2 * rb) * 64], A1 = ap[(2 * rb + 1) * 64];
      f32x4 acc[PB];
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) acc[pb] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) acc[pb] = mfma16(A0, zb[pb][0], acc[pb]);
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) acc[pb] = mfma16(A1, zb[pb][1], acc[pb]);
#pragma unroll
      for (int pb = 0; pb < PB; ++pb)
#pragma unroll
        for (int i = 0; i < 4; ++i) q[pb] = fmaf(acc[pb][i], acc[pb][i], q[pb]);
    }
  }
  // lane groups g and g ^ 2 split the 8 blocks in halves, then g and g ^ 1:
  // lanes of groups 0/1 keep blocks 0..3, groups 2/3 keep 4..7, then even
  // groups keep the first two of their four, odd groups the last two
  float m4[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) m4[i] = pair_sum32(q[i], q[4 + i]);
  float m2[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) m2[i] = pair_sum16(m4[i], m4[2 + i]);
  mA = m2[0];
  mB = m2[1];
}

// Costs of the lane's two patches for component k.  Plain form: L_k plus
// the 64 squared projections.  Flat-tail form (Sec. 3.1, rk < 64 kept
// directions): L_k + Pk |z~|^2 minus the squared projections on the
// ceil(rk / 16) blocks that hold the kept directions (the operand's
// columns carry sqrt(1/nu_P - 1/nu_j), Pk = 1/nu_P); a component without a
// tail (rk = 64, Pk = 0) takes the plain form, rounded identically.
template <bool FLAT>
__device__ __forceinline__ void score(const uint4* ap, const uint4 zb[PB][2], float Lk, int rk,
                                      float Pk, float nzA, float nzB, float& cA, float& cB) {
  float mA, mB;
  if (!FLAT) {
    project<4>(ap, zb, mA, mB);
    cA = Lk + mA;
    cB = Lk + mB;
    return;
  }
  const int nb = (rk + 15) >> 4;
  if (nb == 1)  // the common case (r_k <= 16)
    project<1>(ap, zb, mA, mB);
  else
    project<-1>(ap, zb, mA, mB, nb);
  const float sg = (rk < kP) ? -1.f : 1.f;
  cA = fmaf(sg, mA, fmaf(Pk, nzA, Lk));
  cB = fmaf(sg, mB, fmaf(Pk, nzB, Lk));
}
}  // namespace

template <int MODE, bool FLAT>
__global__ __launch_bounds__(256, 3) void estep_bf16_kernel(BF16Args a) {
  __shared__ uint4 Ash[2][512];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;
  const int col = lane & 15;

  const int nlist = (MODE == kModeListFull) ? *a.list_count : 0;
  // batched list mode: S workgroups per item, each over a share of K
  const int S = (MODE == kModeListBatch) ? max(1, a.ksplit) : 1;
  const int nitems = (MODE == kModeListBatch) ? a.item_pre[a.n_img] * S : 0;
  // work items: list mode, 512 consecutive list entries (batched: times
  // the component parts); spatial all-K mode, one selection tile (4 patch
  // rows x 128 columns) of any image of the batch.  The loop is
  // workgroup-uniform: every wave reaches every barrier of the K loop.
  int item = blockIdx.y * gridDim.x + blockIdx.x;
  const int nwg = gridDim.x * gridDim.y;
  for (;; item += nwg) {
    // ---- this item's image and tables
    const float* x = a.x;
    int H = a.H, W = a.W;
    const uint16_t* Ub = a.Ub;
    const float* Lt = a.L;
    const float* Pt = a.Pinv;
    int32_t* labels = a.labels;
    float* bestp = a.best;
    float* secondp = a.second;
    int tr = blockIdx.y, tc = blockIdx.x;  // tile row / column (spatial modes)
    // list modes: the list, its length and this item's first entry
    const int32_t* list = a.list;
    int nl = nlist, lbase = item * 512;
    // the components this item searches, and where a split part's results go
    int kb_l = 0, ke_l = 0;
    int32_t* pout = nullptr;
    if (MODE == kModeListBatch) {
      if (item >= nitems) break;
      const int li = item / S, part = item - li * S;
      kb_l = part * a.K / S;
      ke_l = (part + 1) * a.K / S;
      // the image of this item: the last one whose first item is <= li
      int lo = 0, hi = a.n_img - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.item_pre[mid] <= li)
          lo = mid;
        else
          hi = mid - 1;
      }
      const ImgDesc d = a.d[lo];
      H = d.H;
      W = d.W;
      x += d.px;
      const size_t slot = (size_t)(d.slot0 + a.t);
      Ub += slot * a.K * kTileStride;
      Lt += slot * a.K;
      if (FLAT) Pt += slot * a.K;
      labels += d.np;
      if (bestp) bestp += d.np;
      if (secondp) secondp += d.np;
      list += d.np;
      nl = a.list_count[lo];
      lbase = (li - a.item_pre[lo]) * 512;
      if (S > 1) pout = a.part_out + (size_t)part * a.part_stride + d.np;
    }
    if (MODE == kModeSpatialFull) {
      if (item >= a.n_est) break;
      const int im = a.est_img[item];
      const ImgDesc d = a.d[im];
      H = d.H;
      W = d.W;
      x += d.px;
      const size_t slot = (size_t)(d.slot0 + a.t);
      Ub += slot * a.K * kTileStride;
      Lt += slot * a.K;
      if (FLAT) Pt += slot * a.K;
      labels += d.np;
      if (bestp) bestp += d.np;
      if (secondp) secondp += d.np;
      const int ntx = (W - 7 + kEstCols - 1) / kEstCols;
      const int lt = item - d.est0;
      tr = lt / ntx;
      tc = lt - tr * ntx;
    }
    const int Hp = H - 7, Wp = W - 7;
    // ---- this wave's 128 patches
    int idx[PB];
    bool valid[PB];
    if (MODE != kModeSpatialFull) {
      if (MODE == kModeListFull && lbase >= nl) break;
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
        const int e = lbase + wave * 128 + 16 * pb + col;
        valid[pb] = e < nl;
        idx[pb] = list[valid[pb] ? e : lbase];
      }
    } else {
      const int r = tr * 4 + wave;
      const int c0 = tc * (16 * PB);
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
        const int c = c0 + 16 * pb + col;
        valid[pb] = (r < Hp) && (c < Wp);
        idx[pb] = min(r, Hp - 1) * Wp + min(c, Wp - 1);
      }
    }
    uint4 zb[PB][2];
    float nzA = 0.f, nzB = 0.f;  // flat tail: |z~|^2 of the lane's own patches
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      float nz = 0.f;
      if (MODE == kModeListFull && a.zop) {  // (uniform)
        load_operand<FLAT>(a.zop, a.znz, idx[pb], g, zb[pb], nz);
      } else {
        const int pr = idx[pb] / Wp;
        load_patch<FLAT>(x, W, pr, idx[pb] - pr * Wp, g, zb[pb], nz);
      }
      if (FLAT) {
        const int ow = 4 * (g >> 1) + 2 * (g & 1);
        nzA = (pb == ow) ? nz : nzA;
        nzB = (pb == ow + 1) ? nz : nzB;
      }
      // one block's raw pixels live at a time (keeps the prologue in registers)
      __builtin_amdgcn_sched_barrier(0);
    }
    // lane's own patches: blocks 4 (g >> 1) + 2 (g & 1) + {0, 1}
    const int own = 4 * (g >> 1) + 2 * (g & 1);
    int iA = idx[0], iB = idx[1];
    bool vA = valid[0], vB = valid[1];
#pragma unroll
    for (int pb = 0; pb < PB; pb += 2)
      if (pb == own) {
        iA = idx[pb];
        iB = idx[pb + 1];
        vA = valid[pb];
        vB = valid[pb + 1];
      }

    float bA = INFINITY, sA = INFINITY, bB = INFINITY, sB = INFINITY;
    int kA = 0, kB = 0;
    {
      // all K: the per-component operand (8 KB) is staged once per
      // workgroup in LDS, double-buffered, the next one already in flight
      // (flat tail: only the 128 uint4 of each block that holds kept
      // directions)
      const uint4* gsrc = reinterpret_cast<const uint4*>(Ub);
      const int tid = threadIdx.x;
      int kb = 0, ke = a.K;
      if constexpr (MODE == kModeListBatch) {
        kb = kb_l;
        ke = ke_l;
      }
      int rn = kP, nu4 = 512;
      uint4 pre0, pre1;
      // component kb's operand (kb < K whenever the range is not empty; an
      // empty one prefetches component kb < K all the same and searches
      // nothing)
      const uint4* gb = gsrc;
      if constexpr (MODE == kModeListBatch) gb += (size_t)kb * 512;
      if (FLAT) {
        rn = a.rk[kb];
        nu4 = 128 * ((rn + 15) >> 4);
        pre0 = pre1 = make_uint4(0, 0, 0, 0);
        if (tid < nu4) pre0 = gb[tid];
        if (256 + tid < nu4) pre1 = gb[256 + tid];
      } else {
        pre0 = gb[tid];
        pre1 = gb[256 + tid];
      }
      for (int k = kb; k < ke; ++k) {
        uint4* As = Ash[k & 1];
        const int rk = rn;
        if (FLAT) {
          if (tid < nu4) As[tid] = pre0;
          if (256 + tid < nu4) As[256 + tid] = pre1;
        } else {
          As[tid] = pre0;
          As[256 + tid] = pre1;
        }
        __syncthreads();
        if (k + 1 < ke) {
          if (FLAT) {
            rn = a.rk[k + 1];
            nu4 = 128 * ((rn + 15) >> 4);
            if (tid < nu4) pre0 = gsrc[(size_t)(k + 1) * 512 + tid];
            if (256 + tid < nu4) pre1 = gsrc[(size_t)(k + 1) * 512 + 256 + tid];
          } else {
            pre0 = gsrc[(size_t)(k + 1) * 512 + tid];
            pre1 = gsrc[(size_t)(k + 1) * 512 + 256 + tid];
          }
        }
        float cA, cB;
        score<FLAT>(As + lane, zb, Lt[k], rk, FLAT ? Pt[k] : 0.f, nzA, nzB, cA, cB);
        keep_best(cA, k, bA, sA, kA);
        keep_best(cB, k, bB, sB, kB);
      }
      __syncthreads();  // the staging buffers are reused by the next pass
    }
    // ---- outputs (a split part's to its slots, for the merge)
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const bool v = p ? vB : vA;
      if (!v) continue;
      const int i = p ? iB : iA;
      const float b = p ? bB : bA, s = p ? sB : sA;
      if constexpr (MODE == kModeListBatch) {
        if (pout) {
          // by list entry: the lane group's 16 entries are contiguous
          const int e = lbase + wave * 128 + 16 * (own + p) + col;
          const size_t ps = (size_t)S * a.part_stride;
          pout[e] = p ? kB : kA;
          pout[ps + e] = __float_as_int(b);
          pout[2 * ps + e] = __float_as_int(s);
          continue;
        }
      }
      labels[i] = p ? kB : kA;
      if (bestp) bestp[i] = b;
      if (secondp) secondp[i] = s;
    }
  }
}

// ---- Exact rescoring of the proposal's candidates.  A workgroup takes
// kRescPatches consecutive patches of one image of the batch: it builds their
// bfloat16 operands in LDS (load_patch: bit for bit the all-K operands),
// groups their (patch, candidate) pairs by component with a counting sort in
// LDS, and each wave scores the pairs of every eighth component, 16 pairs
// per MFMA block and up to 4 blocks per pass, with the all-K arithmetic
// (same products, same squares in the same order, same lane-group sums
// (q0 + q2) + (q1 + q3)), so every (patch, k) cost equals the full search's.
// Per patch, the best (lowest cost, then lowest k) and the second cost are
// kept by two LDS atomic minima on order-preserving keys: an update leaves
// the larger of the old best and the new cost to the second minimum, and
// every cost but the final best is that larger value exactly once, so the
// result does not depend on the order of the updates.  Last, labels, costs
// and the fallback list: half the exact gap of the two best below the
// margin, or fewer than two candidates.

// Order-preserving map of a float cost to uint32 (-0 taken as +0).
__device__ __forceinline__ uint32_t cost_key(float c) {
  const uint32_t u = __float_as_uint(c + 0.f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_cost(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
// LDS slot of uint4 j (0..7) of the record of local patch pl: rotated by the
// patch, so the 16 lanes of a gather spread over the banks
__device__ __forceinline__ int rec_slot(int pl, int j) { return pl * 8 + (j ^ (pl & 7)); }

// Squared projections of NBLK blocks of 16 pairs on NRB eigen blocks of one
// component (A: its operand, 2 depth steps per eigen block): per block the
// lane group's partial sum, accumulated in the order of project().
// Straight-line code for each shape, so the blocks' products interleave.
template <int NBLK, int NRB>
__device__ __forceinline__ void square_blocks(const uint4 A[8], const uint4 zb[4][2],
                                              float q[4]) {
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    f32x4 acc[NBLK];
#pragma unroll
    for (int pb = 0; pb < NBLK; ++pb)
      acc[pb] = mfma16(A[2 * rb], zb[pb][0], (f32x4){0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int pb = 0; pb < NBLK; ++pb) acc[pb] = mfma16(A[2 * rb + 1], zb[pb][1], acc[pb]);
#pragma unroll
    for (int pb = 0; pb < NBLK; ++pb)
#pragma unroll
      for (int i = 0; i < 4; ++i) q[pb] = fmaf(acc[pb][i], acc[pb][i], q[pb]);
  }
}
template <int NRB>
__device__ __forceinline__ void square_chunk(int nblk, const uint4 A[8], const uint4 zb[4][2],
                                             float q[4]) {
  switch (nblk) {  // (wave-uniform)
    case 1: square_blocks<1, NRB>(A, zb, q); break;
    case 2: square_blocks<2, NRB>(A, zb, q); break;
    case 3: square_blocks<3, NRB>(A, zb, q); break;
    default: square_blocks<4, NRB>(A, zb, q); break;
  }
}

constexpr int kRescThreads = 1024;  // 16 waves: 4 per SIMD
constexpr int kRescWaves = kRescThreads / 64;
static_assert(kRescPatches <= kRescThreads && kRescPatches % 16 == 0, "one patch per thread");

template <bool FLAT>
__global__ __launch_bounds__(kRescThreads, 1) void rescore_bf16_kernel(RescoreArgs a) {
  __shared__ uint4 rec[kRescPatches * 8];
  __shared__ float nzs[FLAT ? kRescPatches : 1];
  __shared__ uint16_t plist[kRescPatches * 8];
  __shared__ unsigned long long bkey[kRescPatches];
  __shared__ uint32_t skey[kRescPatches];
  __shared__ int32_t hcnt[kMaxK];
  __shared__ int32_t hend[kMaxK];
  __shared__ int32_t wsum[kRescWaves];
  __shared__ int32_t fbase;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, col = lane & 15;
  const int K = a.K, m = a.m;
  const int im = a.tile_img[blockIdx.x];
  const ImgDesc d = a.d[im];
  const int W = d.W, Wp = d.W - 7;
  const int Np = (d.H - 7) * Wp;
  const int base = (blockIdx.x - d.resc0) * kRescPatches;
  const int npw = min(kRescPatches, Np - base);
  const float* x = a.x + d.px;
  const size_t slot = (size_t)(d.slot0 + a.t);

  // the pairs are taken pair-major (pair e: candidate e & 7 of local patch
  // e >> 3), so the lanes of one LDS atomic name at most 8 patches' j-th
  // candidates (neighbouring patches often share them); the candidates are
  // in flight during the operand build
  const uint16_t* cand = a.cand + ((size_t)d.np + base) * 8;
  constexpr int kPairsPerThread = kRescPatches * 8 / kRescThreads;
  static_assert(kRescPatches * 8 % kRescThreads == 0, "whole pairs per thread");
  int ck[kPairsPerThread];
#pragma unroll
  for (int i = 0; i < kPairsPerThread; ++i) {
    const int e = tid + kRescThreads * i;
    const int k = ((e >> 3) < npw) ? (int)cand[e] : 0xffff;
    ck[i] = ((e & 7) < m && k < K) ? k : -1;  // (an index >= K is never scored)
  }
  for (int k = tid; k < K; k += kRescThreads) hcnt[k] = 0;
  if (tid < kRescPatches) {
    bkey[tid] = ~0ull;
    skey[tid] = ~0u;
  }
  // ---- operands: 16 patches per wave pass (lane group g: rows g, 4 + g);
  // past the image's last patch, copies of it that no pair names
  for (int b = wave; b < kRescPatches / 16; b += kRescWaves) {
    const int pl = 16 * b + col;
    const int p = base + min(pl, npw - 1);
    const int r = p / Wp;
    uint4 zb[2];
    float nz = 0.f;
    load_patch<FLAT>(x, W, r, p - r * Wp, g, zb, nz);
    rec[rec_slot(pl, g)] = zb[0];
    rec[rec_slot(pl, 4 + g)] = zb[1];
    if (FLAT && g == 0) nzs[pl] = nz;
  }
  __syncthreads();
  // ---- the pairs by component: counts, exclusive scan, scatter
#pragma unroll
  for (int i = 0; i < kPairsPerThread; ++i)
    if (ck[i] >= 0) atomicAdd(&hcnt[ck[i]], 1);
  __syncthreads();
  {
    // one component per thread (K <= 1024)
    const int c0 = (tid < K) ? hcnt[tid] : 0;
    int sc = c0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int u = __shfl_up(sc, off);
      if (lane >= off) sc += u;
    }
    if (lane == 63) wsum[wave] = sc;
    __syncthreads();
    int pre = 0;
    for (int w = 0; w < wave; ++w) pre += wsum[w];
    if (tid < K) hend[tid] = pre + sc - c0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kPairsPerThread; ++i)
    if (ck[i] >= 0)
      plist[atomicAdd(&hend[ck[i]], 1)] = (uint16_t)((tid + kRescThreads * i) >> 3);
  __syncthreads();
  // ---- scores: component k's pairs are plist[hend[k] - hcnt[k] .. hend[k])
  const uint4* up = reinterpret_cast<const uint4*>(a.Ub + slot * K * kTileStride) + lane;
  const float* Lt = a.L + slot * K;
  for (int k = wave; k < K; k += kRescWaves) {
    const int n = __builtin_amdgcn_readfirstlane(hcnt[k]);
    if (n == 0) continue;
    const int s0 = __builtin_amdgcn_readfirstlane(hend[k]) - n;
    const int rk = FLAT ? a.rk[k] : kP;
    const float Pk = FLAT ? a.Pinv[slot * K + k] : 0.f;
    const float Lk = Lt[k];
    // flat tail: the eigen blocks past the kept directions get a zero
    // operand (their products add exact zeros), one block when r_k <= 16
    const int nb = FLAT ? __builtin_amdgcn_readfirstlane((rk + 15) >> 4) : 4;
    uint4 A[8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
      A[i] = (!FLAT || i < 2 * nb) ? up[(size_t)k * 512 + i * 64] : make_uint4(0u, 0u, 0u, 0u);
    for (int c0 = 0; c0 < n; c0 += 64) {
      const int nblk = min(4, (n - c0 + 15) >> 4);
      int pl[4];
      uint4 zb[4][2];
#pragma unroll
      for (int pb = 0; pb < 4; ++pb) {
        pl[pb] = plist[s0 + min(c0 + 16 * pb + col, n - 1)];
        zb[pb][0] = rec[rec_slot(pl[pb], g)];
        zb[pb][1] = rec[rec_slot(pl[pb], 4 + g)];
      }
      float q[4] = {0.f, 0.f, 0.f, 0.f};
      if (FLAT && nb == 1)
        square_chunk<1>(nblk, A, zb, q);
      else
        square_chunk<4>(nblk, A, zb, q);
      // lane group g ends with block g's column sums: (q0 + q2) + (q1 + q3)
      const float mm = pair_sum16(pair_sum32(q[0], q[2]), pair_sum32(q[1], q[3]));
      if (c0 + 16 * g + col < n) {
        const int p = (g == 0) ? pl[0] : (g == 1) ? pl[1] : (g == 2) ? pl[2] : pl[3];
        float cst;
        if (FLAT) {
          const float sg = (rk < kP) ? -1.f : 1.f;
          cst = fmaf(sg, mm, fmaf(Pk, nzs[p], Lk));
        } else {
          cst = Lk + mm;
        }
        const unsigned long long kk = ((unsigned long long)cost_key(cst) << 32) | (uint32_t)k;
        const unsigned long long old = atomicMin(&bkey[p], kk);
        atomicMin(&skey[p], (uint32_t)(max(old, kk) >> 32));
      }
    }
  }
  __syncthreads();
  // ---- per patch: label, costs, fallback decision
  bool fb = false;
  if (tid < npw) {
    const unsigned long long bk = bkey[tid];
    const uint32_t sk = skey[tid];
    const float b = (bk == ~0ull) ? INFINITY : key_cost((uint32_t)(bk >> 32));
    const float s = (sk == ~0u) ? INFINITY : key_cost(sk);
    const size_t i = (size_t)d.np + base + tid;
    a.labels[i] = (bk == ~0ull) ? 0x7fffffff : (int)(uint32_t)bk;
    if (a.best) a.best[i] = b;
    if (a.second) a.second[i] = s;
    const float gap = (s < INFINITY) ? 0.5f * (s - b) : -INFINITY;
    fb = !(gap >= a.margin);
  }
  // the image's fallback list: one global atomic per workgroup
  const uint64_t mask = __ballot(fb);
  if (lane == 0) wsum[wave] = __popcll(mask);
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int w = 0; w < kRescWaves; ++w) {
      const int v = wsum[w];
      wsum[w] = run;
      run += v;
    }
    fbase = run ? atomicAdd(&a.fb_count[im], run) : 0;
  }
  __syncthreads();
  if (fb) a.fb_list[d.np + fbase + wsum[wave] + __popcll(mask & ((1ull << lane) - 1ull))] = base + tid;
}

// Items of the batched fallback search: pre[i] = sum over images j < i of
// ceil(count[j] / 512), pre[n] the total (one workgroup).
__global__ __launch_bounds__(1024) void fallback_items_kernel(const int32_t* __restrict__ count,
                                                              int n, int32_t* __restrict__ pre) {
  __shared__ int32_t part[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int carry = 0;
  for (int i0 = 0; i0 < n; i0 += 1024) {
    const int i = i0 + threadIdx.x;
    const int v = (i < n) ? (count[i] + 511) / 512 : 0;
    int s = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int u = __shfl_up(s, off);
      if (lane >= off) s += u;
    }
    if (lane == 63) part[wave] = s;
    __syncthreads();
    int pw = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      pw += (w < wave) ? part[w] : 0;
      tot += part[w];
    }
    if (i < n) pre[i] = carry + pw + s - v;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) pre[n] = carry;
}

// One sparse level of the tree descent: the patches grouped by their
// current node (pair ids 8 i from the pair sort with one candidate per
// patch, the node), one wave per tile of up to 128 patches of one node; the
// wave reads each patch's record once, scores the node's children in index
// order (score(): the selection cost of the all-K modes) and keeps the best
// (ties to the lower child), the patch's node at this level.  best /
// second (or NULL): among the node's children.
template <bool FLAT>
__global__ __launch_bounds__(256, 3) void tree_level_bf16_kernel(
    const uint4* __restrict__ zop, const float* __restrict__ znz,
    const uint16_t* __restrict__ Ub, const float* __restrict__ L, const int32_t* __restrict__ rkt,
    const float* __restrict__ Pinv, int K, const int32_t* __restrict__ seg,
    const int32_t* __restrict__ sorted, const uint16_t* __restrict__ children,
    int32_t* __restrict__ labels, float* __restrict__ best, float* __restrict__ second) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;
  const int col = lane & 15;
  const int32_t* start = seg;
  const int32_t* count = seg + (K + 1);
  const int32_t* tinfo = seg + (3 * K + 3);
  const int total = seg[3 * K + 2];
  const uint4* up = reinterpret_cast<const uint4*>(Ub) + lane;
  for (int t = blockIdx.x * 4 + wave; t < total; t += gridDim.x * 4) {
    const int info = tinfo[t];
    const int k = info & 1023;
    const int first = (info >> 10) * kPairTile;
    const int n = min(kPairTile, count[k] - first);
    const int32_t* ids = sorted + start[k] + first;
    int idx[PB];
    bool valid[PB];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const int e = 16 * pb + col;
      valid[pb] = e < n;
      idx[pb] = ids[valid[pb] ? e : 0] >> 3;
    }
    const int own = 4 * (g >> 1) + 2 * (g & 1);
    uint4 zb[PB][2];
    float nzA = 0.f, nzB = 0.f;
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      float nz = 0.f;
      load_operand<FLAT>(zop, znz, idx[pb], g, zb[pb], nz);
      if (FLAT) {
        nzA = (pb == own) ? nz : nzA;
        nzB = (pb == own + 1) ? nz : nzB;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    float bA = INFINITY, sA = INFINITY, bB = INFINITY, sB = INFINITY;
    int kA = 0, kB = 0;
    for (int j = 0; j < 8; ++j) {
      const int c = children[(size_t)k * 8 + j];
      if (c == 0xffff) break;  // (wave-uniform)
      float cA, cB;
      score<FLAT>(up + (size_t)c * 512, zb, L[c], FLAT ? rkt[c] : kP, FLAT ? Pinv[c] : 0.f, nzA,
                  nzB, cA, cB);
      keep_best(cA, c, bA, sA, kA);
      keep_best(cB, c, bB, sB, kB);
    }
#pragma unroll
    for (int pb = 0; pb < PB; pb += 2)
      if (pb == own) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          if (!valid[pb + p]) continue;
          const int i = idx[pb + p];
          labels[i] = p ? kB : kA;
          if (best) best[i] = p ? bB : bA;
          if (second) second[i] = p ? sB : sA;
        }
      }
  }
}

// The one-candidate "pairs" of a tree level: each patch's current node in
// slot 0 (the pair sort then groups the patches by node).
__global__ __launch_bounds__(256) void tree_group_kernel(const int32_t* __restrict__ cur, int Np,
                                                         uint4* __restrict__ cand) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < Np) cand[i] = make_uint4((uint32_t)cur[i] | 0xffff0000u, ~0u, ~0u, ~0u);
}

// The bfloat16 selection operand of every patch of one image as a record
// (8 uint4 per patch, row dy at uint4 dy) and its float32 squared norm --
// load_patch's arithmetic, so a record scores bit for bit as in the all-K
// selection.  A wave covers 16 consecutive patches (lane group g: rows g and
// 4 + g of patch l & 15).
__global__ __launch_bounds__(256) void records_bf16_kernel(const float* __restrict__ x, int H,
                                                           int W, uint4* __restrict__ zop,
                                                           float* __restrict__ znz) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;
  const int Hp = H - 7, Wp = W - 7;
  const int64_t Np = (int64_t)Hp * Wp;
  const int64_t p0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (p0 >= Np) return;  // (wave-uniform)
  const int64_t p = min(p0 + col, Np - 1);
  const int r = (int)(p / Wp), c = (int)(p - (int64_t)r * Wp);
  uint4 zb[2];
  float nz = 0.f;
  load_patch<true>(x, W, r, c, g, zb, nz);
  if (p0 + col < Np) {
    zop[p * 8 + g] = zb[0];
    zop[p * 8 + 4 + g] = zb[1];
    if (g == 0) znz[p] = nz;
  }
}


// The top levels of the tree descent, dense: the spatial all-K loop over
// the listed nodes instead of the K components (same staging, same score()),
// each lane keeping, per own patch, the best child of its current node.
template <bool FLAT>
__global__ __launch_bounds__(256, 3) void tree_dense_bf16_kernel(TreeDenseArgs a) {
  __shared__ uint4 Ash[2][512];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;
  const int col = lane & 15;
  const int Hp = a.H - 7, Wp = a.W - 7;
  const int ntx = (Wp + kEstCols - 1) / kEstCols;
  const int items = ntx * ((Hp + 3) / 4);
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int tr = item / ntx, tc = item - (item / ntx) * ntx;
    const int r = tr * 4 + wave;
    const int c0 = tc * (16 * PB);
    int idx[PB];
    bool valid[PB];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const int c = c0 + 16 * pb + col;
      valid[pb] = (r < Hp) && (c < Wp);
      idx[pb] = min(r, Hp - 1) * Wp + min(c, Wp - 1);
    }
    uint4 zb[PB][2];
    float nzA = 0.f, nzB = 0.f;
    const int own = 4 * (g >> 1) + 2 * (g & 1);
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      float nz = 0.f;
      const int pr = idx[pb] / Wp;
      load_patch<FLAT>(a.x, a.W, pr, idx[pb] - pr * Wp, g, zb[pb], nz);
      if (a.zop && valid[pb]) {  // the records of the levels below
        a.zop[(size_t)idx[pb] * 8 + g] = zb[pb][0];
        a.zop[(size_t)idx[pb] * 8 + 4 + g] = zb[pb][1];
        if (FLAT && g == 0) a.znz[idx[pb]] = nz;
      }
      if (FLAT) {
        nzA = (pb == own) ? nz : nzA;
        nzB = (pb == own + 1) ? nz : nzB;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    int iA = idx[0], iB = idx[1];
    bool vA = valid[0], vB = valid[1];
#pragma unroll
    for (int pb = 0; pb < PB; pb += 2)
      if (pb == own) {
        iA = idx[pb];
        iB = idx[pb + 1];
        vA = valid[pb];
        vB = valid[pb + 1];
      }
    int curA = a.root, curB = a.root;
    float bA = INFINITY, sA = INFINITY, bB = INFINITY, sB = INFINITY;
    int kA = a.root, kB = a.root;
    {
      const uint4* gsrc = reinterpret_cast<const uint4*>(a.Ub);
      const int tid = threadIdx.x;
      int id = a.node[0];
      int rn = FLAT ? a.rk[id] : kP;
      int nu4 = FLAT ? 128 * ((rn + 15) >> 4) : 512;
      uint4 pre0 = make_uint4(0, 0, 0, 0), pre1 = make_uint4(0, 0, 0, 0);
      if (tid < nu4) pre0 = gsrc[(size_t)id * 512 + tid];
      if (256 + tid < nu4) pre1 = gsrc[(size_t)id * 512 + 256 + tid];
      int lev = 0, lend = a.lend[0];
      for (int j = 0; j < a.n; ++j) {
        uint4* As = Ash[j & 1];
        const int k = id, rk = rn;
        if (tid < nu4) As[tid] = pre0;
        if (256 + tid < nu4) As[256 + tid] = pre1;
        __syncthreads();
        if (j + 1 < a.n) {
          id = a.node[j + 1];
          rn = FLAT ? a.rk[id] : kP;
          nu4 = FLAT ? 128 * ((rn + 15) >> 4) : 512;
          if (tid < nu4) pre0 = gsrc[(size_t)id * 512 + tid];
          if (256 + tid < nu4) pre1 = gsrc[(size_t)id * 512 + 256 + tid];
        }
        float cA, cB;
        score<FLAT>(As + lane, zb, a.L[k], rk, FLAT ? a.Pinv[k] : 0.f, nzA, nzB, cA, cB);
        const int p = a.par[j];
        if (p == curA) keep_best(cA, k, bA, sA, kA);
        if (p == curB) keep_best(cB, k, bB, sB, kB);
        if (j + 1 == lend) {  // the level's end: move down (children in index order)
          curA = kA;
          curB = kB;
          if (++lev < a.nlev) {
            lend = a.lend[lev];
            bA = sA = bB = sB = INFINITY;
          }
        }
      }
      __syncthreads();  // the staging buffers are reused by the next item
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (!(p ? vB : vA)) continue;
      const int i = p ? iB : iA;
      a.labels[i] = p ? curB : curA;
      if (a.best) a.best[i] = p ? bB : bA;
      if (a.second) a.second[i] = p ? sB : sA;
    }
  }
}

hipError_t launch_tree_dense_bf16(const TreeDenseArgs& a, hipStream_t st) {
  const int Hp = a.H - 7, Wp = a.W - 7;
  const int items = ((Wp + kEstCols - 1) / kEstCols) * ((Hp + 3) / 4);
  const int blocks = std::min(items, 768);
  if (blocks < 1 || a.n < 1) return hipSuccess;
  if (a.rk)
    hipLaunchKernelGGL(tree_dense_bf16_kernel<true>, dim3(blocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(tree_dense_bf16_kernel<false>, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_records_bf16(const float* x, int H, int W, uint16_t* zop, float* znz,
                               hipStream_t st) {
  const int64_t Np = (int64_t)(H - 7) * (W - 7);
  const int64_t waves = (Np + 15) / 16;
  hipLaunchKernelGGL(records_bf16_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, x,
                     H, W, reinterpret_cast<uint4*>(zop), znz);
  return hipGetLastError();
}

hipError_t launch_tree_level_bf16(const int32_t* cur, int Np, const uint16_t* zop,
                                  const float* znz, const uint16_t* Ub_t, const float* L32_t,
                                  const int32_t* rk, const float* Pinv_t, int K,
                                  const uint16_t* children, uint16_t* cand, int32_t* hist,
                                  int32_t* seg, int32_t* sorted, int32_t* labels, float* best,
                                  float* second, hipStream_t st) {
  hipLaunchKernelGGL(tree_group_kernel, dim3((Np + 255) / 256), dim3(256), 0, st, cur, Np,
                     reinterpret_cast<uint4*>(cand));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_pair_bucket(cand, Np, 1, K, hist, seg, sorted, st)) != hipSuccess) return e;
  // the tile total depends on the labels: a fixed grid walks the device list
  int64_t blocks = ((int64_t)Np / kPairTile + K + 3) / 4;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  const uint4* z4 = reinterpret_cast<const uint4*>(zop);
  if (rk)
    hipLaunchKernelGGL(tree_level_bf16_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, st, z4,
                       znz, Ub_t, L32_t, rk, Pinv_t, K, seg, sorted, children, labels, best,
                       second);
  else
    hipLaunchKernelGGL(tree_level_bf16_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st, z4,
                       znz, Ub_t, L32_t, rk, Pinv_t, K, seg, sorted, children, labels, best,
                       second);
  return hipGetLastError();
}


// The parts of a split list search, merged in component order: part p + 1
// holds higher components than part p, so over the parts in order the best
// is the first strict improvement (ties stay with the lower component) and
// the second is the second smallest of all the costs, exactly as one
// keep_best pass over all K would leave them.
__global__ __launch_bounds__(256) void fallback_merge_kernel(BF16Args a) {
  const int nitems = a.item_pre[a.n_img];
  const int S = a.ksplit;
  const size_t ps = (size_t)S * a.part_stride;
  for (int li = blockIdx.x; li < nitems; li += gridDim.x) {
    int lo = 0, hi = a.n_img - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.item_pre[mid] <= li)
        lo = mid;
      else
        hi = mid - 1;
    }
    const ImgDesc d = a.d[lo];
    const int nl = a.list_count[lo];
    const int lbase = (li - a.item_pre[lo]) * 512;
    for (int j = threadIdx.x; j < 512; j += 256) {
      const int e = lbase + j;
      if (e >= nl) continue;
      const int i = a.list[d.np + e];
      const int32_t* q = a.part_out + d.np + e;
      int k = q[0];
      float b = __int_as_float(q[ps]), s = __int_as_float(q[2 * ps]);
      for (int p = 1; p < S; ++p) {
        const int kp = q[p * a.part_stride];
        const float bp = __int_as_float(q[ps + p * a.part_stride]);
        const float sp = __int_as_float(q[2 * ps + p * a.part_stride]);
        if (bp < b) {
          s = fminf(b, sp);
          b = bp;
          k = kp;
        } else {
          s = fminf(s, bp);
        }
      }
      a.labels[d.np + i] = k;
      if (a.best) a.best[d.np + i] = b;
      if (a.second) a.second[d.np + i] = s;
    }
  }
}

hipError_t launch_fallback_merge(const BF16Args& args, hipStream_t st) {
  if (args.ksplit < 2 || args.blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(fallback_merge_kernel, dim3((unsigned)args.blocks), dim3(256), 0, st, args);
  return hipGetLastError();
}

hipError_t launch_estep_bf16_mode(int mode, const BF16Args& args, hipStream_t st) {
  if (mode == kModeListBatch) {
    // a fixed grid over the items of all images (their total is on the device)
    int blocks = args.blocks;
    if (blocks < 1) return hipSuccess;
    if (args.rk)
      hipLaunchKernelGGL((estep_bf16_kernel<kModeListBatch, true>), dim3(blocks), dim3(256), 0, st,
                         args);
    else
      hipLaunchKernelGGL((estep_bf16_kernel<kModeListBatch, false>), dim3(blocks), dim3(256), 0,
                         st, args);
    return hipGetLastError();
  }
  if (mode == kModeListFull) {
    const int Np = (args.H - 7) * (args.W - 7);
    int blocks = (Np + 511) / 512;
    if (blocks > 512) blocks = 512;
    if (args.rk)
      hipLaunchKernelGGL((estep_bf16_kernel<kModeListFull, true>), dim3(blocks), dim3(256), 0, st,
                         args);
    else
      hipLaunchKernelGGL((estep_bf16_kernel<kModeListFull, false>), dim3(blocks), dim3(256), 0,
                         st, args);
    return hipGetLastError();
  }
  // persistent: a fixed number of workgroups looping over the tiles
  int blocks = args.n_est;
  if (args.blocks > 0 && args.blocks < blocks) blocks = args.blocks;
  if (blocks < 1) return hipSuccess;
  if (args.rk)
    hipLaunchKernelGGL((estep_bf16_kernel<kModeSpatialFull, true>), dim3(blocks), dim3(256), 0,
                       st, args);
  else
    hipLaunchKernelGGL((estep_bf16_kernel<kModeSpatialFull, false>), dim3(blocks), dim3(256), 0,
                       st, args);
  return hipGetLastError();
}

hipError_t launch_rescore_batch(const RescoreArgs& a, int n_tiles, hipStream_t st) {
  if (n_tiles < 1) return hipSuccess;
  if (a.rk)
    hipLaunchKernelGGL(rescore_bf16_kernel<true>, dim3((unsigned)n_tiles), dim3(kRescThreads), 0, st,
                       a);
  else
    hipLaunchKernelGGL(rescore_bf16_kernel<false>, dim3((unsigned)n_tiles), dim3(kRescThreads), 0,
                       st, a);
  return hipGetLastError();
}

hipError_t launch_fallback_items(const int32_t* count, int n, int32_t* pre, hipStream_t st) {
  hipLaunchKernelGGL(fallback_items_kernel, dim3(1), dim3(1024), 0, st, count, n, pre);
  return hipGetLastError();
}

hipError_t launch_estep_bf16_batch(const Batch& b, const float* x, const uint16_t* Ub,
                                   const float* L32, const int32_t* rk, const float* Pinv, int K,
                                   int t, int32_t* labels, float* best, float* second, int blocks,
                                   hipStream_t st) {
  BF16Args a{};
  a.rk = rk;
  a.Pinv = Pinv;
  a.blocks = blocks;
  a.x = x;
  a.Ub = Ub;
  a.L = L32;
  a.K = K;
  a.labels = labels;
  a.best = best;
  a.second = second;
  a.d = b.d;
  a.est_img = b.est_img;
  a.n_est = b.n_est;
  a.t = t;
  return launch_estep_bf16_mode(kModeSpatialFull, a, st);
}

}  // namespace fepll
