// Patch estimation (Alg. 1, "Patch estimation", eigenspace form of Sec. 2.1):
// z^_i = U_k* diag(gamma_k*) U_k*^t z~_i + m_i = W_k* z~_i + m_i, with the
// patch mean m_i added back unshrunk.  W_k is formed once per beta in
// float64 (prep.hip); here it is applied as a grouped GEMM over the patches
// bucketed by component (bucket.hip): one wave takes a tile of up to 32
// patches that share a component, recomputes their DC-removed pixels from
// the current image, multiplies by W_k on MFMA and writes z^ patch-major,
// Zhat[patch][dy][dx].  The patches of a tile lie anywhere in the image, so
// each patch's 256 bytes are the unit of the output.  The patches are the
// matrix product's rows and the pixels its columns (D = Z~ W_k^t), so each
// accumulator register of a half-wave holds 32 consecutive pixels of one
// patch and every store instruction writes two whole 128-byte lines: no
// line is left partly written for the memory to merge or to read back.
//
// The tile count depends on the labels, so the grid is fixed (a multiple of
// 8 workgroups) and each workgroup walks its share of the device-side tile
// list of the whole batch (images one after the other, each image's tiles
// ordered by component); a wave exits at the end of its share.
//
// Two forms: float32 operands on v_mfma_f32_32x32x2f32 (the float32 path:
// 64 products of 64 cycles per 32-patch tile), and, for the reduced-
// precision modes, binary16 operands on v_mfma_f32_32x32x16_f16 with
// float32 accumulation (8 products per tile, about a sixteenth of the
// matrix-core time).
#include "common.h"

namespace fepll {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Accumulator register r of lane (half, col) is pixel 32 qb + col of tile
// row i = 8 (r / 4) + 4 half + r % 4: the 32 lanes of a half write that
// patch's 128 contiguous bytes, one whole line per half per instruction.
// Lanes i and 32 + i hold row i's patch id and mean (id0, m0); the writing
// lanes fetch them by lane permutes, which keeps them out of long-lived
// registers.
__device__ inline void store_rows(float* __restrict__ Zhat, const f32x16& a, int id0, float m0,
                                  int n, int half, int col, int qb) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 8 * (r >> 2) + 4 * half + (r & 3);
    const int id = __shfl(id0, i);
    const float m = __shfl(m0, i);
    if (i < n) Zhat[(size_t)id * kP + 32 * qb + col] = a[r] + m;
  }
}

__global__ __launch_bounds__(256, 4) void wiener_f32_kernel(Batch bt, const float* __restrict__ xb,
                                                         const float4* __restrict__ Wt_all,
                                                         int K, int it,
                                                         const int32_t* __restrict__ seg_b,
                                                         const int32_t* __restrict__ perm_b,
                                                         const int32_t* __restrict__ wbase,
                                                         float* __restrict__ Zhat_b) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int total = wbase[bt.n];
  // Each workgroup takes a contiguous range of tiles (tiles are ordered by
  // image, then octile of the image's rows, then component, so a range
  // mostly shares one W_k, which then stays in the CU's L1), and
  // consecutive ranges go to workgroups of the same XCD (workgroups are
  // dealt round-robin over the 8 XCDs), so each XCD's L2 holds the filters
  // and the image rows of only its part of the list.
  // With fewer tiles than the grid has waves (a patch subset), only the
  // workgroups needed for one tile per wave take part, still dealt over all
  // 8 XCDs.  (The grid is a multiple of 8.)
  const int G = min((int)gridDim.x, max(8, (((total + 3) >> 2) + 7) & ~7));
  if ((int)blockIdx.x >= G) return;
  const int lb = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int per = (total + G - 1) / G;
  const int t_end = min(total, (lb + 1) * per);
  int t = lb * per + (threadIdx.x >> 6);
  if (t >= t_end) return;
  int im = image_of(wbase, bt.n, t);
  for (; t < t_end; t += 4) {
    while (t >= wbase[im + 1]) ++im;
    const ImgDesc d = bt.d[im];
    const int W = d.W, Wp = d.W - 7;
    const float* x = xb + d.px;
    const int32_t* seg = seg_b + d.seg;
    const int32_t* start = seg;
    const int32_t* count = seg + (K + 1);
    const int32_t* tinfo = seg + (3 * K + 3);
    const float4* Wt = Wt_all + (size_t)(d.slot0 + it) * K * 1024;
    float* Zhat = Zhat_b + (size_t)d.np * kP;
    // component of tile t and the tile's index within the component
    const int info = tinfo[t - wbase[im]];
    const int k = info & 1023;
    const int first = (info >> 10) * kWienerTile;
    const int n = min(kWienerTile, count[k] - first);
    const int32_t* ids = perm_b + d.np + start[k] + first;

    // patches: lane holds pixels 32 half + s (s = 0..31) -- patch rows
    // 4 half .. 4 half + 3, read as float4 -- of patch col
    const bool v0 = col < n;
    const int id0 = v0 ? ids[col] : ids[0];
    const int r0 = id0 / Wp, c0 = id0 - r0 * Wp;
    float z0[32];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const float* p0 = x + (size_t)(r0 + 4 * half + rr) * W + c0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float4 a;
        __builtin_memcpy(&a, p0 + 4 * h, 16);
        const int o = 8 * rr + 4 * h;
        z0[o] = a.x;
        z0[o + 1] = a.y;
        z0[o + 2] = a.z;
        z0[o + 3] = a.w;
      }
    }
    double s0 = 0.0;
#pragma unroll
    for (int s = 0; s < 32; ++s) s0 += (double)z0[s];
    s0 += __shfl_xor(s0, 32);
    const double m0 = s0 * (1.0 / 64.0);
#pragma unroll
    for (int s = 0; s < 32; ++s) z0[s] = (float)((double)fresh(z0[s]) - m0);
    const float fm0 = (float)m0;
    // one 32-column block of W_k^t at a time (pixels q = 32 qb + col)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
      const float4* wp = Wt + (size_t)k * 1024 + qb * 512 + lane;
      float4 A[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) A[i] = wp[i * 64];
      f32x16 a0 = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        a0 = __builtin_amdgcn_mfma_f32_32x32x2f32(z0[4 * i + 0], A[i].x, a0, 0, 0, 0);
        a0 = __builtin_amdgcn_mfma_f32_32x32x2f32(z0[4 * i + 1], A[i].y, a0, 0, 0, 0);
        a0 = __builtin_amdgcn_mfma_f32_32x32x2f32(z0[4 * i + 2], A[i].z, a0, 0, 0, 0);
        a0 = __builtin_amdgcn_mfma_f32_32x32x2f32(z0[4 * i + 3], A[i].w, a0, 0, 0, 0);
      }
      store_rows(Zhat, a0, id0, fm0, n, half, col, qb);
    }
  }
}

// The reduced-precision form: the same tile walk; per tile the lane (half
// h, column col) holds rows h, 2 + h, 4 + h, 6 + h of patch col, depth step
// s of v_mfma_f32_32x32x16_f16 taking row 2 s + h (pixels 16 s + 8 h + e),
// the DC-removed pixels rounded once from float32 to binary16; the B operand
// is the binary16 table Wh (column block qb, depth step s); the accumulator
// layout is the float32 form's, so are the stores.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
__global__ __launch_bounds__(256, 5) void wiener_f16_kernel(Batch bt, const float* __restrict__ xb,
                                                         const uint4* __restrict__ Wh_all, int K,
                                                         int it, const int32_t* __restrict__ seg_b,
                                                         const int32_t* __restrict__ perm_b,
                                                         const int32_t* __restrict__ wbase,
                                                         float* __restrict__ Zhat_b) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int total = wbase[bt.n];
  const int G = min((int)gridDim.x, max(8, (((total + 3) >> 2) + 7) & ~7));
  if ((int)blockIdx.x >= G) return;
  const int lb = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int per = (total + G - 1) / G;
  const int t_end = min(total, (lb + 1) * per);
  int t = lb * per + (threadIdx.x >> 6);
  if (t >= t_end) return;
  int im = image_of(wbase, bt.n, t);
  for (; t < t_end; t += 4) {
    while (t >= wbase[im + 1]) ++im;
    const ImgDesc d = bt.d[im];
    const int W = d.W, Wp = d.W - 7;
    const float* x = xb + d.px;
    const int32_t* seg = seg_b + d.seg;
    const int32_t* start = seg;
    const int32_t* count = seg + (K + 1);
    const int32_t* tinfo = seg + (3 * K + 3);
    const uint4* Wh = Wh_all + (size_t)(d.slot0 + it) * K * 512;
    float* Zhat = Zhat_b + (size_t)d.np * kP;
    const int info = tinfo[t - wbase[im]];
    const int k = info & 1023;
    const int first = (info >> 10) * kWienerTile;
    const int n = min(kWienerTile, count[k] - first);
    const int32_t* ids = perm_b + d.np + start[k] + first;
    const bool v0 = col < n;
    const int id0 = v0 ? ids[col] : ids[0];
    const int r0 = id0 / Wp, c0 = id0 - r0 * Wp;
    float z[4][8];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float* p0 = x + (size_t)(r0 + 2 * s + half) * W + c0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float4 a;
        __builtin_memcpy(&a, p0 + 4 * h, 16);
        z[s][4 * h] = a.x;
        z[s][4 * h + 1] = a.y;
        z[s][4 * h + 2] = a.z;
        z[s][4 * h + 3] = a.w;
      }
    }
    double s0 = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) s0 += (double)z[s][e];
    s0 += __shfl_xor(s0, 32);
    const double m0 = s0 * (1.0 / 64.0);
    f16x8 zb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        // rounded to float32, then to binary16 (two roundings, as defined;
        // fresh() keeps the compiler from fusing them into one)
        const float d32 = (float)((double)fresh(z[s][e]) - m0);
        zb[s][e] = (_Float16)fresh(d32);
      }
    const float fm0 = (float)m0;
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
      const uint4* wp = Wh + (size_t)k * 512 + qb * 256 + lane;
      uint4 A[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) A[s] = wp[s * 64];
      f32x16 a0 = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4; ++s)
        a0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(zb[s], __builtin_bit_cast(f16x8, A[s]), a0,
                                                    0, 0, 0);
      store_rows(Zhat, a0, id0, fm0, n, half, col, qb);
    }
  }
}

hipError_t launch_wiener_batch(const Batch& b, const float* x, const float* Wt,
                               const uint16_t* Wh, int K, int t, const int32_t* seg,
                               const int32_t* perm, const int32_t* wbase, float* Zhat,
                               int max_blocks, hipStream_t st) {
  // tile total <= patches / tile + K per image
  const int64_t max_tiles = b.n_patches / kWienerTile + (int64_t)K * b.n;
  int64_t blocks = (max_tiles + 3) / 4;
  if (blocks > max_blocks) blocks = max_blocks;
  blocks = (blocks + 7) & ~7;  // whole rounds over the 8 XCDs
  if (Wh)
    hipLaunchKernelGGL(wiener_f16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, b, x,
                       reinterpret_cast<const uint4*>(Wh), K, t, seg, perm, wbase, Zhat);
  else
    hipLaunchKernelGGL(wiener_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, b, x,
                       reinterpret_cast<const float4*>(Wt), K, t, seg, perm, wbase, Zhat);
  return hipGetLastError();
}

}  // namespace fepll
