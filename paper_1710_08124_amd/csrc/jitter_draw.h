// The jittered drawing of one iteration (Sec. 3.3) as a device function, so
// that a drawing can run as extra workgroups of another launch; the
// positions, the random numbers and the grid are described in jitter.hip.
#pragma once
#include "common.h"

namespace fepll {

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += W0;  // (the bump after the last round is unused)
    k1 += W1;
  }
  return c;
}

// first grid coordinate along an axis with shift g: g - s n0, n0 the
// smallest n with g - s n <= -b
__device__ __forceinline__ int grid_first(int g, int s, int b) {
  const int n0 = (g + b + s - 1) / s;
  return g - s * n0;
}

// APPEND: each chosen patch is also appended to list at *count (wave-
// aggregated atomics; a patch two grid points clamp to is taken once: its
// flag is set by an exchange), and the flags stay set until a later
// drawing (or jitter_reset_kernel) clears them; the drawing first undoes
// an earlier list (prev, one entry per thread: a list never holds more
// entries than the grid has points) in another flag set.
// Otherwise only the flags are set and *count zeroed for
// jitter_compact_kernel.
// One workgroup of 256 threads, number blk of nblk, of the drawing a.
template <bool APPEND>
__device__ __forceinline__ void jitter_draw_block(const JitterDraw& dr, int blk, int nblk) {
  const int H = dr.H, W = dr.W, s = dr.s, t = dr.t, amax = dr.amax, cmax = dr.cmax;
  const uint32_t k0 = dr.k0, k1 = dr.k1;
  int32_t* flags = dr.flags;
  int32_t* count = dr.count;
  int32_t* list = dr.list;
  const JitterPrev& prev = dr.prev;
  const int i = blk * 256 + (int)threadIdx.x;
  if (APPEND && prev.list && i < *prev.count) {
    const int q = prev.list[i];
    prev.flags[q] = 0;
    if (prev.labels) prev.labels[q] = prev.K;
  }
  if (APPEND && prev.zero && i == 0) *prev.zero = 0;
  if (APPEND && prev.clear)
    for (int j = i; j < prev.nclear; j += nblk * 256) prev.clear[j] = 0;
  const int Hp = H - 7, Wp = W - 7;
  const int b = (8 - s) / 2;
  const U4 sh = philox4x32_10(U4{(uint32_t)t, 0xffffffffu, 0xffffffffu, 0u}, k0, k1);
  const int fy = grid_first((int)(sh.x % (uint32_t)s), s, b);
  const int fx = grid_first((int)(sh.y % (uint32_t)s), s, b);
  // grid extent: points up to the first one whose lowest start reaches the
  // last patch row / column
  const int na = (Hp - 1 + b - fy + s - 1) / s + 1;
  const int nc = (Wp - 1 + b - fx + s - 1) / s + 1;
  if (!APPEND && i == 0) *count = 0;  // the compaction that follows counts the subset
  const int a = i / cmax, c = i - a * cmax;
  int p = 0;
  bool take = false;
  if (i < amax * cmax && a < na && c < nc) {
    const U4 u = philox4x32_10(U4{(uint32_t)t, (uint32_t)a, (uint32_t)c, 0u}, k0, k1);
    const uint32_t n = (uint32_t)(2 * b + 1);
    const int r = min(max(fy + s * a + (int)(u.x % n) - b, 0), Hp - 1);
    const int q = min(max(fx + s * c + (int)(u.y % n) - b, 0), Wp - 1);
    p = r * Wp + q;
    if (APPEND)
      take = atomicExch(&flags[p], 1) == 0;
    else
      flags[p] = 1;
  }
  if (!APPEND) return;
  // one global atomic per workgroup (ballots, LDS prefix over the 4 waves)
  __shared__ int wcnt[4], wbase;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t mask = __ballot(take);
  if (lane == 0) wcnt[wave] = __popcll(mask);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tot = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    wbase = tot ? atomicAdd(count, tot) : 0;
  }
  __syncthreads();
  int off = wbase;
  for (int w = 0; w < wave; ++w) off += wcnt[w];
  if (take) list[off + __popcll(mask & ((1ull << lane) - 1ull))] = p;
}

}  // namespace fepll
