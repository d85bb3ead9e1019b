// Jittered stochastic patch subsampling (Sec. 3.3): the patches of one
// iteration are the points of a grid of spacing s, shifted as a whole by a
// random offset, each point moved independently and uniformly by at most
// b = floor((8 - s) / 2) pixels per direction and clamped to the image, so
// that every pixel stays covered; positions are drawn again at every
// iteration.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011),
// key = the 64-bit seed, counter (t, a, c, 0) for grid point (a, c) of
// iteration t (word 0 moves the row, word 1 the column) and
// (t, 0xffffffff, 0xffffffff, 0) for the shift; uniform integers in
// {0..n-1} as the word modulo n.  Grid rows: i0 = g - s n0 + s a, n0 the
// smallest n with g - s n <= -b, up to the first a with i0 - b >= Hp - 1
// (likewise for columns): consecutive starts differ by at most s + 2 b <= 8
// and the first and last clamp to the image's edges.
//
// After a selection of every patch (float32): two launches per iteration,
// mark (one thread per grid point, flags of the chosen patches set to 1 --
// several points may land on one patch) and compact (the flagged patches
// appended to a list in any order, the others' labels set to K, the "not in
// the subset" mark every later stage reads).  Before a selection of the
// subset alone: one launch, mark appending to the list as it draws, which
// also undoes the previous iteration's list (two flag sets and two lists
// alternate, so the undo and the new marks never touch the same flag).
#include <algorithm>

#include "common.h"

namespace fepll {

namespace {

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
// flag is set by an exchange), and the flags stay set until the next
// iteration's launch (or jitter_reset_kernel) clears them; that launch
// first undoes the previous list (prev, one entry per thread: a list never
// holds more entries than the grid has points) in the other flag set.
// Otherwise only the flags are set and *count zeroed for
// jitter_compact_kernel.
template <bool APPEND>
__global__ __launch_bounds__(256) void jitter_mark_kernel(int H, int W, int s, uint32_t k0,
                                                          uint32_t k1, int t, int amax, int cmax,
                                                          int32_t* __restrict__ flags,
                                                          int32_t* __restrict__ count,
                                                          int32_t* __restrict__ list,
                                                          JitterPrev prev) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (APPEND && prev.list && i < *prev.count) {
    const int q = prev.list[i];
    prev.flags[q] = 0;
    prev.labels[q] = prev.K;
  }
  if (APPEND && prev.zero && i == 0) *prev.zero = 0;
  if (APPEND && prev.clear)
    for (int j = i; j < prev.nclear; j += gridDim.x * blockDim.x) prev.clear[j] = 0;
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

// After an iteration on an appended list: its patches' flags cleared and
// labels set back to K (so every patch not on the next list keeps K), and
// the next iteration's count zeroed.
__global__ __launch_bounds__(256) void jitter_reset_kernel(const int32_t* __restrict__ list,
                                                           const int32_t* __restrict__ count,
                                                           int32_t* __restrict__ next_count,
                                                           int32_t* __restrict__ flags,
                                                           int32_t* __restrict__ labels, int K) {
  const int n = *count;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int p = list[e];
    flags[p] = 0;
    labels[p] = K;
  }
  if (next_count && blockIdx.x == 0 && threadIdx.x == 0) *next_count = 0;
}

// 16 384 patches per workgroup (16 per thread, all flag loads in flight);
// the list slots of the block's chosen patches follow raster order within
// the block (a wave scan over the 16 x 16 wave counts), one global atomic
// per block
constexpr int kCompactPer = 16;

__global__ __launch_bounds__(1024) void jitter_compact_kernel(int Np, int K,
                                                              int32_t* __restrict__ flags,
                                                              int32_t* __restrict__ labels,
                                                              int32_t* __restrict__ count,
                                                              int32_t* __restrict__ list) {
  __shared__ int wcnt[kCompactPer * 16];  // [chunk u][wave], then exclusive offsets
  __shared__ int base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b0 = blockIdx.x * (kCompactPer * 1024) + (int)threadIdx.x;
  bool in[kCompactPer];
#pragma unroll
  for (int u = 0; u < kCompactPer; ++u) {
    const int i = b0 + u * 1024;
    in[u] = i < Np && flags[i] != 0;
  }
#pragma unroll
  for (int u = 0; u < kCompactPer; ++u) {
    const int i = b0 + u * 1024;
    if (in[u])
      flags[i] = 0;  // all zero again for the next marking
    else if (i < Np)
      labels[i] = K;
  }
  uint64_t mask[kCompactPer];
#pragma unroll
  for (int u = 0; u < kCompactPer; ++u) {
    mask[u] = __ballot(in[u]);
    if (lane == 0) wcnt[u * 16 + wave] = __popcll(mask[u]);
  }
  __syncthreads();
  if (wave == 0) {
    // lane l: entries 4 l .. 4 l + 3 of the (u, wave) order
    int v[4], s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = wcnt[4 * lane + q];
      s += v[q];
    }
    int incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(incl, off);
      if (lane >= off) incl += t;
    }
    int run = incl - s;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      wcnt[4 * lane + q] = run;
      run += v[q];
    }
    const int total = __shfl(incl, 63);
    if (lane == 0) base = total ? atomicAdd(count, total) : 0;
  }
  __syncthreads();
  if (!list) return;
  const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
  for (int u = 0; u < kCompactPer; ++u)
    if (in[u]) list[base + wcnt[u * 16 + wave] + __popcll(mask[u] & below)] = b0 + u * 1024;
}

}  // namespace

// Upper bound of the grid points per axis for n patch starts.
static int grid_points_max(int n, int s) { return (n - 1 + 2 * 3 + 2 * s) / s + 2; }

int64_t jitter_points_max(int H, int W, int s) {
  return (int64_t)grid_points_max(H - 7, s) * grid_points_max(W - 7, s);
}

hipError_t launch_jitter_mark(int H, int W, int s, uint64_t seed, int t, int32_t* flags,
                              int32_t* count, int32_t* list, const JitterPrev& prev,
                              hipStream_t st) {
  const int amax = grid_points_max(H - 7, s), cmax = grid_points_max(W - 7, s);
  const int n = amax * cmax;
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  if (list)
    hipLaunchKernelGGL(jitter_mark_kernel<true>, dim3((n + 255) / 256), dim3(256), 0, st, H, W,
                       s, k0, k1, t, amax, cmax, flags, count, list, prev);
  else
    hipLaunchKernelGGL(jitter_mark_kernel<false>, dim3((n + 255) / 256), dim3(256), 0, st, H, W,
                       s, k0, k1, t, amax, cmax, flags, count, list, JitterPrev{});
  return hipGetLastError();
}

hipError_t launch_jitter_reset(const int32_t* list, int64_t list_max, const int32_t* count,
                               int32_t* next_count, int32_t* flags, int32_t* labels, int K,
                               hipStream_t st) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((list_max + 255) / 256, 1024));
  hipLaunchKernelGGL(jitter_reset_kernel, dim3((unsigned)blocks), dim3(256), 0, st, list, count,
                     next_count, flags, labels, K);
  return hipGetLastError();
}

hipError_t launch_jitter_compact(int Np, int K, int32_t* flags, int32_t* labels,
                                 int32_t* count, int32_t* list, hipStream_t st) {
  const int per = kCompactPer * 1024;
  hipLaunchKernelGGL(jitter_compact_kernel, dim3((Np + per - 1) / per), dim3(1024), 0, st, Np, K,
                     flags, labels, count, list);
  return hipGetLastError();
}

}  // namespace fepll
