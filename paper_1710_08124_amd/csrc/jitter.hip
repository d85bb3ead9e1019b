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
// also undoes an earlier iteration's list (three flag sets and lists
// alternate, so the undo and the new marks never touch the same flag);
// the same drawing can also run inside the subset reprojection
// (jitter_draw.h).
#include <algorithm>

#include "jitter_draw.h"

namespace fepll {

namespace {

template <bool APPEND>
__global__ __launch_bounds__(256) void jitter_mark_kernel(JitterDraw a) {
  jitter_draw_block<APPEND>(a, blockIdx.x, gridDim.x);
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

JitterDraw make_jitter_draw(int H, int W, int s, uint64_t seed, int t, int32_t* flags,
                            int32_t* count, int32_t* list, const JitterPrev& prev, int* blocks) {
  JitterDraw a;
  a.H = H;
  a.W = W;
  a.s = s;
  a.k0 = (uint32_t)(seed & 0xffffffffu);
  a.k1 = (uint32_t)(seed >> 32);
  a.t = t;
  a.amax = grid_points_max(H - 7, s);
  a.cmax = grid_points_max(W - 7, s);
  a.flags = flags;
  a.count = count;
  a.list = list;
  a.prev = prev;
  *blocks = (a.amax * a.cmax + 255) / 256;
  return a;
}

hipError_t launch_jitter_mark(int H, int W, int s, uint64_t seed, int t, int32_t* flags,
                              int32_t* count, int32_t* list, const JitterPrev& prev,
                              hipStream_t st) {
  int blocks = 0;
  const JitterDraw a =
      make_jitter_draw(H, W, s, seed, t, flags, count, list, list ? prev : JitterPrev{}, &blocks);
  if (list)
    hipLaunchKernelGGL(jitter_mark_kernel<true>, dim3(blocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(jitter_mark_kernel<false>, dim3(blocks), dim3(256), 0, st, a);
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
