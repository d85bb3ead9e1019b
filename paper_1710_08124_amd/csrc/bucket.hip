// Counting sort of patch indices by their selected component, and the tile
// list of the grouped patch-estimation GEMM.
//
// Patch estimation (Alg. 1) applies the Wiener filter of the chosen
// component to each patch.  Grouping the patches by component turns the
// per-patch 64x64 products into one dense GEMM per component (each filter
// is loaded once per tile of kWienerTile patches instead of once per patch).
//
// Four launches over a batch of images, no atomics on global data (LDS
// counters only); every image is sorted on its own:
//  1. hist:    per block of kSortBlock patches, a per-component count
//              (workgroup-local LDS counters), stored component-major.
//  2. scan:    one workgroup per image turns the counts into exclusive offsets
//              (component-major, so a component's patches are contiguous and
//              ordered by block), and derives per component its start, its
//              count and the exclusive prefix of its tile count.
//  3. scatter: every block writes its patch indices into its slots of each
//              component's range, slots handed out by LDS counters.  The
//              order inside a range is not fixed, and need not be: a patch's
//              estimate depends only on its own pixels and its component
//              (every MFMA output column is computed independently), so the
//              estimates written are the same whatever tile a patch lands in.
//  4. wbase:   the first Wiener tile of each image across the batch.
#include "common.h"

namespace fepll {

// Sort block blockIdx.x of the batch: its image, the image's patch count,
// its number of sort blocks and the block's index within the image.
struct SortBlock {
  ImgDesc d;
  int Np, nb, lb;
};
__device__ __forceinline__ SortBlock sort_block(const Batch& b) {
  SortBlock s;
  s.d = b.d[b.sort_img[blockIdx.x]];
  s.Np = (s.d.H - 7) * (s.d.W - 7);
  s.nb = (s.Np + kSortBlock - 1) / kSortBlock;
  s.lb = blockIdx.x - s.d.sort0;
  return s;
}

__global__ __launch_bounds__(1024) void hist_kernel(Batch b, const int32_t* __restrict__ labels_b,
                                                    int K, int32_t* __restrict__ hist_b) {
  extern __shared__ int32_t h[];
  const SortBlock sb = sort_block(b);
  const int32_t* labels = labels_b + sb.d.np;
  int32_t* hist = hist_b + (size_t)K * sb.d.sort0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) h[k] = 0;
  __syncthreads();
  const int base = sb.lb * kSortBlock;
  for (int i = threadIdx.x; i < kSortBlock; i += blockDim.x) {
    const int g = base + i;
    if (g < sb.Np) atomicAdd(&h[labels[g]], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) hist[(size_t)k * sb.nb + sb.lb] = h[k];
}

// Exclusive scan of the inclusive per-thread totals held in s[0..n), n <= 1024.
__device__ void block_exclusive_scan(int32_t* s, int n) {
  const int t = threadIdx.x;
  for (int off = 1; off < 1024; off <<= 1) {
    int32_t v = 0;
    if (t < n && t >= off) v = s[t - off];
    __syncthreads();
    if (t < n) s[t] += v;
    __syncthreads();
  }
  int32_t ex = 0;
  if (t < n) ex = (t == 0) ? 0 : s[t - 1];
  __syncthreads();
  if (t < n) s[t] = ex;
  __syncthreads();
}

// Exclusive offsets of K x nb block counts (component-major, in place),
// then per component its start, count and tile prefix (tiles of `tile`
// entries), the total and the tile table (entry t = k | (tile index in k) << 10)
// in seg; N entries in all.  Called by one whole workgroup of 1024 threads.
__device__ void scan_segments(int32_t* __restrict__ hist, int K, int nb, int N, int tile,
                              int32_t* __restrict__ seg) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int M = K * nb;
  const int chunk = (M + 1023) / 1024;
  const int lo = min(M, t * chunk), hi = min(M, lo + chunk);
  int32_t sum = 0;
#pragma unroll 8
  for (int i = lo; i < hi; ++i) sum += hist[i];
  part[t] = sum;
  __syncthreads();
  block_exclusive_scan(part, 1024);
  int32_t run = part[t];
#pragma unroll 8
  for (int i = lo; i < hi; ++i) {
    const int32_t v = hist[i];
    hist[i] = run;
    run += v;
  }
  __syncthreads();
  __threadfence_block();
  // per-component start / count / tile prefix
  int32_t* start = seg;
  int32_t* count = seg + (K + 1);
  int32_t* tpre = seg + (2 * K + 1);
  __shared__ int32_t tiles[1024];
  for (int k = t; k < K; k += 1024) {
    const int32_t s = hist[(size_t)k * nb];
    const int32_t e = (k + 1 < K) ? hist[(size_t)(k + 1) * nb] : N;
    start[k] = s;
    count[k] = e - s;
    tiles[k] = (e - s + tile - 1) / tile;
  }
  if (t == 0) start[K] = N;
  __syncthreads();
  // K <= 1024: one scan of the tile counts
  int32_t mine = (t < K) ? tiles[t] : 0;
  __syncthreads();
  part[t] = mine;
  __syncthreads();
  // inclusive scan
  for (int off = 1; off < 1024; off <<= 1) {
    int32_t v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  if (t < K) tpre[t] = part[t] - mine;
  if (t == 1023) {
    tpre[K] = part[1023];
    seg[3 * K + 2] = part[1023];
  }
  // tile table: tile -> (component, index of the tile within the component)
  __shared__ int32_t tp[1025];
  for (int k = t; k <= K; k += 1024) tp[k] = (k < K) ? part[k] - tiles[k] : part[1023];
  __syncthreads();
  const int total = tp[K];
  int32_t* info = seg + (3 * K + 3);
  for (int tl = t; tl < total; tl += 1024) {
    int lo2 = 0, hi2 = K - 1;  // last k with tp[k] <= tl
    while (lo2 < hi2) {
      const int mid = (lo2 + hi2 + 1) >> 1;
      if (tp[mid] <= tl) lo2 = mid;
      else hi2 = mid - 1;
    }
    info[tl] = lo2 | ((tl - tp[lo2]) << 10);
  }
}

// One workgroup per image of the batch.
__global__ __launch_bounds__(1024) void scan_kernel(Batch b, int32_t* __restrict__ hist_b, int K,
                                                    int32_t* __restrict__ seg_b) {
  const ImgDesc d = b.d[blockIdx.x];
  const int Np = (d.H - 7) * (d.W - 7);
  const int nb = (Np + kSortBlock - 1) / kSortBlock;
  scan_segments(hist_b + (size_t)K * d.sort0, K, nb, Np, kWienerTile, seg_b + d.seg);
}

__global__ __launch_bounds__(1024) void scatter_kernel(Batch b, const int32_t* __restrict__ labels_b,
                                                       int K, const int32_t* __restrict__ offs_b,
                                                       int32_t* __restrict__ perm_b) {
  extern __shared__ int32_t cur[];  // [K] next free slot of each component in this block
  const SortBlock sb = sort_block(b);
  const int32_t* labels = labels_b + sb.d.np;
  const int32_t* offs = offs_b + (size_t)K * sb.d.sort0;
  int32_t* perm = perm_b + sb.d.np;
  for (int k = threadIdx.x; k < K; k += blockDim.x) cur[k] = offs[(size_t)k * sb.nb + sb.lb];
  __syncthreads();
  const int base = sb.lb * kSortBlock;
  for (int i = threadIdx.x; i < kSortBlock; i += blockDim.x) {
    const int g = base + i;
    if (g < sb.Np) perm[atomicAdd(&cur[labels[g]], 1)] = g;
  }
}

// First Wiener tile of each image across the batch (exclusive prefix of the
// per-image totals), one workgroup.
__global__ __launch_bounds__(1024) void wbase_kernel(Batch b, int K,
                                                     const int32_t* __restrict__ seg_b,
                                                     int32_t* __restrict__ wbase) {
  __shared__ int32_t part[1024];
  int32_t carry = 0;
  for (int i0 = 0; i0 < b.n; i0 += 1024) {
    const int i = i0 + threadIdx.x;
    const int32_t v = (i < b.n) ? seg_b[b.d[i].seg + 3 * K + 2] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int32_t u = (threadIdx.x >= off) ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += u;
      __syncthreads();
    }
    if (i < b.n) wbase[i] = carry + part[threadIdx.x] - v;
    const int32_t tot = part[1023];
    __syncthreads();
    carry += tot;
  }
  if (threadIdx.x == 0) wbase[b.n] = carry;
}

// ---- (patch, candidate) pairs of the proposal, sorted by component for
// the exact rescoring: pair p = 8 i + j is candidate j < m of patch i.

__global__ __launch_bounds__(1024) void pair_hist_kernel(const uint16_t* __restrict__ cand, int Np,
                                                         int m, int K, int nb,
                                                         int32_t* __restrict__ hist) {
  extern __shared__ int32_t h[];
  for (int k = threadIdx.x; k < K; k += blockDim.x) h[k] = 0;
  __syncthreads();
  const int base = blockIdx.x * kPairBlock;
  for (int e = threadIdx.x; e < kPairBlock * m; e += blockDim.x) {
    const int i = base + e / m, j = e - (e / m) * m;
    if (i >= Np) continue;
    const int k = cand[(size_t)i * 8 + j];
    if (k < K) atomicAdd(&h[k], 1);  // (an index >= K is skipped everywhere)
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) hist[(size_t)k * nb + blockIdx.x] = h[k];
}

__global__ __launch_bounds__(1024) void pair_scan_kernel(int32_t* __restrict__ hist, int K, int nb,
                                                         int N, int32_t* __restrict__ seg) {
  scan_segments(hist, K, nb, N, kPairTile, seg);
}

__global__ __launch_bounds__(1024) void pair_scatter_kernel(const uint16_t* __restrict__ cand,
                                                            int Np, int m, int K, int nb,
                                                            const int32_t* __restrict__ offs,
                                                            int32_t* __restrict__ sorted) {
  extern __shared__ int32_t cur[];
  for (int k = threadIdx.x; k < K; k += blockDim.x) cur[k] = offs[(size_t)k * nb + blockIdx.x];
  __syncthreads();
  const int base = blockIdx.x * kPairBlock;
  for (int e = threadIdx.x; e < kPairBlock * m; e += blockDim.x) {
    const int i = base + e / m, j = e - (e / m) * m;
    if (i >= Np) continue;
    const int k = cand[(size_t)i * 8 + j];
    if (k < K) sorted[atomicAdd(&cur[k], 1)] = 8 * i + j;
  }
}

hipError_t launch_pair_bucket(const uint16_t* cand, int Np, int m, int K, int32_t* hist,
                              int32_t* seg, int32_t* sorted, hipStream_t st) {
  const int nb = (Np + kPairBlock - 1) / kPairBlock;
  hipLaunchKernelGGL(pair_hist_kernel, dim3(nb), dim3(1024), K * sizeof(int32_t), st, cand, Np,
                     m, K, nb, hist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pair_scan_kernel, dim3(1), dim3(1024), 0, st, hist, K, nb, Np * m, seg);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pair_scatter_kernel, dim3(nb), dim3(1024), K * sizeof(int32_t), st, cand,
                     Np, m, K, nb, hist, sorted);
  return hipGetLastError();
}

hipError_t launch_bucket_batch(const Batch& b, const int32_t* labels, int K, int32_t* hist,
                               int32_t* seg, int32_t* perm, int32_t* wbase, hipStream_t st) {
  hipLaunchKernelGGL(hist_kernel, dim3(b.n_sort), dim3(1024), K * sizeof(int32_t), st, b, labels,
                     K, hist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_kernel, dim3(b.n), dim3(1024), 0, st, b, hist, K, seg);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scatter_kernel, dim3(b.n_sort), dim3(1024), K * sizeof(int32_t), st, b,
                     labels, K, hist, perm);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(wbase_kernel, dim3(1), dim3(1024), 0, st, b, K, seg, wbase);
  return hipGetLastError();
}

}  // namespace fepll
