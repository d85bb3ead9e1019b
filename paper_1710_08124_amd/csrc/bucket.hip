// Counting sort of patch indices by their selected component, and the tile
// list of the grouped patch-estimation GEMM.
//
// Patch estimation (Alg. 1) applies the Wiener filter of the chosen
// component to each patch.  Grouping the patches by component turns the
// per-patch 64x64 products into one dense GEMM per component (each filter
// is loaded once per tile of kWienerTile patches instead of once per patch).
//
// Three launches, no atomics on global data (LDS counters only):
//  1. hist:    per block of kSortBlock patches, a per-component count
//              (workgroup-local LDS counters), stored component-major.
//  2. scan:    one workgroup turns the counts into exclusive offsets
//              (component-major, so a component's patches are contiguous and
//              ordered by block), and derives per component its start, its
//              count and the exclusive prefix of its tile count.
//  3. scatter: every block writes its patch indices into its slots of each
//              component's range, slots handed out by LDS counters.  The
//              order inside a range is not fixed, and need not be: a patch's
//              estimate depends only on its own pixels and its component
//              (every MFMA output column is computed independently), so the
//              estimates written are the same whatever tile a patch lands in.
#include "common.h"

namespace fepll {

__global__ __launch_bounds__(1024) void hist_kernel(const int32_t* __restrict__ labels, int Np,
                                                    int K, int nb, int32_t* __restrict__ hist) {
  extern __shared__ int32_t h[];
  for (int k = threadIdx.x; k < K; k += blockDim.x) h[k] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortBlock;
  for (int i = threadIdx.x; i < kSortBlock; i += blockDim.x) {
    const int g = base + i;
    if (g < Np) atomicAdd(&h[labels[g]], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) hist[(size_t)k * nb + blockIdx.x] = h[k];
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

__global__ __launch_bounds__(1024) void scan_kernel(int32_t* __restrict__ hist, int K, int nb,
                                                    int Np, int32_t* __restrict__ seg) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int M = K * nb;
  const int chunk = (M + 1023) / 1024;
  const int lo = min(M, t * chunk), hi = min(M, lo + chunk);
  int32_t sum = 0;
  for (int i = lo; i < hi; ++i) sum += hist[i];
  part[t] = sum;
  __syncthreads();
  block_exclusive_scan(part, 1024);
  int32_t run = part[t];
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
    const int32_t e = (k + 1 < K) ? hist[(size_t)(k + 1) * nb] : Np;
    start[k] = s;
    count[k] = e - s;
    tiles[k] = (e - s + kWienerTile - 1) / kWienerTile;
  }
  if (t == 0) start[K] = Np;
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
  for (int tile = t; tile < total; tile += 1024) {
    int lo = 0, hi = K - 1;  // last k with tp[k] <= tile
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tp[mid] <= tile) lo = mid;
      else hi = mid - 1;
    }
    info[tile] = lo | ((tile - tp[lo]) << 10);
  }
}

__global__ __launch_bounds__(1024) void scatter_kernel(const int32_t* __restrict__ labels, int Np,
                                                       int K, int nb,
                                                       const int32_t* __restrict__ offs,
                                                       int32_t* __restrict__ perm) {
  extern __shared__ int32_t cur[];  // [K] next free slot of each component in this block
  for (int k = threadIdx.x; k < K; k += blockDim.x) cur[k] = offs[(size_t)k * nb + blockIdx.x];
  __syncthreads();
  const int base = blockIdx.x * kSortBlock;
  for (int i = threadIdx.x; i < kSortBlock; i += blockDim.x) {
    const int g = base + i;
    if (g < Np) perm[atomicAdd(&cur[labels[g]], 1)] = g;
  }
}

hipError_t launch_bucket(const int32_t* labels, int Np, int K, int32_t* hist, int32_t* seg,
                         int32_t* perm, hipStream_t st) {
  const int nb = (Np + kSortBlock - 1) / kSortBlock;
  hipLaunchKernelGGL(hist_kernel, dim3(nb), dim3(1024), K * sizeof(int32_t), st, labels, Np, K, nb,
                     hist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, hist, K, nb, Np, seg);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scatter_kernel, dim3(nb), dim3(1024), K * sizeof(int32_t), st, labels, Np,
                     K, nb, hist, perm);
  return hipGetLastError();
}

}  // namespace fepll
