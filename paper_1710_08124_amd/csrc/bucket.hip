// Counting sort of patch indices by their selected component, and the tile
// list of the grouped patch-estimation GEMM.
//
// Patch estimation (Alg. 1) applies the Wiener filter of the chosen
// component to each patch.  Grouping the patches by component turns the
// per-patch 64x64 products into one dense GEMM per component (each filter
// is loaded once per tile of kWienerTile patches instead of once per patch).
//
// Launches over a batch of images, no atomics on global data (LDS counters
// only); every image is sorted on its own:
//  1. hist:    per block of kSortBlock patches, a per-component count
//              (workgroup-local LDS counters), stored component-major.
//  2. tables:  the counts become exclusive offsets within each component
//              (component-major, so a component's patches are contiguous and
//              ordered by block), and per component its start, its count and
//              the exclusive prefix of its tile count, plus the tile table
//              (three launches, parallel over components and tiles).
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
  // the block's labels, all loads in flight (label K: not in the patch subset)
  const int base = sb.lb * kSortBlock;
  int lab[kSortBlock / 1024];
#pragma unroll
  for (int u = 0; u < kSortBlock / 1024; ++u) {
    const int g = base + u * 1024 + (int)threadIdx.x;
    lab[u] = (g < sb.Np) ? labels[g] : K;
  }
#pragma unroll
  for (int u = 0; u < kSortBlock / 1024; ++u)
    if (lab[u] < K) atomicAdd(&h[lab[u]], 1);
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) hist[(size_t)k * sb.nb + sb.lb] = h[k];
}

// ---- segment tables, in three parallel launches (shared by the Wiener
// sort and the pair rescoring).  A problem is K x nb block counts at hist
// (component-major) and its table seg (start[K+1], count[K],
// tile_prefix[K+1], total tiles, tile table); `tile` entries per tile.
//  A. one workgroup per (component, problem): exclusive scan of the
//     component's nb block counts in place -> offsets within the component,
//     and count[k];
//  B. one workgroup per problem: start[k] and the tile prefix (K <= 1024);
//  C. one thread per tile: the tile table, entry t = k | (tile in k) << 10.
// The scatter adds start[k] to the offsets of A.

struct SegProblem {
  int32_t* hist;
  int32_t* seg;
  int nb;
};
// problem blockIdx.y: an image of the batch (BATCH: blocks of kSortBlock
// patches), or the one problem given by (hist, seg, nb)
template <bool BATCH>
__device__ __forceinline__ SegProblem seg_problem(const Batch& b, int32_t* hist, int32_t* seg,
                                                  int nb, int K) {
  if (!BATCH) return {hist, seg, nb};
  const ImgDesc d = b.d[blockIdx.y];
  const int Np = (d.H - 7) * (d.W - 7);
  return {hist + (size_t)K * d.sort0, seg + d.seg, (Np + kSortBlock - 1) / kSortBlock};
}

// inclusive scan of v over a workgroup of 256 threads (wave prefix by
// shuffles, then the 4 wave totals); returns the inclusive value, *total
// the workgroup's sum
__device__ __forceinline__ int32_t wg256_inclusive_scan(int32_t v, int32_t* wsum, int32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t u = __shfl_up(v, off);
    if (lane >= off) v += u;
  }
  if (lane == 63) wsum[wave] = v;
  __syncthreads();
  int32_t before = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) before += (w < wave) ? wsum[w] : 0;
  *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  __syncthreads();  // wsum is reused by the next call
  return v + before;
}

template <bool BATCH>
__global__ __launch_bounds__(256) void seg_comp_kernel(Batch b, int32_t* __restrict__ hist_a,
                                                       int32_t* __restrict__ seg_a, int nb_a,
                                                       int K) {
  __shared__ int32_t wsum[4];
  const SegProblem p = seg_problem<BATCH>(b, hist_a, seg_a, nb_a, K);
  const int k = blockIdx.x;
  int32_t* h = p.hist + (size_t)k * p.nb;
  int32_t carry = 0;
  for (int i0 = 0; i0 < p.nb; i0 += 256) {
    const int i = i0 + threadIdx.x;
    const int32_t v = (i < p.nb) ? h[i] : 0;
    int32_t tot;
    const int32_t inc = wg256_inclusive_scan(v, wsum, &tot);
    if (i < p.nb) h[i] = carry + inc - v;
    carry += tot;
  }
  if (threadIdx.x == 0) p.seg[(K + 1) + k] = carry;  // count[k]
}

template <bool BATCH>
__global__ __launch_bounds__(1024) void seg_total_kernel(Batch b, int32_t* __restrict__ hist_a,
                                                         int32_t* __restrict__ seg_a, int nb_a,
                                                         int K, int tile,
                                                         int32_t* __restrict__ wbase1) {
  __shared__ int32_t part[1024];
  const SegProblem p = seg_problem<BATCH>(b, hist_a, seg_a, nb_a, K);
  int32_t* start = p.seg;
  const int32_t* count = p.seg + (K + 1);
  int32_t* tpre = p.seg + (2 * K + 1);
  const int t = threadIdx.x;
  const int32_t c = (t < K) ? count[t] : 0;
  const int32_t nt = (c + tile - 1) / tile;
  // the starts (exclusive prefix of the counts), then the tile prefix
  part[t] = c;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t u = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += u;
    __syncthreads();
  }
  if (t < K) start[t] = part[t] - c;
  if (t == 1023) start[K] = part[1023];
  __syncthreads();
  part[t] = nt;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t u = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += u;
    __syncthreads();
  }
  if (t < K) tpre[t] = part[t] - nt;
  if (t == 1023) {
    tpre[K] = part[1023];
    p.seg[3 * K + 2] = part[1023];
    // a batch of one image: its tile base too (0, then the total)
    if (wbase1) {
      wbase1[0] = 0;
      wbase1[1] = part[1023];
    }
  }
}

// The tile table.  For the pair sort (BATCH false) in component order.  For
// the patch-estimation tiles of a batch (BATCH true) octile-major: tile j of
// component k (n_k tiles, its patches in sort-block order, so in image
// order up to a block) lies in octile x when floor(x n_k / 8) <= j <
// floor((x + 1) n_k / 8), and an image's list holds octile 0 of every
// component, then octile 1, and so on.  The patch-estimation launch hands
// consecutive eighths of the list to the workgroups of one XCD each, so an
// XCD gathers its patches from about one eighth of the image's rows, which
// stay in its L2, instead of from the whole image.
template <bool BATCH>
__global__ __launch_bounds__(256) void seg_info_kernel(Batch b, int32_t* __restrict__ hist_a,
                                                       int32_t* __restrict__ seg_a, int nb_a,
                                                       int K) {
  constexpr int kParts = BATCH ? 8 : 1;
  __shared__ int32_t tp[kParts][kMaxK + 1];
  __shared__ int32_t base[kParts + 1];
  static_assert(kParts == 1 || kParts == 8, "two octiles per wave of 256 threads");
  const SegProblem p = seg_problem<BATCH>(b, hist_a, seg_a, nb_a, K);
  const int32_t* tpre = p.seg + (2 * K + 1);
  const int32_t total = p.seg[3 * K + 2];
  const int tl = blockIdx.x * 256 + threadIdx.x;
  if ((int)(blockIdx.x * 256) >= total) return;  // (workgroup-uniform)
  if (kParts == 1) {
    for (int k = threadIdx.x; k <= K; k += 256) tp[0][k] = tpre[k];
    if (threadIdx.x == 0) base[0] = 0;
  } else {
    // per octile, the exclusive prefix over the components of its tiles:
    // wave w scans octiles 2 w and 2 w + 1, 64 components per step
    const int lane = threadIdx.x & 63;
    for (int x = 2 * (threadIdx.x >> 6); x < 2 * (threadIdx.x >> 6) + 2; ++x) {
      int32_t carry = 0;
      for (int k0 = 0; k0 < K; k0 += 64) {
        const int k = k0 + lane;
        int32_t c = 0;
        if (k < K) {
          const int32_t n = tpre[k + 1] - tpre[k];
          c = (((x + 1) * n) >> 3) - ((x * n) >> 3);
        }
        int32_t v = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const int32_t u = __shfl_up(v, off);
          if (lane >= off) v += u;
        }
        if (k < K) tp[x][k] = carry + v - c;
        carry += __shfl(v, 63);
      }
      if (lane == 0) tp[x][K] = carry;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t s = 0;
      for (int x = 0; x < kParts; ++x) {
        base[x] = s;
        s += tp[x][K];
      }
      base[kParts] = s;
    }
  }
  __syncthreads();
  if (tl >= total) return;
  int x = 0;  // the last octile starting at or before tl
  while (x + 1 < kParts && base[x + 1] <= tl) ++x;
  const int r = tl - base[x];
  int lo = 0, hi = K - 1;  // the last k with tp[x][k] <= r
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tp[x][mid] <= r)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int32_t first = kParts == 1 ? 0 : ((x * (tpre[lo + 1] - tpre[lo])) >> 3);
  p.seg[(3 * K + 3) + tl] = lo | ((first + r - tp[x][lo]) << 10);
}

// A, B and C for `nprob` problems (BATCH: the images of b); max_tiles bounds
// the tile count of every problem
// (wbase1: a batch of one image's tile bases, written with the totals, or NULL)
template <bool BATCH>
hipError_t launch_seg_tables(const Batch& b, int32_t* hist, int32_t* seg, int nb, int K,
                             int tile, int nprob, int64_t max_tiles, hipStream_t st,
                             int32_t* wbase1 = nullptr) {
  hipLaunchKernelGGL(seg_comp_kernel<BATCH>, dim3(K, nprob), dim3(256), 0, st, b, hist, seg, nb,
                     K);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(seg_total_kernel<BATCH>, dim3(1, nprob), dim3(1024), 0, st, b, hist, seg, nb,
                     K, tile, wbase1);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t gx = (max_tiles + 255) / 256;
  if (gx < 1) return hipSuccess;
  hipLaunchKernelGGL(seg_info_kernel<BATCH>, dim3((unsigned)gx, nprob), dim3(256), 0, st, b, hist,
                     seg, nb, K);
  return hipGetLastError();
}

__global__ __launch_bounds__(1024) void scatter_kernel(Batch b, const int32_t* __restrict__ labels_b,
                                                       int K, const int32_t* __restrict__ offs_b,
                                                       const int32_t* __restrict__ seg_b,
                                                       int32_t* __restrict__ perm_b) {
  extern __shared__ int32_t cur[];  // [K] next free slot of each component in this block
  const SortBlock sb = sort_block(b);
  const int32_t* labels = labels_b + sb.d.np;
  const int32_t* offs = offs_b + (size_t)K * sb.d.sort0;
  int32_t* perm = perm_b + sb.d.np;
  const int32_t* start = seg_b + sb.d.seg;
  for (int k = threadIdx.x; k < K; k += blockDim.x)
    cur[k] = start[k] + offs[(size_t)k * sb.nb + sb.lb];
  __syncthreads();
  const int base = sb.lb * kSortBlock;
  int lab[kSortBlock / 1024];
#pragma unroll
  for (int u = 0; u < kSortBlock / 1024; ++u) {
    const int g = base + u * 1024 + (int)threadIdx.x;
    lab[u] = (g < sb.Np) ? labels[g] : K;
  }
#pragma unroll
  for (int u = 0; u < kSortBlock / 1024; ++u)
    if (lab[u] < K) perm[atomicAdd(&cur[lab[u]], 1)] = base + u * 1024 + (int)threadIdx.x;
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

__global__ __launch_bounds__(1024) void pair_scatter_kernel(const uint16_t* __restrict__ cand,
                                                            int Np, int m, int K, int nb,
                                                            const int32_t* __restrict__ offs,
                                                            const int32_t* __restrict__ start,
                                                            int32_t* __restrict__ sorted) {
  extern __shared__ int32_t cur[];
  for (int k = threadIdx.x; k < K; k += blockDim.x)
    cur[k] = start[k] + offs[(size_t)k * nb + blockIdx.x];
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
  e = launch_seg_tables<false>(Batch{}, hist, seg, nb, K, kPairTile, 1,
                               (int64_t)Np * m / kPairTile + K, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pair_scatter_kernel, dim3(nb), dim3(1024), K * sizeof(int32_t), st, cand,
                     Np, m, K, nb, hist, seg, sorted);
  return hipGetLastError();
}

// B and C of the tables for one image from its per-component counts cnt[]
// (in LDS): the starts, counts and tile prefixes written to seg (and with
// one image the Wiener bases) when `write`, and part `part` of `nparts` of
// the tile table (entries part * 1024 + tid, stride nparts * 1024); returns
// start[tid] for tid < K.  Called by all 1024 threads, after the barrier
// that completes cnt (`write`, `part`, `nparts`: workgroup-uniform).
__device__ __forceinline__ int32_t tables_bc(int K, const int32_t* cnt, int32_t* tp, int32_t* wa,
                                             int32_t* wb, int32_t* seg, int32_t* wbase,
                                             bool write, int part = 0, int nparts = 1) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t c = (tid < K) ? cnt[tid] : 0;
  const int32_t nt = (c + kWienerTile - 1) / kWienerTile;
  int32_t sa = c, st = nt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t ua = __shfl_up(sa, off), ub = __shfl_up(st, off);
    if (lane >= off) {
      sa += ua;
      st += ub;
    }
  }
  if (lane == 63) {
    wa[wave] = sa;
    wb[wave] = st;
  }
  __syncthreads();
  int32_t pa = 0, pt = 0, tot_c = 0, tot_t = 0;
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    pa += (w < wave) ? wa[w] : 0;
    pt += (w < wave) ? wb[w] : 0;
    tot_c += wa[w];
    tot_t += wb[w];
  }
  const int32_t start = pa + sa - c;
  if (tid < K) tp[tid] = pt + st - nt;
  if (tid == 0) tp[K] = tot_t;
  if (write) {
    if (tid < K) {
      seg[tid] = start;                       // start[k]
      seg[(K + 1) + tid] = c;                 // count[k]
      seg[(2 * K + 1) + tid] = pt + st - nt;  // tile prefix
    }
    if (tid == 0) {
      seg[K] = tot_c;
      seg[3 * K + 1] = tot_t;
      seg[3 * K + 2] = tot_t;
      if (wbase) {
        wbase[0] = 0;
        wbase[1] = tot_t;
      }
    }
  }
  __syncthreads();
  // C: entry t = k | (tile in k) << 10, k the last with tp[k] <= t
  for (int tl = part * blockDim.x + tid; tl < tot_t; tl += nparts * blockDim.x) {
    int lo = 0, hi = K - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tp[mid] <= tl)
        lo = mid;
      else
        hi = mid - 1;
    }
    seg[(3 * K + 3) + tl] = lo | ((tl - tp[lo]) << 10);
  }
  return start;
}

// ---- the tables of a short tile list (a patch subset) in one launch: one
// workgroup per image does A (each component's exclusive scan over its
// block counts: a wave per component, 64 counts per load, the loads of up to
// kCompPerWave components in flight at once), B (a workgroup scan of counts
// and tile counts) and C (the tile table), and with one image the Wiener
// bases too.
constexpr int kCompPerWave = 8;

// nbl > 0: the counts come from the list chunks of hist_list_kernel (nbl
// per image, image i's at K nbl i) instead of the image's sort blocks.
__global__ __launch_bounds__(1024) void tables_small_kernel(Batch b, int K,
                                                            int32_t* __restrict__ hist_b,
                                                            int32_t* __restrict__ seg_b,
                                                            int32_t* __restrict__ wbase, int nbl) {
  __shared__ int32_t tp[kMaxK + 1];
  __shared__ int32_t cnt[kMaxK];
  __shared__ int32_t wa[16], wb[16];
  const ImgDesc d = b.d[blockIdx.x];
  const int Np = (d.H - 7) * (d.W - 7);
  const int nb = nbl > 0 ? nbl : (Np + kSortBlock - 1) / kSortBlock;
  int32_t* hist =
      hist_b + (size_t)K * (nbl > 0 ? (size_t)blockIdx.x * nbl : (size_t)d.sort0);
  int32_t* seg = seg_b + d.seg;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // A: wave w scans components w, w + 16, ...
  for (int k0 = wave; k0 < K; k0 += 16 * kCompPerWave) {
    int32_t carry[kCompPerWave];
#pragma unroll
    for (int i = 0; i < kCompPerWave; ++i) carry[i] = 0;
    for (int j0 = 0; j0 < nb; j0 += 64) {
      int32_t v[kCompPerWave];
#pragma unroll
      for (int i = 0; i < kCompPerWave; ++i) {
        const int k = k0 + 16 * i;
        v[i] = (k < K && j0 + lane < nb) ? hist[(size_t)k * nb + j0 + lane] : 0;
      }
#pragma unroll
      for (int i = 0; i < kCompPerWave; ++i) {
        const int k = k0 + 16 * i;
        int32_t x = v[i];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const int32_t u = __shfl_up(x, off);
          if (lane >= off) x += u;
        }
        if (k < K && j0 + lane < nb) hist[(size_t)k * nb + j0 + lane] = carry[i] + x - v[i];
        carry[i] += __shfl(x, 63);
      }
    }
#pragma unroll
    for (int i = 0; i < kCompPerWave; ++i) {
      const int k = k0 + 16 * i;
      if (k < K && lane == 0) cnt[k] = carry[i];
    }
  }
  __syncthreads();
  tables_bc(K, cnt, tp, wa, wb, seg, wbase, true);
}

hipError_t launch_bucket_batch(const Batch& b, const int32_t* labels, int K, int32_t* hist,
                               int32_t* seg, int32_t* perm, int32_t* wbase,
                               int64_t max_tiles_image, hipStream_t st) {
  hipLaunchKernelGGL(hist_kernel, dim3(b.n_sort), dim3(1024), K * sizeof(int32_t), st, b, labels,
                     K, hist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool small = max_tiles_image <= kSmallTiles;
  if (small) {
    hipLaunchKernelGGL(tables_small_kernel, dim3(b.n), dim3(1024), 0, st, b, K, hist, seg,
                       b.n == 1 ? wbase : nullptr, 0);
    e = hipGetLastError();
  } else {
    e = launch_seg_tables<true>(b, hist, seg, 0, K, kWienerTile, b.n,
                                b.max_np / kWienerTile + K, st, b.n == 1 ? wbase : nullptr);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scatter_kernel, dim3(b.n_sort), dim3(1024), K * sizeof(int32_t), st, b,
                     labels, K, hist, seg, perm);
  e = hipGetLastError();
  if (e != hipSuccess || b.n == 1) return e;  // (one image: the tables wrote its bases)
  hipLaunchKernelGGL(wbase_kernel, dim3(1), dim3(1024), 0, st, b, K, seg, wbase);
  return hipGetLastError();
}

// ---- the same sort over per-image patch lists (a jittered subset listed
// as drawn; list + d.np, counts[i] entries): chunks of kListChunk list
// entries (one per thread: the label gathers of many workgroups in flight)
// take the place of the sort blocks (nbl per image, a 2-D grid of chunks x
// images; a chunk past its list's end stores zero counts), so the work
// follows the subset, not the image.
__global__ __launch_bounds__(1024) void hist_list_kernel(Batch b,
                                                         const int32_t* __restrict__ labels_b,
                                                         const int32_t* __restrict__ list_b,
                                                         const int32_t* __restrict__ counts, int K,
                                                         int nbl, int32_t* __restrict__ hist_b) {
  extern __shared__ int32_t h[];
  const int img = blockIdx.y, ch = blockIdx.x;
  const ImgDesc d = b.d[img];
  const int n = counts[img];
  const int32_t* list = list_b + d.np;
  const int32_t* labels = labels_b + d.np;
  int32_t* hist = hist_b + (size_t)K * ((size_t)img * nbl);
  for (int k = threadIdx.x; k < K; k += blockDim.x) h[k] = 0;
  __syncthreads();
  const int e = ch * kListChunk + (int)threadIdx.x;
  const int lab = (e < n) ? labels[list[e]] : K;
  if (lab < K) atomicAdd(&h[lab], 1);
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) hist[(size_t)k * nbl + ch] = h[k];
}

__global__ __launch_bounds__(1024) void scatter_list_kernel(Batch b,
                                                            const int32_t* __restrict__ labels_b,
                                                            const int32_t* __restrict__ list_b,
                                                            const int32_t* __restrict__ counts,
                                                            int K, int nbl,
                                                            const int32_t* __restrict__ offs_b,
                                                            const int32_t* __restrict__ seg_b,
                                                            int32_t* __restrict__ perm_b) {
  extern __shared__ int32_t cur[];
  const int img = blockIdx.y, ch = blockIdx.x;
  const ImgDesc d = b.d[img];
  const int n = counts[img];
  if (ch * kListChunk >= n) return;  // (workgroup-uniform)
  const int32_t* list = list_b + d.np;
  const int32_t* labels = labels_b + d.np;
  const int32_t* offs = offs_b + (size_t)K * ((size_t)img * nbl);
  const int32_t* start = seg_b + d.seg;
  int32_t* perm = perm_b + d.np;
  for (int k = threadIdx.x; k < K; k += blockDim.x) cur[k] = start[k] + offs[(size_t)k * nbl + ch];
  __syncthreads();
  const int e = ch * kListChunk + (int)threadIdx.x;
  if (e < n) {
    const int p = list[e];
    perm[atomicAdd(&cur[labels[p]], 1)] = p;
  }
}

// With at most 64 chunks per image the tables need no launch of their own:
// every scatter workgroup reads its image's whole chunk histogram (a wave
// per component, one count per lane) and takes both sums it needs, the
// counts of the chunks before its own and the component totals; the scan of
// the totals is then the workgroup scan of tables_bc, chunk 0 of each image
// writes the image's tables and the chunks that hold entries share its tile
// table.  Same slots as scatter_list_kernel after tables_small_kernel.
constexpr int kFusedChunks = 64;
constexpr int kFusedCompPerWave = 16;  // K <= 256: one round of loads

__global__ __launch_bounds__(1024) void scatter_tables_list_kernel(
    Batch b, const int32_t* __restrict__ labels_b, const int32_t* __restrict__ list_b,
    const int32_t* __restrict__ counts, int K, int nbl, const int32_t* __restrict__ hist_b,
    int32_t* __restrict__ seg_b, int32_t* __restrict__ perm_b, int32_t* __restrict__ wbase) {
  __shared__ int32_t tp[kMaxK + 1];
  __shared__ int32_t cnt[kMaxK];
  __shared__ int32_t cur[kMaxK];
  __shared__ int32_t wa[16], wb[16];
  const int img = blockIdx.y, ch = blockIdx.x;
  const ImgDesc d = b.d[img];
  const int n = counts[img];
  const int nact = max(1, (n + kListChunk - 1) / kListChunk);  // chunks at work
  if (ch >= nact) return;  // (workgroup-uniform)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // the entry's label first: its two dependent loads overlap the scans
  const int e = ch * kListChunk + tid;
  int p = 0, lab = K;
  if (e < n) {
    p = list_b[d.np + e];
    lab = labels_b[d.np + p];
  }
  const int32_t* hist = hist_b + (size_t)K * ((size_t)img * nbl);
  for (int k0 = wave; k0 < K; k0 += 16 * kFusedCompPerWave) {
    int32_t v[kFusedCompPerWave];
#pragma unroll
    for (int i = 0; i < kFusedCompPerWave; ++i) {
      const int k = k0 + 16 * i;
      v[i] = (k < K && lane < nbl) ? hist[(size_t)k * nbl + lane] : 0;
    }
#pragma unroll
    for (int i = 0; i < kFusedCompPerWave; ++i) {
      const int k = k0 + 16 * i;
      int32_t x = v[i];
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int32_t u = __shfl_up(x, off);
        if (lane >= off) x += u;
      }
      const int32_t before = ch > 0 ? __shfl(x, ch - 1) : 0;
      const int32_t total = __shfl(x, 63);
      if (k < K && lane == 0) {
        cur[k] = before;
        cnt[k] = total;
      }
    }
  }
  __syncthreads();
  const int32_t start = tables_bc(K, cnt, tp, wa, wb, seg_b + d.seg, wbase, ch == 0, ch, nact);
  if (tid < K) cur[tid] += start;
  __syncthreads();
  if (lab < K) perm_b[d.np + atomicAdd(&cur[lab], 1)] = p;
}

hipError_t launch_bucket_list(const Batch& b, const int32_t* labels, const int32_t* list,
                              const int32_t* counts, int K, int nbl, int32_t* hist, int32_t* seg,
                              int32_t* perm, int32_t* wbase, bool have_hist, hipStream_t st) {
  const dim3 grid((unsigned)nbl, (unsigned)b.n);
  hipError_t e;
  if (!have_hist) {
    hipLaunchKernelGGL(hist_list_kernel, grid, dim3(1024), K * sizeof(int32_t), st, b, labels,
                       list, counts, K, nbl, hist);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nbl <= kFusedChunks) {
    hipLaunchKernelGGL(scatter_tables_list_kernel, grid, dim3(1024), 0, st, b, labels, list,
                       counts, K, nbl, hist, seg, perm, b.n == 1 ? wbase : nullptr);
    e = hipGetLastError();
  } else {
    hipLaunchKernelGGL(tables_small_kernel, dim3(b.n), dim3(1024), 0, st, b, K, hist, seg,
                       b.n == 1 ? wbase : nullptr, nbl);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scatter_list_kernel, grid, dim3(1024), K * sizeof(int32_t), st, b,
                       labels, list, counts, K, nbl, hist, seg, perm);
    e = hipGetLastError();
  }
  if (e != hipSuccess || b.n == 1) return e;
  hipLaunchKernelGGL(wbase_kernel, dim3(1), dim3(1024), 0, st, b, K, seg, wbase);
  return hipGetLastError();
}

}  // namespace fepll
