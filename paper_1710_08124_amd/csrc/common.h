// Internal declarations shared by the HIP kernels and the host runtime.
//
// Layout of the per-beta constant tables the kernels read (all in device
// memory, built once per beta schedule by prep.hip):
//
//  * Ut   float,  [T][K][2][8][64][4]: the E-step MFMA A operand.  For
//    iteration t, component k, eigen block jb (0/1), MFMA step s = 4*i + e
//    (i = 0..7, e = 0..3) and lane l, the float at [t][k][jb][i][l][e] is
//    U_k[p][j] / sqrt(nu_kj) with p = 2*s + (l >> 5) and j = 32*jb + (l & 31).
//    Scaling the eigenvectors by nu^-1/2 turns the Mahalanobis term
//    sum_j c_j^2 / nu_kj of the selection cost into a plain sum of squares.
//  * Wt   float,  [T][K][2][8][64][4]: the patch-estimation B operand
//    (pixels of the estimate as columns), entry W_k[q][p] with
//    q = 32*qb + (l & 31), p = 32*(l >> 5) + s, where
//    W_k = U_k diag(gamma_k) U_k^t (the Wiener filter of Alg. 1, patch
//    estimation, written back in pixel space).
//  * Wh   binary16 bits (uint16), [T][K][2][4][64][8]: the patch-estimation
//    B operand of the reduced-precision modes (v_mfma_f32_32x32x16_f16),
//    entry W_k[q][p] with q = 32*qb + (l & 31), p = 16*s + 8*(l >> 5) + e for
//    column block qb, depth step s, lane l, element e (float64 -> float32 ->
//    binary16, nearest even).
//  * Ub   bf16 bits (uint16), [T][K][4][2][64][8]: the bfloat16 E-step A
//    operand (v_mfma_f32_16x16x32_bf16), entry Ut_k[p][j] with
//    j = 16*rb + (l & 15) and p = 32*t + 8*(l >> 4) + e for eigen block rb
//    (0..3), depth step t (0..1), lane l, element e.
//  * Uf   e4m3 bytes, [T][K][2][2][64][16]: the 8-bit E-step A operand
//    (v_mfma_scale_f32_32x32x64_f8f6f4), byte b of [t][k][rb][part][l] is
//    Ut_k[p][j] 2^-e_k with j = 32*rb + (l & 31), p = 32*(l >> 5) + 16*part + b;
//    Ue int32 [T][K] holds the E8M0 code e_k + 127 of each component's scale.
//  * L32  float,  [T][K]: L_k = iota_k + sum_j log nu_kj rounded from float64.
//  * L64  double, [T][K] and invnu64 double [T][K][64]: the same terms in
//    float64 for the re-selection of uncertified patches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fepll {

constexpr int kP = 64;          // pixels per patch
constexpr int kTileStride = 4096;  // floats per (t, k) operand table
constexpr int kMaxT = 16;
constexpr int kMaxK = 1024;

// Which per-beta tables a prep launch fills (Wt and L32 always).
enum { kTabF32 = 1, kTabBF16 = 2, kTabF8 = 4 };

// Device pointers of the per-beta tables, [S][K][...] for S beta slots.
struct ConstTables {
  float* Ut;
  uint16_t* Ub;
  float* Wt;
  uint16_t* Wh;  // with Ub or Uf (the reduced-precision modes' estimate)
  float* L32;
  double* L64;
  double* invnu64;
  uint8_t* Uf;
  int32_t* Ue;
  // flat-tail spectrum approximation (Sec. 3.1): rk[k] eigenvalues kept per
  // component (64: none replaced; NULL: all 64); with a tail, the bf16 / e4m3
  // operands hold only the first rk columns, scaled by
  // sqrt(1/nu_j - 1/nu_P), and Pinv [S][K] = 1/nu_P multiplies |z~|^2 (0
  // without a tail)
  const int32_t* rk;
  float* Pinv;
};

// One image of a batch (a single restoration is a batch of one): its size
// and where it lives in the packed buffers.  Images are packed one after
// the other: pixels (H x W, contiguous rows) from px, patches from np (the
// labels, the sorted patch list and the patch estimates of the image),
// the bucket segment table from seg.  Work is split into tiles numbered
// across the batch: the image's first sort block, selection tile and
// reprojection tile are sort0, est0 and ola0; its beta of iteration t is
// slot slot0 + t of the per-beta tables.
struct ImgDesc {
  int32_t H, W;
  int64_t px;
  int64_t np;
  int64_t seg;
  int32_t sort0, est0, ola0, slot0;
  int32_t resc0;  // first rescoring tile of the proposal
  int32_t pad;
};

// Selection tile: 4 patch rows x kEstCols patch columns (one workgroup).
constexpr int kEstCols = 128;
// Reprojection tile: kOlaX columns x Batch::ola_rows (16, 32 or 64) rows.
constexpr int kOlaX = 64;
constexpr int kMaxBatch = 65536;

struct Batch {
  const ImgDesc* d;         // device, n entries
  const int32_t* est_img;   // device: image of each selection tile
  const int32_t* sort_img;  // device: image of each sort block
  const int32_t* ola_img;   // device: image of each reprojection tile
  const int32_t* resc_img;  // device: image of each rescoring tile (proposal)
  int n;
  int n_est, n_sort, n_ola, n_resc;  // tile totals
  int64_t n_patches;         // patches of the whole batch
  int64_t max_np;            // patches of the largest image
  int ola_rows;              // rows of a reprojection tile
};

// The value itself, as if just produced: a float read again after its
// float64 conversion has fed a sum is converted afresh, so the compiler keeps
// the 32-bit value live rather than the 64-bit conversion (half the
// registers in the patch-loading prologues).
__device__ __forceinline__ float fresh(float v) {
  asm volatile("" : "+v"(v));
  return v;
}

// ------------------------------------------------------------ launches
// Every launcher returns hipSuccess or the launch error; none synchronises.

// Tables of S beta slots (betas: device, S entries) for the tables in mask.
hipError_t launch_prep(const double* U64, const double* lam64, const double* w64, int K,
                       const double* betas, int S, int mask, const ConstTables& tb,
                       hipStream_t st);

// Single-image selection kernels (tables of one beta).
hipError_t launch_estep_f32(const float* x, int H, int W, const float* Ut_t, const float* L32_t,
                            int K, double beta, int32_t* labels, float* best, float* second,
                            int32_t* flags, int32_t* list_count, int32_t* list, hipStream_t st);

hipError_t launch_recheck_f64(const float* x, int H, int W, const double* U64,
                              const double* invnu64_t, const double* L64_t, int K,
                              const int32_t* list_count, const int32_t* list, int32_t* labels,
                              int max_list, hipStream_t st);

// Batched selection, all K components, iteration t: x, labels, best, second
// are packed buffers (best / second may be NULL); Ub / Uf / Ue / L32 the
// tables of all slots.
// blocks: workgroups of the persistent launch (0: one per tile).
// (rk / Pinv: the flat-tail tables of ConstTables, or NULL for the plain form)
hipError_t launch_estep_bf16_batch(const Batch& b, const float* x, const uint16_t* Ub,
                                   const float* L32, const int32_t* rk, const float* Pinv, int K,
                                   int t, int32_t* labels, float* best, float* second, int blocks,
                                   hipStream_t st);
hipError_t launch_estep_fp8_batch(const Batch& b, const float* x, const uint8_t* Uf,
                                  const int32_t* Ue, const float* L32, const int32_t* rk,
                                  const float* Pinv, int K, int t, int32_t* labels, float* best,
                                  float* second, int blocks, hipStream_t st);

// Counting sort of each image's patch indices by label and the Wiener tile
// lists.  hist: [K][sort blocks of the image] int32 per image, at
// K * sort0; seg (per image, at d.seg, seg_size(Np, K) entries): start[K+1],
// count[K], tile_prefix[K+1], total_tiles, then the tile table, entry
// t = k | (tile index in k) << 10; perm: patch indices (local to the image)
// sorted by label, at d.np; wbase (n + 1): first Wiener tile of each image
// across the batch, wbase[n] the total.
constexpr int kSortBlock = 16384;
constexpr int kWienerTile = 32;
inline size_t seg_size(size_t Np, int K) { return 3 * (size_t)K + 3 + Np / kWienerTile + K + 1; }
// max_tiles_image bounds every image's tile count; at most kSmallTiles (a
// patch subset), one workgroup per image builds its tables in one launch.
constexpr int64_t kSmallTiles = 4096;
hipError_t launch_bucket_batch(const Batch& b, const int32_t* labels, int K, int32_t* hist,
                               int32_t* seg, int32_t* perm, int32_t* wbase,
                               int64_t max_tiles_image, hipStream_t st);
// The same sort over per-image patch lists (list + d.np, counts[i] entries,
// labels below K; every tile list short): nbl chunks of kListChunk entries
// per image, hist holding K x nbl counts per image (K nbl n in all,
// component-major per image).  have_hist: the selection has already
// counted them (launch_estep_fp8_list with hist), no histogram launch.
constexpr int kListChunk = 1024;
hipError_t launch_bucket_list(const Batch& b, const int32_t* labels, const int32_t* list,
                              const int32_t* counts, int K, int nbl, int32_t* hist, int32_t* seg,
                              int32_t* perm, int32_t* wbase, bool have_hist, hipStream_t st);

// Pairs (patch i, candidate j < m) of the proposal, sorted by component:
// hist [K][nb] with nb = ceil(Np / kPairBlock); seg as above with tiles of
// kPairTile pairs (pair_seg_size entries); sorted: pair ids 8 i + j.
constexpr int kPairBlock = 4096;
constexpr int kPairTile = 128;
inline size_t pair_seg_size(size_t Np, int K) {
  return 3 * (size_t)K + 3 + 8 * Np / kPairTile + K + 1;
}
hipError_t launch_pair_bucket(const uint16_t* cand, int Np, int m, int K, int32_t* hist,
                              int32_t* seg, int32_t* sorted, hipStream_t st);

// Patch estimates z^: float [patches][64], patch-major (pixel 8 dy + dx of
// patch i at i * 64 + 8 dy + dx), at d.np * 64 per image.
// blocks: workgroups of the launch, a multiple of 8 (a cap: never more than
// the tiles need).  Wh: NULL (float32 operands Wt, float32 products), or the
// binary16 table (binary16 operands, float32 accumulation).
hipError_t launch_wiener_batch(const Batch& b, const float* x, const float* Wt,
                               const uint16_t* Wh, int K, int t, const int32_t* seg,
                               const int32_t* perm, const int32_t* wbase, float* Zhat, int blocks,
                               hipStream_t st);

struct JitterDraw;

// Reprojection + image update of iteration t: bvals[slot] = beta sigma^2.
// member: NULL (every patch), or packed per-patch words, a patch being in
// the subset when its word differs from `none` (the labels with none = K,
// or the subset flags with none = 0; the average then runs over the
// subset's patches only).
// raw: write x~ itself (the image estimation of an operator A follows).
// draw: NULL, or (with member) a jittered drawing run by extra workgroups
// of the same launch; it must touch no word the reprojection reads.
hipError_t launch_ola_batch(const Batch& b, const float* Zhat, const float* y,
                            const float* bvals, int t, float* xnew, const int32_t* member,
                            int none, int raw, const JitterDraw* draw, hipStream_t st);

// Deblurring (periodic convolution A), float64 half spectra of m = H (W/2+1)
// complex entries (double2): see deblur.hip.
hipError_t launch_f2d(const float* in, double* out, int n, hipStream_t st);
hipError_t launch_d2f_scale(const double* in, float* out, int n, double scale, hipStream_t st);
hipError_t launch_spec_prep(const void* Hh, const void* Yh, void* AtY, double* a2, int m,
                            hipStream_t st);
hipError_t launch_spec_update(const void* AtY, const double* a2, void* X, int m, double b,
                              hipStream_t st);
hipError_t launch_spec_init(const void* AtY, const double* a2, void* X, int H, int W, double c,
                            hipStream_t st);

// Jittered subsampling (Sec. 3.3) of one image, iteration t.  Without list:
// flags (Np, all zero before) of the chosen patches set to 1 and *count
// zeroed, then launch_jitter_compact appends every flagged patch to list
// (any order), clears its flag and sets every other patch's label to K.
// With list (*count zero before, flags all zero before): each chosen patch
// is appended to list at *count and flagged.  The same launch first undoes
// an earlier iteration's list when prev.list is set: its prev.count
// entries get flag 0 in prev.flags (another flag set) and, with
// prev.labels, label K (every label not on the new list is K before the
// selection), and *prev.zero (a count a later drawing appends to) is
// zeroed.
// launch_jitter_reset does the same for the last list of a restoration
// (next_count may be NULL).  With clear set, the launch also zeroes its
// nclear words (the chunk histogram the selection then adds to).
struct JitterPrev {
  const int32_t* list = nullptr;
  const int32_t* count = nullptr;
  int32_t* flags = nullptr;
  int32_t* labels = nullptr;
  int K = 0;
  int32_t* zero = nullptr;
  int32_t* clear = nullptr;
  int nclear = 0;
};
// A drawing's launch arguments (make_jitter_draw) and its workgroups of 256
// threads (*blocks), for a launch of its own (launch_jitter_mark) or as the
// extra workgroups of the subset reprojection (launch_ola_batch).
struct JitterDraw {
  int H = 0, W = 0, s = 0;
  uint32_t k0 = 0, k1 = 0;
  int t = 0, amax = 0, cmax = 0;
  int32_t* flags = nullptr;
  int32_t* count = nullptr;
  int32_t* list = nullptr;
  JitterPrev prev;
};
JitterDraw make_jitter_draw(int H, int W, int s, uint64_t seed, int t, int32_t* flags,
                            int32_t* count, int32_t* list, const JitterPrev& prev, int* blocks);
hipError_t launch_jitter_mark(int H, int W, int s, uint64_t seed, int t, int32_t* flags,
                              int32_t* count, int32_t* list, const JitterPrev& prev,
                              hipStream_t st);
hipError_t launch_jitter_reset(const int32_t* list, int64_t list_max, const int32_t* count,
                               int32_t* next_count, int32_t* flags, int32_t* labels, int K,
                               hipStream_t st);
hipError_t launch_jitter_compact(int Np, int K, int32_t* flags, int32_t* labels,
                                 int32_t* count, int32_t* list, hipStream_t st);
// e4m3 selection of the patches in list (*count <= list_max entries,
// indices within the image) of the one image d[0] of a batch at iteration
// t; x, the tables, labels / best / second: packed batch buffers and
// all-slot tables, as for launch_estep_fp8_batch.  part: NULL, or
// fp8_list_split(list_max, K) x list_max float4 of scratch, which lets a
// short list be split over the components (same labels): *nsplit receives
// the number of component ranges, and when it is above 1 launch_fp8_merge
// must follow to write the results.  hist: NULL, or the image's K x nbl
// chunk histogram of launch_bucket_list (zero before), to which a one-pass
// selection adds the counts of its labels per chunk of kListChunk entries
// (NULL required with part).
int fp8_list_split(int64_t list_max, int K);
hipError_t launch_estep_fp8_list(const ImgDesc* d, int64_t list_max, int t, const float* x,
                                 const uint8_t* Uf, const int32_t* Ue, const float* L32,
                                 const int32_t* rk, const float* Pinv, int K,
                                 const int32_t* count, const int32_t* list, int32_t* labels,
                                 float* best, float* second, float4* part, int* nsplit,
                                 int32_t* hist, int nbl, hipStream_t st);
hipError_t launch_fp8_merge(const ImgDesc* d, int64_t list_max, const int32_t* count,
                            const int32_t* list, const float4* part, int nsplit, int32_t* labels,
                            float* best, float* second, hipStream_t st);
// Bound on the number of patches the jittered grid of spacing s chooses in
// an H x W image (grid points).
int64_t jitter_points_max(int H, int W, int s);

// Image of tile `tile` given each image's first tile (first[0] = 0,
// ascending): the last i with first[i] <= tile.
__device__ __forceinline__ int image_of(const int32_t* __restrict__ first, int n, int tile) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace fepll
