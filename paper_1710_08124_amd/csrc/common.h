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
//  * Wt   float,  [T][K][2][8][64][4]: the patch-estimation A operand,
//    entry W_k[q][p] with q = 32*qb + (l & 31), p = 32*(l >> 5) + s, where
//    W_k = U_k diag(gamma_k) U_k^t (the Wiener filter of Alg. 1, patch
//    estimation, written back in pixel space).
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

struct Schedule {
  int T;
  double beta[kMaxT];
};

// ------------------------------------------------------------ launches
// Every launcher returns hipSuccess or the launch error; none synchronises.

hipError_t launch_prep(const double* U64, const double* lam64, const double* w64, int K,
                       const Schedule& sch, float* Ut, uint16_t* Ub, float* Wt, float* L32,
                       double* L64, double* invnu64, uint8_t* Uf, int32_t* Ue, hipStream_t st);

hipError_t launch_estep_f32(const float* x, int H, int W, const float* Ut_t, const float* L32_t,
                            int K, double beta, int32_t* labels, float* best, float* second,
                            int32_t* flags, int32_t* list_count, int32_t* list, hipStream_t st);

hipError_t launch_estep_bf16(const float* x, int H, int W, const uint16_t* Ub_t,
                             const float* L32_t, int K, int32_t* labels, float* best,
                             float* second, hipStream_t st);

hipError_t launch_estep_fp8(const float* x, int H, int W, const uint8_t* Uf_t,
                            const int32_t* Ue_t, const float* L32_t, int K, int32_t* labels,
                            float* best, float* second, hipStream_t st);

hipError_t launch_recheck_f64(const float* x, int H, int W, const double* U64,
                              const double* invnu64_t, const double* L64_t, int K,
                              const int32_t* list_count, const int32_t* list, int32_t* labels,
                              int max_list, hipStream_t st);

// Counting sort of patch indices by label and the Wiener tile list.
// hist: [K][nb] int32, nb = ceil(Np / kSortBlock); seg: int32, laid out as
// start[K+1], count[K], tile_prefix[K+1], total_tiles, then the tile table
// (seg_size(Np, K) entries in all): entry t = k | (tile index in k) << 10.
constexpr int kSortBlock = 16384;
constexpr int kWienerTile = 32;
inline size_t seg_size(size_t Np, int K) { return 3 * (size_t)K + 3 + Np / kWienerTile + K + 1; }
hipError_t launch_bucket(const int32_t* labels, int Np, int K, int32_t* hist, int32_t* seg,
                         int32_t* perm, hipStream_t st);

// Patch estimates z^: float [Np][64], patch-major (pixel 8 dy + dx of patch i
// at i * 64 + 8 dy + dx).
hipError_t launch_wiener_f32(const float* x, int H, int W, const float* Wt_t, int K,
                             const int32_t* seg, const int32_t* perm, float* Zhat,
                             hipStream_t st);

hipError_t launch_ola_update(const float* Zhat, const float* y, int H, int W, double b,
                             float* xnew, hipStream_t st);

}  // namespace fepll
