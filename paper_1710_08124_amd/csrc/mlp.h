// Internal declarations of the proposal-network kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fepll {

constexpr int kFeat = 65;        // input features: 64 DC-removed pixels + log sigma_beta
constexpr int kHidden = 256;     // width of both hidden layers
constexpr float kScaleIn = 128.f;  // pixels enter the network as z~ / 128

enum { kEpiNone = 0, kEpiBias = 1, kEpiBiasGelu = 2, kEpiGeluGrad = 3 };

// Offsets of the flat float32 parameter vector W1 b1 W2 b2 W3 b3, W stored
// (out, in) row-major.
struct MlpLayout {
  int K;
  size_t W1, b1, W2, b2, W3, b3, n;
  explicit MlpLayout(int K_) : K(K_) {
    W1 = 0;
    b1 = W1 + (size_t)kHidden * kFeat;
    W2 = b1 + kHidden;
    b2 = W2 + (size_t)kHidden * kHidden;
    W3 = b2 + kHidden;
    b3 = W3 + (size_t)K * kHidden;
    n = b3 + K;
  }
};

hipError_t launch_gemm_f32(const float* A, int lda, bool transA, const float* B, int ldb,
                           bool transB, float* C, int ldc, int M, int N, int Kd, int epi,
                           const float* bias, float* aux, int ldaux, hipStream_t st);
hipError_t launch_softmax_xent(const float* Z, int n, int K, const int32_t* y, float scale,
                               float* dZ, float* loss, hipStream_t st);
hipError_t launch_colsum(const float* Mx, int rows, int cols, float* out, hipStream_t st);
hipError_t launch_sum(const float* v, int n, float* out, hipStream_t st);
hipError_t launch_adamw(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                        float b2, float eps, float wd, int step, hipStream_t st);
hipError_t launch_features(const float* x, int H, int W, int64_t ld, double beta, float* X,
                           hipStream_t st);

}  // namespace fepll
