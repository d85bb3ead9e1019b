// Training kernels of the component-proposal network (float32):
//   h1 = GELU(W1 x + b1), h2 = GELU(W2 h1 + b2), z = W3 h2 + b3,
// softmax cross-entropy against the selected component, backpropagation and
// AdamW.  The network is this project's replacement for the paper's search
// tree (Sec. 3.2) in the role of limiting how many components the
// selection step scores; its output is always rescored with the exact cost
// of Eq. (8).
//
// One tiled float32 MFMA GEMM serves every product of the forward and
// backward passes (C = op(A) op(B), A or B optionally transposed) with fused
// epilogues (bias, bias + GELU keeping the pre-activation, multiplication by
// GELU'(pre-activation)).  All reductions run in a fixed order, so training
// is bitwise reproducible.
#include "common.h"
#include "mlp.h"

namespace fepll {

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {
constexpr int TM = 64, TN = 64, TK = 32;

// GELU in its tanh form (Hendrycks & Gimpel, 2016): a sigmoid(2 u) with
// u = sqrt(2/pi) (a + 0.044715 a^3), i.e. 0.5 a (1 + tanh u); the inference
// kernel evaluates the same function.
__device__ __forceinline__ float gelu(float a) {
  const float u2 = a * fmaf(0.0713548162726f, a * a, 1.59576912161f);  // 2 u
  return a / (1.f + expf(-u2));
}
__device__ __forceinline__ float gelu_grad(float a) {
  const float a2 = a * a;
  const float s = 1.f / (1.f + expf(-a * fmaf(0.0713548162726f, a2, 1.59576912161f)));
  // d(2u)/da = 2 sqrt(2/pi) (1 + 3 * 0.044715 a^2)
  return fmaf(a * s * (1.f - s), fmaf(0.214064448818f, a2, 1.59576912161f), s);
}
}  // namespace

// C[m][n] (row stride ldc) = sum_k A(m,k) B(k,n); A(m,k) = A[m*lda + k] or,
// transposed, A[k*lda + m]; B(k,n) = B[k*ldb + n] or, transposed, B[n*ldb + k].
__global__ __launch_bounds__(256) void gemm_f32_kernel(const float* __restrict__ A, int lda,
                                                       int transA, const float* __restrict__ B,
                                                       int ldb, int transB, float* __restrict__ C,
                                                       int ldc, int M, int N, int Kd, int epi,
                                                       const float* __restrict__ bias,
                                                       float* __restrict__ aux, int ldaux) {
  __shared__ float As[TM][TK + 1];
  __shared__ float Bs[TK][TN + 1];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  f32x16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < Kd; k0 += TK) {
    for (int e = threadIdx.x; e < TM * TK; e += 256) {
      int m, k;
      if (transA) {
        m = e & (TM - 1);
        k = e / TM;
      } else {
        k = e & (TK - 1);
        m = e / TK;
      }
      const int gm = m0 + m, gk = k0 + k;
      float v = 0.f;
      if (gm < M && gk < Kd) v = transA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
      As[m][k] = v;
    }
    for (int e = threadIdx.x; e < TK * TN; e += 256) {
      int k, n;
      if (transB) {
        k = e & (TK - 1);
        n = e / TK;
      } else {
        n = e & (TN - 1);
        k = e / TN;
      }
      const int gk = k0 + k, gn = n0 + n;
      float v = 0.f;
      if (gk < Kd && gn < N) v = transB ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn];
      Bs[k][n] = v;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < TK / 2; ++s) {
      const float a = As[wm * 32 + (lane & 31)][2 * s + (lane >> 5)];
      const float b = Bs[2 * s + (lane >> 5)][wn * 32 + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int n = n0 + wn * 32 + (lane & 31);
  if (n >= N) return;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int m = m0 + wm * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
    if (m >= M) continue;
    float v = acc[i];
    if (epi == kEpiBias) {
      v += bias[n];
    } else if (epi == kEpiBiasGelu) {
      v += bias[n];
      aux[(size_t)m * ldaux + n] = v;
      v = gelu(v);
    } else if (epi == kEpiGeluGrad) {
      v *= gelu_grad(aux[(size_t)m * ldaux + n]);
    }
    C[(size_t)m * ldc + n] = v;
  }
}

hipError_t launch_gemm_f32(const float* A, int lda, bool transA, const float* B, int ldb,
                           bool transB, float* C, int ldc, int M, int N, int Kd, int epi,
                           const float* bias, float* aux, int ldaux, hipStream_t st) {
  dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
  hipLaunchKernelGGL(gemm_f32_kernel, grid, dim3(256), 0, st, A, lda, transA ? 1 : 0, B, ldb,
                     transB ? 1 : 0, C, ldc, M, N, Kd, epi, bias, aux, ldaux);
  return hipGetLastError();
}

// Row-wise softmax cross-entropy: one wave per row.  dZ = (softmax - onehot)
// * scale, loss[row] = logsumexp - z[target].
__global__ __launch_bounds__(256) void softmax_xent_kernel(const float* __restrict__ Z, int n,
                                                           int K, const int32_t* __restrict__ y,
                                                           float scale, float* __restrict__ dZ,
                                                           float* __restrict__ loss) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const float* z = Z + (size_t)row * K;
  float mx = -INFINITY;
  for (int k = lane; k < K; k += 64) mx = fmaxf(mx, z[k]);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
  float s = 0.f;
  for (int k = lane; k < K; k += 64) s += expf(z[k] - mx);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
  const float lse = mx + logf(s);
  const int t = y[row];
  float* d = dZ + (size_t)row * K;
  for (int k = lane; k < K; k += 64) {
    const float p = expf(z[k] - lse);
    d[k] = (p - (k == t ? 1.f : 0.f)) * scale;
  }
  if (lane == 0) loss[row] = lse - z[t];
}

hipError_t launch_softmax_xent(const float* Z, int n, int K, const int32_t* y, float scale,
                               float* dZ, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(softmax_xent_kernel, dim3((n + 3) / 4), dim3(256), 0, st, Z, n, K, y, scale,
                     dZ, loss);
  return hipGetLastError();
}

// out[j] = sum_i M[i][j] (row order fixed): bias gradients.
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ Mx, int rows,
                                                     int cols, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int i = 0; i < rows; ++i) s += Mx[(size_t)i * cols + j];
  out[j] = s;
}

hipError_t launch_colsum(const float* Mx, int rows, int cols, float* out, hipStream_t st) {
  hipLaunchKernelGGL(colsum_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, Mx, rows, cols,
                     out);
  return hipGetLastError();
}

// Sum of v[0..n) in a fixed order by one workgroup (the mean loss).
__global__ __launch_bounds__(256) void sum_kernel(const float* __restrict__ v, int n,
                                                  float* __restrict__ out) {
  __shared__ float part[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) s += v[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
}

hipError_t launch_sum(const float* v, int n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, v, n, out);
  return hipGetLastError();
}

// AdamW with bias-corrected moments and decoupled weight decay.
__global__ __launch_bounds__(256) void adamw_kernel(float* __restrict__ p,
                                                    const float* __restrict__ g,
                                                    float* __restrict__ m, float* __restrict__ v,
                                                    int n, float lr, float b1, float b2, float eps,
                                                    float wd, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  p[i] = p[i] - lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
}

hipError_t launch_adamw(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                        float b2, float eps, float wd, int step, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)step);
  const float c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adamw_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, g, m, v, n, lr, b1,
                     b2, eps, wd, c1, c2);
  return hipGetLastError();
}

// Network input of every patch of image x: [z~ / 128, log sigma_beta],
// z~ the DC-removed patch (mean in float64), sigma_beta = beta^-1/2.
__global__ __launch_bounds__(256) void features_kernel(const float* __restrict__ x, int H, int W,
                                                       int64_t ld, float logsb,
                                                       float* __restrict__ X) {
  const int lane = threadIdx.x & 63;
  const int Wp = W - 7;
  const int Np = (H - 7) * Wp;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= Np) return;
  const int r = i / Wp, c = i - (i / Wp) * Wp;
  const float v = x[(size_t)(r + (lane >> 3)) * ld + c + (lane & 7)];
  double s = (double)v;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
  const float zt = (float)((double)v - s * (1.0 / 64.0));
  float* out = X + (size_t)i * kFeat;
  out[lane] = zt * (1.f / kScaleIn);
  if (lane == 0) out[64] = logsb;
}

hipError_t launch_features(const float* x, int H, int W, int64_t ld, double beta, float* X,
                           hipStream_t st) {
  const int Np = (H - 7) * (W - 7);
  hipLaunchKernelGGL(features_kernel, dim3((Np + 3) / 4), dim3(256), 0, st, x, H, W, ld,
                     (float)(-0.5 * log(beta)), X);
  return hipGetLastError();
}

}  // namespace fepll
