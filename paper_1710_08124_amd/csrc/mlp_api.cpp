// C ABI of the proposal network: handle, training, serialization.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "fepll.h"
#include "internal.h"
#include "mlp.h"

using namespace fepll;

struct fepll_mlp {
  int K = 0;
  int max_batch = 0;
  int step = 0;
  MlpLayout lay{1};
  float* p = nullptr;  // parameters
  float* g = nullptr;  // gradients
  float* m = nullptr;  // AdamW moments
  float* v = nullptr;
  float *A1 = nullptr, *H1 = nullptr, *A2 = nullptr, *H2 = nullptr, *Z = nullptr, *dZ = nullptr,
        *dH = nullptr, *dA = nullptr, *loss_rows = nullptr;
  float* Xb = nullptr;    // gathered minibatch
  int32_t* yb = nullptr;
};

namespace {

uint64_t fnv1a(const void* data, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(data);
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

struct BlobHeader {
  char magic[8];      // "FEPLLMLP"
  uint32_t version;   // 1
  uint32_t K;
  uint32_t d_in;      // 65
  uint32_t hidden;    // 256
  float scale_in;     // 128
  uint32_t gelu;      // 2 = tanh form (the only one inference evaluates)
  uint64_t nparam;
  uint64_t checksum;  // FNV-1a-64 of the parameter bytes
  uint8_t pad[64 - 48];
};
static_assert(sizeof(BlobHeader) == 64, "header layout");

// Forward pass of rows [0, n) of X into m->Z (n <= max_batch), keeping the
// activations the backward pass needs.
fepll_status forward_chunk(fepll_mlp* m, const float* X, int n, float* Zout, hipStream_t st) {
  const MlpLayout& L = m->lay;
  HIPX(launch_gemm_f32(X, kFeat, false, m->p + L.W1, kFeat, true, m->H1, kHidden, n, kHidden,
                       kFeat, kEpiBiasGelu, m->p + L.b1, m->A1, kHidden, st));
  HIPX(launch_gemm_f32(m->H1, kHidden, false, m->p + L.W2, kHidden, true, m->H2, kHidden, n,
                       kHidden, kHidden, kEpiBiasGelu, m->p + L.b2, m->A2, kHidden, st));
  HIPX(launch_gemm_f32(m->H2, kHidden, false, m->p + L.W3, kHidden, true, Zout, m->K, n, m->K,
                       kHidden, kEpiBias, m->p + L.b3, nullptr, 0, st));
  return FEPLL_OK;
}

fepll_status loss_grad(fepll_mlp* m, const float* X, const int32_t* y, int n, float* loss,
                       hipStream_t st) {
  const MlpLayout& L = m->lay;
  const int K = m->K;
  fepll_status s;
  if ((s = forward_chunk(m, X, n, m->Z, st)) != FEPLL_OK) return s;
  HIPX(launch_softmax_xent(m->Z, n, K, y, 1.f / n, m->dZ, m->loss_rows, st));
  // layer 3
  HIPX(launch_gemm_f32(m->dZ, K, true, m->H2, kHidden, false, m->g + L.W3, kHidden, K, kHidden,
                       n, kEpiNone, nullptr, nullptr, 0, st));
  HIPX(launch_colsum(m->dZ, n, K, m->g + L.b3, st));
  HIPX(launch_gemm_f32(m->dZ, K, false, m->p + L.W3, kHidden, false, m->dA, kHidden, n, kHidden,
                       K, kEpiGeluGrad, nullptr, m->A2, kHidden, st));
  // layer 2
  HIPX(launch_gemm_f32(m->dA, kHidden, true, m->H1, kHidden, false, m->g + L.W2, kHidden,
                       kHidden, kHidden, n, kEpiNone, nullptr, nullptr, 0, st));
  HIPX(launch_colsum(m->dA, n, kHidden, m->g + L.b2, st));
  HIPX(launch_gemm_f32(m->dA, kHidden, false, m->p + L.W2, kHidden, false, m->dH, kHidden, n,
                       kHidden, kHidden, kEpiGeluGrad, nullptr, m->A1, kHidden, st));
  // layer 1
  HIPX(launch_gemm_f32(m->dH, kHidden, true, X, kFeat, false, m->g + L.W1, kFeat, kHidden, kFeat,
                       n, kEpiNone, nullptr, nullptr, 0, st));
  HIPX(launch_colsum(m->dH, n, kHidden, m->g + L.b1, st));
  if (loss) {
    HIPX(launch_sum(m->loss_rows, n, loss, st));
  }
  return FEPLL_OK;
}

__global__ void scale_kernel(float* v, float s) { v[0] *= s; }

__global__ void gather_rows_kernel(const float* __restrict__ X, const int32_t* __restrict__ y,
                                   const int32_t* __restrict__ rows, int n,
                                   float* __restrict__ Xb, int32_t* __restrict__ yb) {
  const int i = blockIdx.x;
  if (i >= n) return;
  const int r = rows[i];
  for (int j = threadIdx.x; j < kFeat; j += blockDim.x)
    Xb[(size_t)i * kFeat + j] = X[(size_t)r * kFeat + j];
  if (threadIdx.x == 0) yb[i] = y[r];
}

}  // namespace

extern "C" {

int64_t fepll_mlp_param_count(int32_t K) {
  if (K < 1 || K > kMaxK) return -1;
  return (int64_t)MlpLayout(K).n;
}

fepll_status fepll_mlp_create(int32_t K, const float* params, int32_t max_batch,
                              fepll_mlp** out) {
  clear_error();
  if (!out) return fail(FEPLL_EINVAL, "out is NULL");
  if (K < 1 || K > kMaxK) return fail(FEPLL_EINVAL, "K must be in 1..1024");
  if (max_batch < 1 || max_batch > (1 << 20)) return fail(FEPLL_EINVAL, "max_batch out of range");
  if (!params) return fail(FEPLL_EINVAL, "params is NULL");
  const MlpLayout L(K);
  for (size_t i = 0; i < L.n; ++i)
    if (!std::isfinite(params[i])) return fail(FEPLL_EINVAL, "params has a non-finite value");
  fepll_mlp* m = new (std::nothrow) fepll_mlp();
  if (!m) return fail(FEPLL_ENOMEM, "host allocation failed");
  m->K = K;
  m->max_batch = max_batch;
  m->lay = L;
  const size_t B = max_batch;
  auto bad = [&](hipError_t e) {
    fepll_mlp_destroy(m);
    return fail(e == hipErrorOutOfMemory ? FEPLL_ENOMEM : FEPLL_EDEVICE,
                std::string("device setup failed: ") + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = dalloc(&m->p, L.n)) || (e = dalloc(&m->g, L.n)) || (e = dalloc(&m->m, L.n)) ||
      (e = dalloc(&m->v, L.n)) || (e = dalloc(&m->A1, B * kHidden)) ||
      (e = dalloc(&m->H1, B * kHidden)) || (e = dalloc(&m->A2, B * kHidden)) ||
      (e = dalloc(&m->H2, B * kHidden)) || (e = dalloc(&m->Z, B * K)) ||
      (e = dalloc(&m->dZ, B * K)) || (e = dalloc(&m->dH, B * kHidden)) ||
      (e = dalloc(&m->dA, B * kHidden)) || (e = dalloc(&m->loss_rows, B)) ||
      (e = dalloc(&m->Xb, B * kFeat)) || (e = dalloc(&m->yb, B)))
    return bad(e);
  if ((e = hipMemcpy(m->p, params, L.n * sizeof(float), hipMemcpyHostToDevice)) ||
      (e = hipMemset(m->m, 0, L.n * sizeof(float))) ||
      (e = hipMemset(m->v, 0, L.n * sizeof(float))) ||
      (e = hipMemset(m->g, 0, L.n * sizeof(float))))
    return bad(e);
  *out = m;
  return FEPLL_OK;
}

void fepll_mlp_destroy(fepll_mlp* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  dfree(m->p);
  dfree(m->g);
  dfree(m->m);
  dfree(m->v);
  dfree(m->A1);
  dfree(m->H1);
  dfree(m->A2);
  dfree(m->H2);
  dfree(m->Z);
  dfree(m->dZ);
  dfree(m->dH);
  dfree(m->dA);
  dfree(m->loss_rows);
  dfree(m->Xb);
  dfree(m->yb);
  delete m;
}

fepll_status fepll_mlp_get_params(fepll_mlp* m, float* params) {
  clear_error();
  if (!m || !params) return fail(FEPLL_EINVAL, "NULL argument");
  HIPX(hipDeviceSynchronize());
  HIPX(hipMemcpy(params, m->p, m->lay.n * sizeof(float), hipMemcpyDeviceToHost));
  return FEPLL_OK;
}

fepll_status fepll_mlp_forward(fepll_mlp* m, const float* X, int32_t n, float* logits,
                               void* stream) {
  clear_error();
  if (!m || !X || !logits) return fail(FEPLL_EINVAL, "NULL argument");
  if (n < 0) return fail(FEPLL_EINVAL, "n < 0");
  hipStream_t st = (hipStream_t)stream;
  for (int s0 = 0; s0 < n; s0 += m->max_batch) {
    const int c = std::min(m->max_batch, n - s0);
    fepll_status s = forward_chunk(m, X + (size_t)s0 * kFeat, c, logits + (size_t)s0 * m->K, st);
    if (s != FEPLL_OK) return s;
  }
  return FEPLL_OK;
}

fepll_status fepll_mlp_loss_grad(fepll_mlp* m, const float* X, const int32_t* labels, int32_t n,
                                 float* grads, float* loss, void* stream) {
  clear_error();
  if (!m || !X || !labels) return fail(FEPLL_EINVAL, "NULL argument");
  if (n < 1 || n > m->max_batch) return fail(FEPLL_EINVAL, "n must be in 1..max_batch");
  hipStream_t st = (hipStream_t)stream;
  fepll_status s = loss_grad(m, X, labels, n, loss, st);
  if (s != FEPLL_OK) return s;
  if (loss) {
    hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(1), 0, st, loss, 1.f / n);
    HIPX(hipGetLastError());
  }
  if (grads)
    HIPX(hipMemcpyAsync(grads, m->g, m->lay.n * sizeof(float), hipMemcpyDeviceToDevice, st));
  return FEPLL_OK;
}

fepll_status fepll_mlp_train_step(fepll_mlp* m, const float* X, const int32_t* labels,
                                  const int32_t* rows, int32_t n, const fepll_adamw* hp,
                                  float* loss, void* stream) {
  clear_error();
  if (!m || !X || !labels || !hp) return fail(FEPLL_EINVAL, "NULL argument");
  if (n < 1 || n > m->max_batch) return fail(FEPLL_EINVAL, "n must be in 1..max_batch");
  if (!(hp->lr >= 0) || !(hp->beta1 >= 0 && hp->beta1 < 1) || !(hp->beta2 >= 0 && hp->beta2 < 1) ||
      !(hp->eps > 0) || !(hp->weight_decay >= 0))
    return fail(FEPLL_EINVAL, "AdamW hyper-parameters out of range");
  hipStream_t st = (hipStream_t)stream;
  if (rows) {
    hipLaunchKernelGGL(gather_rows_kernel, dim3(n), dim3(64), 0, st, X, labels, rows, n, m->Xb,
                       m->yb);
    HIPX(hipGetLastError());
    X = m->Xb;
    labels = m->yb;
  }
  fepll_status s = loss_grad(m, X, labels, n, loss, st);
  if (s != FEPLL_OK) return s;
  if (loss) {
    hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(1), 0, st, loss, 1.f / n);
    HIPX(hipGetLastError());
  }
  m->step += 1;
  HIPX(launch_adamw(m->p, m->g, m->m, m->v, (int)m->lay.n, (float)hp->lr, (float)hp->beta1,
                    (float)hp->beta2, (float)hp->eps, (float)hp->weight_decay, m->step, st));
  return FEPLL_OK;
}

fepll_status fepll_features(const fepll_image* x, double beta, float* X, void* stream) {
  clear_error();
  if (!x || !x->data || !X) return fail(FEPLL_EINVAL, "NULL argument");
  if (!x->on_device) return fail(FEPLL_EINVAL, "fepll_features takes a device image");
  if (x->height < 8 || x->width < 8 || x->row_stride < x->width)
    return fail(FEPLL_EINVAL, "image shape");
  if (!(beta > 0) || !std::isfinite(beta)) return fail(FEPLL_EINVAL, "beta must be > 0");
  HIPX(launch_features(x->data, x->height, x->width, x->row_stride, beta, X,
                       (hipStream_t)stream));
  return FEPLL_OK;
}

fepll_status fepll_mlp_serialize(fepll_mlp* m, void* buf, size_t cap, size_t* nbytes) {
  clear_error();
  if (!m || !nbytes) return fail(FEPLL_EINVAL, "NULL argument");
  const size_t need = sizeof(BlobHeader) + m->lay.n * sizeof(float);
  *nbytes = need;
  if (!buf) return FEPLL_OK;
  if (cap < need) return fail(FEPLL_EINVAL, "buffer too small");
  std::vector<float> p(m->lay.n);
  HIPX(hipDeviceSynchronize());
  HIPX(hipMemcpy(p.data(), m->p, p.size() * sizeof(float), hipMemcpyDeviceToHost));
  BlobHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, "FEPLLMLP", 8);
  h.version = 1;
  h.K = m->K;
  h.d_in = kFeat;
  h.hidden = kHidden;
  h.scale_in = kScaleIn;
  h.gelu = 2;
  h.nparam = m->lay.n;
  h.checksum = fnv1a(p.data(), p.size() * sizeof(float));
  std::memcpy(buf, &h, sizeof(h));
  std::memcpy(static_cast<char*>(buf) + sizeof(h), p.data(), p.size() * sizeof(float));
  return FEPLL_OK;
}

}  // extern "C"

namespace fepll {

// Validates a serialized network; on success fills params (host).
fepll_status parse_proposal_blob(const void* blob, size_t nbytes, int K,
                                 std::vector<float>& params) {
  if (!blob) return fail(FEPLL_EINVAL, "blob is NULL");
  if (nbytes < sizeof(BlobHeader)) return fail(FEPLL_EINVAL, "blob shorter than its header");
  BlobHeader h;
  std::memcpy(&h, blob, sizeof(h));
  if (std::memcmp(h.magic, "FEPLLMLP", 8) != 0 || h.version != 1)
    return fail(FEPLL_EINVAL, "not a proposal network blob (magic/version)");
  if ((int)h.K != K) return fail(FEPLL_EINVAL, "network K differs from the mixture's K");
  if (h.d_in != (uint32_t)kFeat || h.hidden != (uint32_t)kHidden || h.scale_in != kScaleIn ||
      h.gelu != 2)
    return fail(FEPLL_EINVAL, "network shape, input scale or GELU variant not supported");
  const MlpLayout L(K);
  if (h.nparam != L.n || nbytes != sizeof(BlobHeader) + L.n * sizeof(float))
    return fail(FEPLL_EINVAL, "blob size does not match its parameter count");
  params.resize(L.n);
  std::memcpy(params.data(), static_cast<const char*>(blob) + sizeof(BlobHeader),
              L.n * sizeof(float));
  if (fnv1a(params.data(), L.n * sizeof(float)) != h.checksum)
    return fail(FEPLL_ECHECKSUM, "parameter checksum mismatch");
  for (float f : params)
    if (!std::isfinite(f)) return fail(FEPLL_EINVAL, "blob has a non-finite parameter");
  return FEPLL_OK;
}

}  // namespace fepll

namespace fepll {

namespace {
uint16_t host_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
}  // namespace

size_t proposal_wb_count(int K) {
  const int n3 = (K + 31) / 32;
  return (size_t)(8 * 5 + 8 * 16 + n3 * 16) * 64 * 8;
}

size_t proposal_bias_count(int K) { return 2 * kHidden + 32 * (size_t)((K + 31) / 32); }

// MFMA A-operand order of propose.hip: slab (layer, 32-row block nt), depth
// step s, lane l, element e holds W[32 nt + (l & 31)][16 s + 8 (l >> 5) + e].
void pack_proposal(const float* params, int K, uint16_t* wb, float* bias) {
  const MlpLayout L(K);
  const int n3 = (K + 31) / 32;
  size_t o = 0;
  auto layer = [&](const float* Wm, int rows, int cols, int nblk, int nsteps) {
    for (int nt = 0; nt < nblk; ++nt)
      for (int s = 0; s < nsteps; ++s)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e) {
            const int row = 32 * nt + (l & 31);
            const int k = 16 * s + 8 * (l >> 5) + e;
            const float v = (row < rows && k < cols) ? Wm[(size_t)row * cols + k] : 0.f;
            wb[o++] = host_bf16(v);
          }
  };
  layer(params + L.W1, kHidden, kFeat, 8, 5);
  layer(params + L.W2, kHidden, kHidden, 8, 16);
  layer(params + L.W3, K, kHidden, n3, 16);
  for (int i = 0; i < kHidden; ++i) bias[i] = params[L.b1 + i];
  for (int i = 0; i < kHidden; ++i) bias[kHidden + i] = params[L.b2 + i];
  for (int i = 0; i < 32 * n3; ++i)
    bias[2 * kHidden + i] = (i < K) ? params[L.b3 + i] : -INFINITY;
}

}  // namespace fepll
