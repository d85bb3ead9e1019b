// Host runtime behind include/fepll.h: argument validation, device copies of
// the mixture, the per-beta constant cache, scratch memory, and the
// per-iteration launch sequence of Alg. 1 (selection -> float64 recheck ->
// bucketing -> patch estimation -> reprojection + image estimation).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "fepll.h"
#include "internal.h"
#include "propose.h"

using namespace fepll;

namespace fepll {
fepll_status parse_proposal_blob(const void* blob, size_t nbytes, int K, std::vector<float>& params);
}

namespace {
thread_local std::string g_err;

__global__ void zero_i32_kernel(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
}  // namespace

namespace fepll {
fepll_status fail(fepll_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
void clear_error() { g_err.clear(); }
}  // namespace fepll

struct fepll_gmm {
  int K = 0;
  int device = 0;
  double* U64 = nullptr;    // [K][64][64]
  double* lam64 = nullptr;  // [K][64]
  double* w64 = nullptr;    // [K]
  // per-schedule constants
  bool have_sched = false;
  Schedule sched{};
  int T_cap = 0;
  float* Ut = nullptr;
  uint16_t* Ub = nullptr;
  float* Wt = nullptr;
  float* L32 = nullptr;
  double* L64 = nullptr;
  double* invnu64 = nullptr;
  uint8_t* Uf = nullptr;
  int32_t* Ue = nullptr;
  // scratch
  size_t np_cap = 0, px_cap = 0;
  int32_t* labels = nullptr;
  int32_t* list = nullptr;
  int32_t* count = nullptr;
  int32_t* hist = nullptr;
  int32_t* seg = nullptr;
  int32_t* perm = nullptr;
  float* Zhat = nullptr;
  float* ybuf = nullptr;
  float* xa = nullptr;
  float* xb = nullptr;
  // proposal network (bfloat16 inference layout) and its scratch
  uint16_t* pWb = nullptr;
  float* pbias = nullptr;
  bool has_proposal = false;
  uint16_t* cand = nullptr;   // Np x 8
  int32_t* fb_list = nullptr;  // Np
  hipStream_t last_stream = nullptr;
  bool used = false;
  // profiling: events recorded around stages, resolved in fepll_profile
  struct Mark {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  bool profiling = false;
};

namespace {

constexpr int kStages = 8;

hipEvent_t take_event(fepll_gmm* g) {
  if (!g->pool.empty()) {
    hipEvent_t e = g->pool.back();
    g->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one stage with events when profiling is on.
struct StageTimer {
  fepll_gmm* g;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  StageTimer(fepll_gmm* g_, int s_, hipStream_t st_) : g(g_), stage(s_), st(st_) {
    if (g->profiling && (a = take_event(g))) (void)hipEventRecord(a, st);
  }
  ~StageTimer() {
    if (!a) return;
    hipEvent_t b = take_event(g);
    if (!b) {
      g->pool.push_back(a);
      return;
    }
    (void)hipEventRecord(b, st);
    g->marks.push_back({stage, a, b});
  }
};

fepll_status use_stream(fepll_gmm* g, hipStream_t st) {
  // scratch is shared by every call on the handle: work left on another
  // stream must finish before this call reuses it
  if (g->used && g->last_stream != st) HIPX(hipStreamSynchronize(g->last_stream));
  g->last_stream = st;
  g->used = true;
  return FEPLL_OK;
}

fepll_status ensure_consts(fepll_gmm* g, const Schedule& s, hipStream_t st) {
  if (g->have_sched && g->sched.T == s.T &&
      std::memcmp(g->sched.beta, s.beta, sizeof(double) * s.T) == 0)
    return FEPLL_OK;
  if (s.T > g->T_cap) {
    dfree(g->Ut);
    dfree(g->Ub);
    dfree(g->Wt);
    dfree(g->L32);
    dfree(g->L64);
    dfree(g->invnu64);
    dfree(g->Uf);
    dfree(g->Ue);
    g->T_cap = 0;
    const size_t K = g->K;
    HIPX(dalloc(&g->Ut, (size_t)s.T * K * kTileStride));
    HIPX(dalloc(&g->Ub, (size_t)s.T * K * kTileStride));
    HIPX(dalloc(&g->Wt, (size_t)s.T * K * kTileStride));
    HIPX(dalloc(&g->L32, (size_t)s.T * K));
    HIPX(dalloc(&g->L64, (size_t)s.T * K));
    HIPX(dalloc(&g->invnu64, (size_t)s.T * K * kP));
    HIPX(dalloc(&g->Uf, (size_t)s.T * K * kTileStride));
    HIPX(dalloc(&g->Ue, (size_t)s.T * K));
    g->T_cap = s.T;
  }
  {
    StageTimer tm(g, 5, st);
    HIPX(launch_prep(g->U64, g->lam64, g->w64, g->K, s, g->Ut, g->Ub, g->Wt, g->L32, g->L64,
                     g->invnu64, g->Uf, g->Ue, st));
  }
  g->sched = s;
  g->have_sched = true;
  return FEPLL_OK;
}

fepll_status ensure_ws(fepll_gmm* g, int H, int W) {
  const size_t Np = (size_t)(H - 7) * (W - 7);
  const size_t px = (size_t)H * W;
  if (Np > g->np_cap) {
    dfree(g->labels);
    dfree(g->list);
    dfree(g->count);
    dfree(g->hist);
    dfree(g->seg);
    dfree(g->perm);
    dfree(g->Zhat);
    dfree(g->cand);
    dfree(g->fb_list);
    g->np_cap = 0;
    const size_t nb = (Np + kSortBlock - 1) / kSortBlock;
    HIPX(dalloc(&g->labels, Np));
    HIPX(dalloc(&g->list, 4 * Np));  // int4 entries
    HIPX(dalloc(&g->count, 64));
    HIPX(dalloc(&g->hist, nb * g->K));
    HIPX(dalloc(&g->seg, seg_size(Np, g->K)));
    HIPX(dalloc(&g->perm, Np));
    HIPX(dalloc(&g->Zhat, Np * kP));
    HIPX(dalloc(&g->cand, Np * 8));
    HIPX(dalloc(&g->fb_list, Np));
    g->np_cap = Np;
  }
  if (px > g->px_cap) {
    dfree(g->ybuf);
    dfree(g->xa);
    dfree(g->xb);
    g->px_cap = 0;
    HIPX(dalloc(&g->ybuf, px));
    HIPX(dalloc(&g->xa, px));
    HIPX(dalloc(&g->xb, px));
    g->px_cap = px;
  }
  return FEPLL_OK;
}

fepll_status check_image(const fepll_image* im, const char* what) {
  if (!im) return fail(FEPLL_EINVAL, std::string(what) + " is NULL");
  if (!im->data) return fail(FEPLL_EINVAL, std::string(what) + "->data is NULL");
  if (im->height < 8 || im->width < 8)
    return fail(FEPLL_EINVAL, std::string(what) + ": height and width must be >= 8");
  if (im->row_stride < im->width)
    return fail(FEPLL_EINVAL, std::string(what) + ": row_stride < width");
  if ((int64_t)(im->height - 7) * (im->width - 7) > (int64_t)INT32_MAX / kP)
    return fail(FEPLL_EUNSUPPORTED, std::string(what) + ": image too large");
  return FEPLL_OK;
}

fepll_status host_finite(const fepll_image* im, const char* what) {
  if (im->on_device) return FEPLL_OK;
  for (int r = 0; r < im->height; ++r) {
    const float* row = im->data + (size_t)r * im->row_stride;
    for (int c = 0; c < im->width; ++c)
      if (!std::isfinite(row[c]))
        return fail(FEPLL_EINVAL, std::string(what) + " has a non-finite value");
  }
  return FEPLL_OK;
}

hipError_t copy_in(float* dst, const fepll_image* im, hipStream_t st) {
  return hipMemcpy2DAsync(dst, (size_t)im->width * 4, im->data, (size_t)im->row_stride * 4,
                          (size_t)im->width * 4, im->height,
                          im->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st);
}

hipError_t copy_out(fepll_image* im, const float* src, hipStream_t st) {
  return hipMemcpy2DAsync(im->data, (size_t)im->row_stride * 4, src, (size_t)im->width * 4,
                          (size_t)im->width * 4, im->height,
                          im->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st);
}

fepll_status check_opt(const fepll_gmm* g, const fepll_options* o) {
  if (o->precision != FEPLL_FP32 && o->precision != FEPLL_BF16 && o->precision != FEPLL_FP8)
    return fail(FEPLL_EINVAL, "options.precision must be FEPLL_FP32, FEPLL_BF16 or FEPLL_FP8");
  if (o->use_proposal) {
    if (!g->has_proposal) return fail(FEPLL_EINVAL, "no proposal network is loaded");
    if (o->top_m < 1 || o->top_m > 8 || o->top_m > g->K)
      return fail(FEPLL_EINVAL, "options.top_m out of 1..min(8, K)");
    if (o->precision != FEPLL_BF16)
      return fail(FEPLL_EUNSUPPORTED, "the proposal path runs with FEPLL_BF16 projections");
  }
  if (std::isnan(o->margin_nats)) return fail(FEPLL_EINVAL, "options.margin_nats is NaN");
  return FEPLL_OK;
}

// One Gaussian selection (E-step + optional float64 recheck) of image x.
__global__ void mark_kernel(const int32_t* count, const int32_t* list, int32_t* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < *count) flags[list[i]] = 1;
}

fepll_status run_select(fepll_gmm* g, const float* x, int H, int W, int t, double beta,
                        int precision, bool recheck, const fepll_options* prop, int32_t* labels,
                        float* best, float* second, int32_t* flags, hipStream_t st) {
  const int Np = (H - 7) * (W - 7);
  const size_t K = g->K;
  if (precision == FEPLL_FP8) {
    if (flags) {
      hipLaunchKernelGGL(zero_i32_kernel, dim3((Np + 255) / 256), dim3(256), 0, st, flags, Np);
      HIPX(hipGetLastError());
    }
    StageTimer tm(g, 0, st);
    HIPX(launch_estep_fp8(x, H, W, g->Uf + (size_t)t * K * kTileStride, g->Ue + (size_t)t * K,
                          g->L32 + (size_t)t * K, g->K, labels, best, second, st));
    return FEPLL_OK;
  }
  if (precision == FEPLL_BF16) {
    if (flags) {
      hipLaunchKernelGGL(zero_i32_kernel, dim3((Np + 255) / 256), dim3(256), 0, st, flags, Np);
      HIPX(hipGetLastError());
    }
    if (!prop) {
      StageTimer tm(g, 0, st);
      HIPX(launch_estep_bf16(x, H, W, g->Ub + (size_t)t * K * kTileStride,
                             g->L32 + (size_t)t * K, g->K, labels, best, second, st));
      return FEPLL_OK;
    }
    {
      StageTimer tm(g, 6, st);
      HIPX(launch_propose_bf16(x, H, W, beta, g->pWb, g->pbias, g->K, prop->top_m, g->cand, st));
    }
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, g->count, 1);
    HIPX(hipGetLastError());
    BF16Args a{};
    a.x = x;
    a.H = H;
    a.W = W;
    a.Ub = g->Ub + (size_t)t * K * kTileStride;
    a.L = g->L32 + (size_t)t * K;
    a.K = g->K;
    a.labels = labels;
    a.best = best;
    a.second = second;
    a.cand = reinterpret_cast<const uint4*>(g->cand);
    a.margin = (float)prop->margin_nats;
    a.fb_count = g->count;
    a.fb_list = g->fb_list;
    a.list_count = g->count;
    a.list = g->fb_list;
    {
      StageTimer tm(g, 0, st);
      HIPX(launch_estep_bf16_mode(kModeSpatialCand, a, st));
    }
    {
      StageTimer tm(g, 7, st);
      HIPX(launch_estep_bf16_mode(kModeListFull, a, st));
    }
    if (flags) {
      hipLaunchKernelGGL(mark_kernel, dim3((Np + 255) / 256), dim3(256), 0, st, g->count,
                         g->fb_list, flags);
      HIPX(hipGetLastError());
    }
    return FEPLL_OK;
  }
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, g->count, 1);
  HIPX(hipGetLastError());
  {
    StageTimer tm(g, 0, st);
    HIPX(launch_estep_f32(x, H, W, g->Ut + (size_t)t * K * kTileStride,
                          g->L32 + (size_t)t * K, g->K, beta, labels, best, second, flags,
                          g->count, recheck ? g->list : nullptr, st));
  }
  if (recheck) {
    StageTimer tm(g, 1, st);
    HIPX(launch_recheck_f64(x, H, W, g->U64, g->invnu64 + (size_t)t * K * kP,
                            g->L64 + (size_t)t * K, g->K, g->count, g->list, labels, Np, st));
  }
  return FEPLL_OK;
}

}  // namespace

extern "C" {

void fepll_options_default(fepll_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = FEPLL_FP32;
  o->recheck = 1;
  o->use_proposal = 0;
  o->top_m = 8;
  o->margin_nats = 0.5;
  o->init = nullptr;
  o->stream = nullptr;
  o->profile = 0;
}

const char* fepll_last_error(void) { return g_err.c_str(); }

const char* fepll_version(void) { return "fepll-gfx950 0.1"; }

fepll_status fepll_gmm_create(const double* U, const double* lambda, const double* w, int32_t K,
                              int32_t d, fepll_gmm** out) {
  g_err.clear();
  if (!out) return fail(FEPLL_EINVAL, "out is NULL");
  if (!U || !lambda || !w) return fail(FEPLL_EINVAL, "U, lambda and w must be non-NULL");
  if (d != kP) return fail(FEPLL_EINVAL, "d must be 64 (8x8 patches)");
  if (K < 1 || K > kMaxK) return fail(FEPLL_EINVAL, "K must be in 1..1024");
  double wsum = 0.0;
  for (int k = 0; k < K; ++k) {
    if (!(w[k] > 0.0) || !std::isfinite(w[k]))
      return fail(FEPLL_EINVAL, "weights must be finite and > 0");
    wsum += w[k];
    for (int j = 0; j < d; ++j) {
      const double l = lambda[(size_t)k * d + j];
      if (!std::isfinite(l) || l < 0.0)
        return fail(FEPLL_EINVAL, "eigenvalues must be finite and >= 0");
    }
  }
  if (std::fabs(wsum - 1.0) > 1e-6) return fail(FEPLL_EINVAL, "weights must sum to 1 (1e-6)");
  for (int k = 0; k < K; ++k) {
    const double* u = U + (size_t)k * d * d;
    for (int a = 0; a < d; ++a)
      for (int b = a; b < d; ++b) {
        double s = 0.0;
        for (int p = 0; p < d; ++p) s += u[p * d + a] * u[p * d + b];
        if (!std::isfinite(s) || std::fabs(s - (a == b ? 1.0 : 0.0)) > 1e-8)
          return fail(FEPLL_EINVAL, "U_" + std::to_string(k) + " is not orthonormal (1e-8)");
      }
  }
  fepll_gmm* g = new (std::nothrow) fepll_gmm();
  if (!g) return fail(FEPLL_ENOMEM, "host allocation failed");
  g->K = K;
  auto bad = [&](hipError_t e) {
    fepll_gmm_destroy(g);
    return fail(e == hipErrorOutOfMemory ? FEPLL_ENOMEM : FEPLL_EDEVICE,
                std::string("device setup failed: ") + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipGetDevice(&g->device)) != hipSuccess) return bad(e);
  if ((e = dalloc(&g->U64, (size_t)K * d * d)) != hipSuccess) return bad(e);
  if ((e = dalloc(&g->lam64, (size_t)K * d)) != hipSuccess) return bad(e);
  if ((e = dalloc(&g->w64, (size_t)K)) != hipSuccess) return bad(e);
  if ((e = hipMemcpy(g->U64, U, sizeof(double) * K * d * d, hipMemcpyHostToDevice)) != hipSuccess)
    return bad(e);
  if ((e = hipMemcpy(g->lam64, lambda, sizeof(double) * K * d, hipMemcpyHostToDevice)) !=
      hipSuccess)
    return bad(e);
  if ((e = hipMemcpy(g->w64, w, sizeof(double) * K, hipMemcpyHostToDevice)) != hipSuccess)
    return bad(e);
  *out = g;
  return FEPLL_OK;
}

fepll_status fepll_profile(fepll_gmm* g, double* ms, int32_t* launches, int32_t n) {
  g_err.clear();
  if (!g) return fail(FEPLL_EINVAL, "gmm handle is NULL");
  if (n < 0) return fail(FEPLL_EINVAL, "n < 0");
  double acc[kStages] = {0};
  int32_t cnt[kStages] = {0};
  fepll_status ret = FEPLL_OK;
  for (auto& m : g->marks) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(m.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, m.a, m.b);
    if (e != hipSuccess && ret == FEPLL_OK)
      ret = fail(FEPLL_EDEVICE, std::string("event timing failed: ") + hipGetErrorString(e));
    acc[m.stage] += t;
    cnt[m.stage] += 1;
    g->pool.push_back(m.a);
    g->pool.push_back(m.b);
  }
  g->marks.clear();
  for (int i = 0; i < n && i < kStages; ++i) {
    if (ms) ms[i] = acc[i];
    if (launches) launches[i] = cnt[i];
  }
  return ret;
}

void fepll_gmm_destroy(fepll_gmm* g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  for (auto& m : g->marks) {
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  for (auto e : g->pool) (void)hipEventDestroy(e);
  dfree(g->U64);
  dfree(g->lam64);
  dfree(g->w64);
  dfree(g->Ut);
  dfree(g->Ub);
  dfree(g->Wt);
  dfree(g->L32);
  dfree(g->L64);
  dfree(g->invnu64);
  dfree(g->Uf);
  dfree(g->Ue);
  dfree(g->labels);
  dfree(g->list);
  dfree(g->count);
  dfree(g->hist);
  dfree(g->seg);
  dfree(g->perm);
  dfree(g->Zhat);
  dfree(g->cand);
  dfree(g->fb_list);
  dfree(g->pWb);
  dfree(g->pbias);
  dfree(g->ybuf);
  dfree(g->xa);
  dfree(g->xb);
  delete g;
}

fepll_status fepll_restore(fepll_gmm* g, const fepll_image* y, const void* Hop, double sigma,
                           const double* beta_schedule, int32_t T, fepll_image* out,
                           const fepll_options* opt, int32_t* labels_out) {
  g_err.clear();
  if (!g) return fail(FEPLL_EINVAL, "gmm handle is NULL");
  fepll_status s;
  if ((s = check_image(y, "y")) != FEPLL_OK) return s;
  if ((s = check_image(out, "out")) != FEPLL_OK) return s;
  if (Hop) return fail(FEPLL_EUNSUPPORTED, "only the identity degradation (H = NULL) is supported");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(FEPLL_EINVAL, "sigma must be > 0");
  if (out->height != y->height || out->width != y->width)
    return fail(FEPLL_EINVAL, "out must have the shape of y");
  fepll_options o;
  fepll_options_default(&o);
  if (opt) o = *opt;
  if ((s = check_opt(g, &o)) != FEPLL_OK) return s;
  Schedule sch{};
  if (!beta_schedule) {
    if (T != 0 && T != 5) return fail(FEPLL_EINVAL, "default schedule has T = 5");
    sch.T = 5;
    const double m[5] = {1.0, 4.0, 8.0, 16.0, 32.0};
    for (int t = 0; t < 5; ++t) sch.beta[t] = m[t] / (sigma * sigma);
  } else {
    if (T < 1 || T > kMaxT) return fail(FEPLL_EINVAL, "T must be in 1..16");
    sch.T = T;
    for (int t = 0; t < T; ++t) {
      if (!(beta_schedule[t] > 0.0) || !std::isfinite(beta_schedule[t]))
        return fail(FEPLL_EINVAL, "beta values must be finite and > 0");
      sch.beta[t] = beta_schedule[t];
    }
  }
  if (o.init) {
    if ((s = check_image(o.init, "options.init")) != FEPLL_OK) return s;
    if (o.init->height != y->height || o.init->width != y->width)
      return fail(FEPLL_EINVAL, "options.init must have the shape of y");
    if ((s = host_finite(o.init, "options.init")) != FEPLL_OK) return s;
  }
  if ((s = host_finite(y, "y")) != FEPLL_OK) return s;

  const int H = y->height, W = y->width;
  const int Np = (H - 7) * (W - 7);
  hipStream_t st = (hipStream_t)o.stream;
  if ((s = use_stream(g, st)) != FEPLL_OK) return s;
  g->profiling = o.profile != 0;
  if ((s = ensure_ws(g, H, W)) != FEPLL_OK) return s;
  if ((s = ensure_consts(g, sch, st)) != FEPLL_OK) return s;

  HIPX(copy_in(g->ybuf, y, st));
  if (o.init) HIPX(copy_in(g->xa, o.init, st));
  else HIPX(hipMemcpyAsync(g->xa, g->ybuf, sizeof(float) * H * W, hipMemcpyDeviceToDevice, st));

  float* xc = g->xa;
  float* xn = g->xb;
  for (int t = 0; t < sch.T; ++t) {
    const double beta = sch.beta[t];
    if ((s = run_select(g, xc, H, W, t, beta, o.precision, o.recheck != 0,
                        o.use_proposal ? &o : nullptr, g->labels, nullptr, nullptr, nullptr,
                        st)) != FEPLL_OK)
      return s;
    if (labels_out)
      HIPX(hipMemcpyAsync(labels_out + (size_t)t * Np, g->labels, sizeof(int32_t) * Np,
                          y->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    {
      StageTimer tm(g, 2, st);
      HIPX(launch_bucket(g->labels, Np, g->K, g->hist, g->seg, g->perm, st));
    }
    {
      StageTimer tm(g, 3, st);
      HIPX(launch_wiener_f32(xc, H, W, g->Wt + (size_t)t * g->K * kTileStride, g->K, g->seg,
                             g->perm, g->Zhat, st));
    }
    {
      StageTimer tm(g, 4, st);
      HIPX(launch_ola_update(g->Zhat, g->ybuf, H, W, beta * sigma * sigma, xn, st));
    }
    std::swap(xc, xn);
  }
  HIPX(copy_out(out, xc, st));
  if (!out->on_device || !y->on_device || (labels_out && !y->on_device))
    HIPX(hipStreamSynchronize(st));
  return FEPLL_OK;
}

fepll_status fepll_gmm_load_proposal(fepll_gmm* g, const void* blob, size_t nbytes) {
  g_err.clear();
  if (!g) return fail(FEPLL_EINVAL, "gmm handle is NULL");
  std::vector<float> params;
  fepll_status s = parse_proposal_blob(blob, nbytes, g->K, params);
  if (s != FEPLL_OK) return s;
  std::vector<uint16_t> wb(proposal_wb_count(g->K));
  std::vector<float> bias(proposal_bias_count(g->K));
  pack_proposal(params.data(), g->K, wb.data(), bias.data());
  HIPX(hipDeviceSynchronize());
  dfree(g->pWb);
  dfree(g->pbias);
  g->has_proposal = false;
  HIPX(dalloc(&g->pWb, wb.size()));
  HIPX(dalloc(&g->pbias, bias.size()));
  HIPX(hipMemcpy(g->pWb, wb.data(), wb.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  HIPX(hipMemcpy(g->pbias, bias.data(), bias.size() * sizeof(float), hipMemcpyHostToDevice));
  g->has_proposal = true;
  return FEPLL_OK;
}

fepll_status fepll_propose(fepll_gmm* g, const fepll_image* x, double beta, int32_t top_m,
                           uint16_t* cand, void* stream) {
  g_err.clear();
  if (!g) return fail(FEPLL_EINVAL, "gmm handle is NULL");
  fepll_status s;
  if ((s = check_image(x, "x")) != FEPLL_OK) return s;
  if (!x->on_device) return fail(FEPLL_EINVAL, "fepll_propose takes a device image");
  if (!cand) return fail(FEPLL_EINVAL, "cand is NULL");
  if (!g->has_proposal) return fail(FEPLL_EINVAL, "no proposal network is loaded");
  if (top_m < 1 || top_m > 8 || top_m > g->K) return fail(FEPLL_EINVAL, "top_m out of range");
  if (!(beta > 0.0) || !std::isfinite(beta)) return fail(FEPLL_EINVAL, "beta must be > 0");
  const int H = x->height, W = x->width;
  hipStream_t st = (hipStream_t)stream;
  if ((s = use_stream(g, st)) != FEPLL_OK) return s;
  if ((s = ensure_ws(g, H, W)) != FEPLL_OK) return s;
  HIPX(copy_in(g->xa, x, st));
  HIPX(launch_propose_bf16(g->xa, H, W, beta, g->pWb, g->pbias, g->K, top_m, cand, st));
  return FEPLL_OK;
}

fepll_status fepll_select(fepll_gmm* g, const fepll_image* x, double beta, int32_t* labels,
                          float* best, float* second, int32_t* flags, const fepll_options* opt) {
  g_err.clear();
  if (!g) return fail(FEPLL_EINVAL, "gmm handle is NULL");
  fepll_status s;
  if ((s = check_image(x, "x")) != FEPLL_OK) return s;
  if (!x->on_device) return fail(FEPLL_EINVAL, "fepll_select takes a device image");
  if (!labels) return fail(FEPLL_EINVAL, "labels is NULL");
  if (!(beta > 0.0) || !std::isfinite(beta)) return fail(FEPLL_EINVAL, "beta must be > 0");
  fepll_options o;
  fepll_options_default(&o);
  if (opt) o = *opt;
  if ((s = check_opt(g, &o)) != FEPLL_OK) return s;
  const int H = x->height, W = x->width;
  hipStream_t st = (hipStream_t)o.stream;
  if ((s = use_stream(g, st)) != FEPLL_OK) return s;
  g->profiling = o.profile != 0;
  if ((s = ensure_ws(g, H, W)) != FEPLL_OK) return s;
  Schedule sch{};
  sch.T = 1;
  sch.beta[0] = beta;
  if ((s = ensure_consts(g, sch, st)) != FEPLL_OK) return s;
  HIPX(copy_in(g->xa, x, st));
  return run_select(g, g->xa, H, W, 0, beta, o.precision, o.recheck != 0,
                    o.use_proposal ? &o : nullptr, labels, best, second, flags, st);
}

}  // extern "C"
