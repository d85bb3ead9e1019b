// Host runtime behind include/fepll.h: argument validation, device copies of
// the mixture, the per-beta constant cache, the packed layout of a batch of
// images ("plan"), scratch memory, and the per-iteration launch sequence of
// Alg. 1 (selection -> float64 recheck -> bucketing -> patch estimation ->
// reprojection + image estimation), run eagerly or replayed from a captured
// HIP graph.  A single restoration is a batch of one.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <unordered_map>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "fepll.h"
#include "internal.h"
#include "propose.h"
#include <rocprofiler-sdk-roctx/roctx.h>

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

__global__ void fill_i32_kernel(int32_t* p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// two buffers zeroed by one launch: p[0..n) and q[0..m), m <= n
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
  double* lam64 = nullptr;  // [K][64]: the spectra in use (flat-tailed or not)
  double* w64 = nullptr;    // [K]
  // the spectra as created, and the flat-tail approximation in use (Sec.
  // 3.1; rho = 1: none)
  std::vector<double> lam_h;
  std::vector<double> U_h;  // [K][64][64], as created
  double rho = 1.0;
  std::vector<int32_t> h_rk;
  int32_t* rk = nullptr;  // [K] kept ranks, device
  // per-beta constants of the beta slots of the last call
  std::vector<double> cbeta;
  int cmask = 0;
  size_t S_cap = 0;
  double* dbeta = nullptr;
  float* dlogsb = nullptr;  // log sigma_beta = -log(beta) / 2 of each slot (network input)
  ConstTables tb{};
  // plan of the last call: host copies (kept for the asynchronous uploads
  // and to skip unchanged uploads) and device copies
  std::vector<ImgDesc> hd;
  std::vector<int32_t> h_est, h_sort, h_ola, h_resc;
  std::vector<float> hbvals;
  Batch batch{};
  bool plan_valid = false;
  size_t n_cap = 0, wb_cap = 0, est_cap = 0, sort_cap = 0, ola_cap = 0, slot_cap = 0,
         resc_cap = 0, fb_cap = 0;
  ImgDesc* d = nullptr;
  int32_t* est_img = nullptr;
  int32_t* sort_img = nullptr;
  int32_t* ola_img = nullptr;
  int32_t* resc_img = nullptr;
  int32_t* wbase = nullptr;
  float* bvals = nullptr;
  // scratch, sized for the packed batch
  size_t np_cap = 0, px_cap = 0, hist_cap = 0, seg_cap = 0;
  int32_t* labels = nullptr;
  int32_t* list = nullptr;
  int32_t* count = nullptr;
  int32_t* hist = nullptr;
  int32_t* seg = nullptr;
  int32_t* perm = nullptr;
  float* Zhat = nullptr;
  // jittered subsampling: chosen-patch flags and lists (three sets of np_cap
  // each, packed like labels; iteration t uses set t % 3), list lengths per
  // image (four sets of n; iteration t appends to set t % 4)
  int32_t* jflags = nullptr;
  bool jflags_dirty = true;  // jflags may hold set entries (cleared on next use)
  int32_t* jlist = nullptr;
  size_t jcount_cap = 0;
  int32_t* jcount = nullptr;
  size_t jpart_cap = 0;
  float4* jpart = nullptr;  // partial results of the component-split list selection
  // the restoration under way sorts its lists in jit_nbl chunks per image
  // (0: no list sort), and the selection counts the chunks' labels itself
  int jit_nbl = 0;
  bool jit_hist = false;
  // ... and draws the next iteration's subset inside the reprojection
  bool jit_fused = false;
  // deblurring (periodic convolution): float64 FFT plans and spectra of the
  // last image size
  struct Deblur {
    int H = 0, W = 0;
    hipfftHandle fwd = 0, inv = 0;
    bool plans = false;
    size_t n_cap = 0, m_cap = 0;
    double* r = nullptr;      // H x W real
    double2* Hh = nullptr;    // half spectrum of the kernel
    double2* AtY = nullptr;   // conj(Hh) Yh
    double* a2 = nullptr;     // |Hh|^2
    double2* X = nullptr;     // scratch spectrum
  } db;
  // search tree (Sec. 3.2): all nodes, leaves first (ids 0..K-1), then the
  // levels above from the one over the leaves up to the root
  struct Tree {
    int Kall = 0, root = 0, nlevels = 0, maxch = 0;
    std::vector<int> lvl_size;           // root first
    std::vector<double> U_h, lam_h, w_h;  // all nodes, spectra before any flat tail
    double* U64 = nullptr;
    double* lam64 = nullptr;
    double* w64 = nullptr;
    int32_t* rk = nullptr;
    uint16_t* children = nullptr;  // [Kall][8]
    // the top levels scored densely (levels 1..dense_levels, each of at
    // most kDenseNodes nodes): node ids in level order, their parents' ids,
    // each level's end position
    int dense_levels = 0, dense_n = 0;
    int32_t* dnode = nullptr;
    int32_t* dpar = nullptr;
    int32_t* dlend = nullptr;
    ConstTables tb{};
    std::vector<double> cbeta;
    size_t S_cap = 0;
    double* dbeta = nullptr;
  } tree;
  uint64_t tree_gen = 0;  // counts fepll_gmm_set_tree calls
  float* ybuf = nullptr;
  float* xa = nullptr;
  float* xb = nullptr;
  // proposal network (bfloat16 inference layout) and its scratch
  uint16_t* pWb = nullptr;
  float* pbias = nullptr;
  bool has_proposal = false;
  uint16_t* cand = nullptr;   // 8 per patch, packed like the labels
  int32_t* fb_list = nullptr;  // fallback lists, packed like the labels
  int32_t* fbpart = nullptr;   // split fallback search: the parts' results (3 kFallbackSplit NP)
  int32_t* fbcnt = nullptr;    // fallback list length per image
  int32_t* fbitems = nullptr;  // fallback items: first of each image, then the total
  // the search tree's descent: patches grouped by node (pair sort scratch)
  size_t pair_cap = 0, phist_cap = 0, pseg_cap = 0;
  int32_t* psorted = nullptr;  // 8 Np
  // the patches' bfloat16 selection operands and squared norms, written for
  // the search tree's sparse levels
  size_t zop_cap = 0, znz_cap = 0;
  uint16_t* zop = nullptr;  // 64 Np
  float* znz = nullptr;     // Np
  int32_t* phist = nullptr;
  int32_t* pseg = nullptr;
  hipStream_t last_stream = nullptr;
  bool used = false;
  // launch shapes (fepll_set_tuning / fepll_autotune)
  fepll_tuning tune{};
  // the captured iteration loop of the last graph-eligible call
  hipGraphExec_t gexec = nullptr;
  std::vector<uint8_t> gkey;
  hipStream_t cap_stream = nullptr;
  // profiling: events recorded around stages, resolved in fepll_profile
  struct Mark {
    int stage;
    hipEvent_t a, b;
    bool own_a;  // false: a is the previous mark's b
  };
  hipEvent_t chain_ev = nullptr;  // the last stage's end event, for a stage that follows at once
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  uint32_t profiling = 0;  // bit s: stage s is timed
};

namespace fepll {
GmmView gmm_view(const fepll_gmm* g) { return GmmView{g->K, g->device, g->U64, g->lam64, g->w64}; }

namespace {
std::mutex g_mem_mu;
std::unordered_map<void*, size_t> g_mem_held;
size_t g_mem_in_use = 0;
size_t g_mem_limit = 0;  // 0: none
}  // namespace

hipError_t dev_alloc(void** p, size_t bytes) {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  *p = nullptr;
  if (g_mem_limit && g_mem_in_use + bytes > g_mem_limit) return hipErrorOutOfMemory;
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  g_mem_held[*p] = bytes;
  g_mem_in_use += bytes;
  return hipSuccess;
}

void dev_free(void* p) {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  auto it = g_mem_held.find(p);
  if (it != g_mem_held.end()) {
    g_mem_in_use -= it->second;
    g_mem_held.erase(it);
  }
  (void)hipFree(p);
}
}  // namespace fepll

namespace {

constexpr int kStages = 9;
constexpr int kDenseNodes = 16;  // tree levels of at most this many nodes are scored densely
constexpr int kDefaultT = 5;
// The full-K search of the proposal's fallback lists runs each item of 512
// listed patches as this many workgroups over shares of K (merged after):
// the lists hold a sixth of the patches or fewer, too few items to fill the
// chip otherwise.
constexpr int kFallbackSplit = 2;
const double kDefaultB[kDefaultT] = {1.0, 4.0, 8.0, 16.0, 32.0};

void default_tuning(fepll_tuning* t) {
  t->est_blocks = 768;  // 3 workgroups per compute unit
  t->wiener_blocks = 4096;
  t->ola_rows = 16;  // 1024 reprojection tiles at 1024^2: 6 us per iteration less than 32 rows
  t->reserved = 0;
}

// The tuning cache (a text file named by FEPLL_TUNING_CACHE): one line per
// autotuned workload, "fepll-tuning 1 <key> <est> <wiener> <ola>", the key
// naming what the launch shapes depend on: the device, the precision and
// selection path, K, and the batch's shape class (image count, total and
// largest image size, each to a power of two).  The last line for a key
// wins.
int log2_class(int64_t v) {
  int c = 0;
  while (v > 1) {
    v >>= 1;
    ++c;
  }
  return c;
}
std::string tuning_key(const fepll_gmm* g, const fepll_options& o, int n, int64_t total,
                       int64_t largest) {
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  const char* path = o.use_proposal ? "proposal" : o.use_tree ? "tree" : o.jitter ? "jitter" : "all";
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s:p%d:%s:flat%d:K%d:n%d:px%d:max%d", arch.c_str(),
                (int)o.precision, path, g->tb.rk ? 1 : 0, g->K, log2_class(n),
                log2_class(total), log2_class(largest));
  return buf;
}
bool tuning_lookup(const char* path, const std::string& key, fepll_tuning* t) {
  std::FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    char k[300];
    int ver = 0, e = 0, w = 0, r = 0;
    if (std::sscanf(line, "fepll-tuning %d %299s %d %d %d", &ver, k, &e, &w, &r) == 5 &&
        ver == 1 && key == k) {
      *t = fepll_tuning{e, w, r, 0};
      found = true;
    }
  }
  std::fclose(f);
  return found;
}
void tuning_store(const char* path, const std::string& key, const fepll_tuning& t) {
  std::FILE* f = std::fopen(path, "a");
  if (!f) return;  // a cache that cannot be written is no error
  std::fprintf(f, "fepll-tuning 1 %s %d %d %d\n", key.c_str(), t.est_blocks, t.wiener_blocks,
               t.ola_rows);
  std::fclose(f);
}

hipEvent_t take_event(fepll_gmm* g) {
  if (!g->pool.empty()) {
    hipEvent_t e = g->pool.back();
    g->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  // timing only: no system-scope fence (an L2 writeback and invalidation on
  // every record, which would slow the stages being timed)
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// The stages options.profile times: bit 0 every stage, else bit s + 1
// stage s.
uint32_t profile_mask(int32_t profile) {
  if (profile & 1) return 0xffffffffu;
  return (uint32_t)profile >> 1;
}

// A named range on the host timeline of a tracer (roctx; no cost without
// one): each HQS iteration of a restoration, and each call.
struct TraceRange {
  explicit TraceRange(const char* what, int t = -1) {
    char buf[64];
    if (t >= 0)
      std::snprintf(buf, sizeof buf, "%s %d", what, t + 1);
    else
      std::snprintf(buf, sizeof buf, "%s", what);
    roctxRangePushA(buf);
  }
  ~TraceRange() { roctxRangePop(); }
};

// Brackets one stage with events when profiling is on.
// chain: the stage follows the previous timed stage with no launch between,
// so the previous end event is its start (one record fewer).
struct StageTimer {
  fepll_gmm* g;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  bool own_a = true;
  StageTimer(fepll_gmm* g_, int s_, hipStream_t st_, bool chain = false)
      : g(g_), stage(s_), st(st_) {
    if (!((g->profiling >> stage) & 1u)) {
      g->chain_ev = nullptr;  // a timed stage after this one starts its own interval
      return;
    }
    if (chain && g->chain_ev) {
      a = g->chain_ev;
      own_a = false;
    } else if ((a = take_event(g))) {
      (void)hipEventRecord(a, st);
    }
    g->chain_ev = nullptr;
  }
  ~StageTimer() {
    if (!a) return;
    hipEvent_t b = take_event(g);
    if (!b) {
      if (own_a) g->pool.push_back(a);
      return;
    }
    (void)hipEventRecord(b, st);
    g->marks.push_back({stage, a, b, own_a});
    g->chain_ev = b;
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

int table_mask(const fepll_options& o) {
  if (o.precision == FEPLL_FP8) return kTabF8;
  if (o.precision == FEPLL_BF16) return kTabBF16;
  return kTabF32;
}

// Sec. 3.1 on n spectra of kP eigenvalues (in place): ranks r_k (kP: no
// tail) and the tail replaced by its average; the trace, the partial sums
// and the tail sum in index order.  rho >= 1: no change, ranks kP.
void flat_tail_host(std::vector<double>& lam, int n, double rho, std::vector<int32_t>& rk) {
  rk.assign(n, kP);
  if (rho >= 1.0) return;
  for (int k = 0; k < n; ++k) {
    double* l = lam.data() + (size_t)k * kP;
    double cum[kP];
    double c = 0.0;
    for (int j = 0; j < kP; ++j) cum[j] = (c += l[j]);
    const double goal = rho * cum[kP - 1];
    int r = kP;
    for (int j = 0; j < kP; ++j)
      if (cum[j] >= goal) {
        r = j + 1;
        break;
      }
    rk[k] = r;
    if (r < kP) {
      double tail = 0.0;
      for (int j = r; j < kP; ++j) tail += l[j];
      const double avg = tail / (kP - r);
      for (int j = r; j < kP; ++j) l[j] = avg;
    }
  }
}

// The tree's spectra on the device, flat-tailed like the mixture.
fepll_status tree_upload_spectra(fepll_gmm* g) {
  auto& T = g->tree;
  std::vector<double> lam = T.lam_h;
  std::vector<int32_t> rk;
  flat_tail_host(lam, T.Kall, g->rho, rk);
  HIPX(hipMemcpy(T.lam64, lam.data(), sizeof(double) * lam.size(), hipMemcpyHostToDevice));
  HIPX(hipMemcpy(T.rk, rk.data(), sizeof(int32_t) * rk.size(), hipMemcpyHostToDevice));
  T.tb.rk = (g->rho < 1.0) ? T.rk : nullptr;
  T.cbeta.clear();
  return FEPLL_OK;
}

// bfloat16 tables of the tree's nodes for the beta slots `betas`.
fepll_status ensure_tree_consts(fepll_gmm* g, const std::vector<double>& betas, hipStream_t st) {
  auto& T = g->tree;
  if (T.cbeta == betas) return FEPLL_OK;
  const size_t S = betas.size(), K = T.Kall;
  if (S > T.S_cap) {
    HIPX(hipStreamSynchronize(st));
    dfree(T.dbeta);
    dfree(T.tb.Ub);
    dfree(T.tb.Wt);
    dfree(T.tb.L32);
    dfree(T.tb.Pinv);
    T.S_cap = 0;
    HIPX(dalloc(&T.dbeta, S));
    HIPX(dalloc(&T.tb.Ub, S * K * kTileStride));
    HIPX(dalloc(&T.tb.Wt, S * K * kTileStride));
    HIPX(dalloc(&T.tb.L32, S * K));
    HIPX(dalloc(&T.tb.Pinv, S * K));
    T.S_cap = S;
  }
  HIPX(hipMemcpyAsync(T.dbeta, betas.data(), sizeof(double) * S, hipMemcpyHostToDevice, st));
  {
    StageTimer tm(g, 5, st);
    HIPX(launch_prep(T.U64, T.lam64, T.w64, T.Kall, T.dbeta, (int)S, kTabBF16, T.tb, st));
  }
  HIPX(hipStreamSynchronize(st));
  T.cbeta = betas;
  return FEPLL_OK;
}

// Per-beta tables for the beta slots `betas` (at least the tables in mask).
fepll_status ensure_consts(fepll_gmm* g, const std::vector<double>& betas, int mask,
                           hipStream_t st) {
  if (g->cbeta == betas && (g->cmask & mask) == mask) return FEPLL_OK;
  const size_t S = betas.size();
  const size_t K = g->K;
  if (S > g->S_cap) {
    HIPX(hipStreamSynchronize(st));
    dfree(g->dbeta);
    dfree(g->dlogsb);
    dfree(g->tb.Ut);
    dfree(g->tb.Ub);
    dfree(g->tb.Wh);
    dfree(g->tb.Wt);
    dfree(g->tb.L32);
    dfree(g->tb.Pinv);
    dfree(g->tb.L64);
    dfree(g->tb.invnu64);
    dfree(g->tb.Uf);
    dfree(g->tb.Ue);
    g->S_cap = 0;
    g->cbeta.clear();
    g->cmask = 0;
    HIPX(dalloc(&g->dbeta, S));
    HIPX(dalloc(&g->dlogsb, S));
    HIPX(dalloc(&g->tb.Wt, S * K * kTileStride));
    HIPX(dalloc(&g->tb.L32, S * K));
    HIPX(dalloc(&g->tb.Pinv, S * K));
    g->S_cap = S;
  }
  // the tables of a precision are allocated the first time it is used
  const size_t C = g->S_cap;
  if ((mask & kTabF32) && !g->tb.Ut) {
    HIPX(dalloc(&g->tb.Ut, C * K * kTileStride));
    HIPX(dalloc(&g->tb.L64, C * K));
    HIPX(dalloc(&g->tb.invnu64, C * K * kP));
  }
  if ((mask & kTabBF16) && !g->tb.Ub) HIPX(dalloc(&g->tb.Ub, C * K * kTileStride));
  // (the reduced-precision modes' binary16 estimate operand, with either)
  if ((mask & (kTabBF16 | kTabF8)) && !g->tb.Wh) HIPX(dalloc(&g->tb.Wh, C * K * kTileStride));
  if ((mask & kTabF8) && !g->tb.Uf) {
    HIPX(dalloc(&g->tb.Uf, C * K * kTileStride));
    HIPX(dalloc(&g->tb.Ue, C * K));
  }
  // same slots: add the missing tables; new slots: these tables only
  const int build = (g->cbeta == betas) ? (mask | g->cmask) : mask;
  HIPX(hipMemcpyAsync(g->dbeta, betas.data(), sizeof(double) * S, hipMemcpyHostToDevice, st));
  std::vector<float> logsb(S);
  for (size_t i = 0; i < S; ++i) logsb[i] = (float)(-0.5 * std::log(betas[i]));
  HIPX(hipMemcpyAsync(g->dlogsb, logsb.data(), sizeof(float) * S, hipMemcpyHostToDevice, st));
  {
    StageTimer tm(g, 5, st);
    HIPX(launch_prep(g->U64, g->lam64, g->w64, g->K, g->dbeta, (int)S, build, g->tb, st));
  }
  // the host betas must outlive their asynchronous upload
  HIPX(hipStreamSynchronize(st));
  g->cbeta = betas;
  g->cmask = build;
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
  if (o->jitter < 0 || o->jitter > 8) return fail(FEPLL_EINVAL, "options.jitter must be in 0..8");
  if (o->profile < 0 || o->profile >= (2 << kStages))
    return fail(FEPLL_EINVAL, "options.profile must be 0, 1 or a mask of stages (bits 1..9)");
  if (o->jitter && o->use_proposal)
    return fail(FEPLL_EUNSUPPORTED, "jittered subsampling does not run with the proposal");
  if (o->use_tree) {
    if (!g->tree.Kall) return fail(FEPLL_EINVAL, "no search tree is set (fepll_gmm_set_tree)");
    if (o->precision != FEPLL_BF16)
      return fail(FEPLL_EUNSUPPORTED, "the tree descent runs with FEPLL_BF16 costs");
    if (o->use_proposal || o->jitter)
      return fail(FEPLL_EUNSUPPORTED, "the tree descent runs alone (no proposal, no jitter)");
  }
  return FEPLL_OK;
}

template <class T>
fepll_status grow(T** p, size_t& cap, size_t n) {
  if (n <= cap && *p) return FEPLL_OK;
  dfree(*p);
  cap = 0;
  HIPX(dalloc(p, n));
  cap = n;
  return FEPLL_OK;
}

// Lay out n images of sizes H[i] x W[i] (T iterations, beta slots i*T + t,
// bvals[slot] = beta sigma^2) in the packed buffers, size the scratch and
// upload the plan (skipped when unchanged).
fepll_status make_plan(fepll_gmm* g, int n, const int* H, const int* W, int T,
                       const std::vector<float>& bvals, hipStream_t st) {
  const int K = g->K;
  const int ola_rows = g->tune.ola_rows;
  std::vector<ImgDesc> hd(n);
  std::vector<int32_t> est, sort, ola, resc;
  int64_t px = 0, np = 0, seg = 0;
  for (int i = 0; i < n; ++i) {
    const int Hp = H[i] - 7, Wp = W[i] - 7;
    const int64_t Np = (int64_t)Hp * Wp;
    ImgDesc& d = hd[i];
    d.H = H[i];
    d.W = W[i];
    d.px = px;
    d.np = np;
    d.seg = seg;
    d.sort0 = (int32_t)sort.size();
    d.est0 = (int32_t)est.size();
    d.ola0 = (int32_t)ola.size();
    d.slot0 = i * T;
    d.resc0 = (int32_t)resc.size();
    d.pad = 0;
    const int64_t nb = (Np + kSortBlock - 1) / kSortBlock;
    const int64_t nr = (Np + kRescPatches - 1) / kRescPatches;
    const int64_t ne = (int64_t)((Wp + kEstCols - 1) / kEstCols) * ((Hp + 3) / 4);
    const int64_t no =
        (int64_t)((W[i] + kOlaX - 1) / kOlaX) * ((H[i] + ola_rows - 1) / ola_rows);
    if ((int64_t)est.size() + ne > INT32_MAX / 2 || (int64_t)ola.size() + no > INT32_MAX / 2)
      return fail(FEPLL_EUNSUPPORTED, "batch too large");
    sort.insert(sort.end(), (size_t)nb, i);
    est.insert(est.end(), (size_t)ne, i);
    ola.insert(ola.end(), (size_t)no, i);
    resc.insert(resc.end(), (size_t)nr, i);
    px += ((int64_t)H[i] * W[i] + 63) / 64 * 64;  // 256-byte aligned images
    np += Np;
    seg += (int64_t)seg_size(Np, K);
  }
  if (np > INT32_MAX) return fail(FEPLL_EUNSUPPORTED, "batch too large");
  const bool same = g->plan_valid && g->hd.size() == hd.size() &&
                    std::memcmp(g->hd.data(), hd.data(), sizeof(ImgDesc) * n) == 0 &&
                    g->hbvals == bvals;
  fepll_status s;
  const size_t NP = (size_t)np, PX = (size_t)px;
  // buffers in use by earlier work are only freed once it is done
  if (NP > g->np_cap || PX > g->px_cap || (size_t)K * sort.size() > g->hist_cap ||
      (size_t)seg > g->seg_cap || !same)
    HIPX(hipStreamSynchronize(st));
  if (NP > g->np_cap) {
    dfree(g->labels);
    dfree(g->list);
    dfree(g->perm);
    dfree(g->Zhat);
    dfree(g->cand);
    dfree(g->fb_list);
    dfree(g->fbpart);
    dfree(g->jflags);
    dfree(g->jlist);
    g->np_cap = 0;
    HIPX(dalloc(&g->labels, NP));
    HIPX(dalloc(&g->list, 4 * NP));  // int4 entries
    HIPX(dalloc(&g->perm, NP));
    HIPX(dalloc(&g->Zhat, NP * kP));
    HIPX(dalloc(&g->cand, NP * 8));
    HIPX(dalloc(&g->fb_list, NP));
    HIPX(dalloc(&g->fbpart, 3 * kFallbackSplit * NP));
    HIPX(dalloc(&g->jflags, 3 * NP));
    HIPX(dalloc(&g->jlist, 3 * NP));
    g->np_cap = NP;
    // the subset flags start (and stay, between calls) all zero
    hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)((3 * NP + 255) / 256)), dim3(256), 0, st,
                       g->jflags, (int)(3 * NP));
    HIPX(hipGetLastError());
    g->jflags_dirty = false;
  }
  {
    // the search tree's pair scratch, sized for the largest image
    size_t npmax = 0;
    for (int i = 0; i < n; ++i) npmax = std::max(npmax, (size_t)(H[i] - 7) * (W[i] - 7));
    if ((s = grow(&g->psorted, g->pair_cap, 8 * npmax)) != FEPLL_OK) return s;
    const size_t nb2 = (npmax + kPairBlock - 1) / kPairBlock;
    // (the tree descent buckets over all its nodes)
    const int Kp = std::max(K, g->tree.Kall);
    if ((s = grow(&g->phist, g->phist_cap, (size_t)Kp * nb2)) != FEPLL_OK) return s;
    if ((s = grow(&g->pseg, g->pseg_cap, pair_seg_size(npmax, Kp))) != FEPLL_OK) return s;
    if (g->tree.Kall) {
      if ((s = grow(&g->zop, g->zop_cap, 64 * npmax)) != FEPLL_OK) return s;
      if ((s = grow(&g->znz, g->znz_cap, npmax)) != FEPLL_OK) return s;
    }
  }
  if (PX > g->px_cap) {
    dfree(g->ybuf);
    dfree(g->xa);
    dfree(g->xb);
    g->px_cap = 0;
    HIPX(dalloc(&g->ybuf, PX));
    HIPX(dalloc(&g->xa, PX));
    HIPX(dalloc(&g->xb, PX));
    g->px_cap = PX;
  }
  if (!g->count) HIPX(dalloc(&g->count, 64));
  if ((s = grow(&g->jcount, g->jcount_cap, 4 * (size_t)n)) != FEPLL_OK) return s;
  if ((s = grow(&g->fbcnt, g->fb_cap, 2 * (size_t)n + 1)) != FEPLL_OK) return s;
  g->fbitems = g->fbcnt + n;
  if ((s = grow(&g->hist, g->hist_cap, (size_t)K * sort.size())) != FEPLL_OK) return s;
  if ((s = grow(&g->seg, g->seg_cap, (size_t)seg)) != FEPLL_OK) return s;
  if (!same) {
    g->plan_valid = false;  // (until every plan buffer is uploaded)
    if ((s = grow(&g->d, g->n_cap, (size_t)n)) != FEPLL_OK) return s;
    if ((s = grow(&g->wbase, g->wb_cap, (size_t)n + 1)) != FEPLL_OK) return s;
    if ((s = grow(&g->est_img, g->est_cap, est.size())) != FEPLL_OK) return s;
    if ((s = grow(&g->sort_img, g->sort_cap, sort.size())) != FEPLL_OK) return s;
    if ((s = grow(&g->ola_img, g->ola_cap, ola.size())) != FEPLL_OK) return s;
    if ((s = grow(&g->resc_img, g->resc_cap, resc.size())) != FEPLL_OK) return s;
    if ((s = grow(&g->bvals, g->slot_cap, bvals.size())) != FEPLL_OK) return s;
    g->hd = std::move(hd);
    g->h_est = std::move(est);
    g->h_sort = std::move(sort);
    g->h_ola = std::move(ola);
    g->h_resc = std::move(resc);
    g->hbvals = bvals;
    HIPX(hipMemcpyAsync(g->d, g->hd.data(), sizeof(ImgDesc) * n, hipMemcpyHostToDevice, st));
    HIPX(hipMemcpyAsync(g->est_img, g->h_est.data(), sizeof(int32_t) * g->h_est.size(),
                        hipMemcpyHostToDevice, st));
    HIPX(hipMemcpyAsync(g->sort_img, g->h_sort.data(), sizeof(int32_t) * g->h_sort.size(),
                        hipMemcpyHostToDevice, st));
    HIPX(hipMemcpyAsync(g->ola_img, g->h_ola.data(), sizeof(int32_t) * g->h_ola.size(),
                        hipMemcpyHostToDevice, st));
    HIPX(hipMemcpyAsync(g->resc_img, g->h_resc.data(), sizeof(int32_t) * g->h_resc.size(),
                        hipMemcpyHostToDevice, st));
    HIPX(hipMemcpyAsync(g->bvals, g->hbvals.data(), sizeof(float) * g->hbvals.size(),
                        hipMemcpyHostToDevice, st));
    g->plan_valid = true;
  }
  Batch& b = g->batch;
  b.d = g->d;
  b.est_img = g->est_img;
  b.sort_img = g->sort_img;
  b.ola_img = g->ola_img;
  b.resc_img = g->resc_img;
  b.n = n;
  b.n_est = (int)g->h_est.size();
  b.n_sort = (int)g->h_sort.size();
  b.n_ola = (int)g->h_ola.size();
  b.n_resc = (int)g->h_resc.size();
  b.n_patches = np;
  b.max_np = 0;
  for (const ImgDesc& dd : g->hd)
    b.max_np = std::max<int64_t>(b.max_np, (int64_t)(dd.H - 7) * (dd.W - 7));
  b.ola_rows = ola_rows;
  return FEPLL_OK;
}

__global__ void mark_kernel(const int32_t* count, const int32_t* list, int32_t* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < *count) flags[list[i]] = 1;
}

// Gaussian selection of one image by the search tree (Sec. 3.2) with the
// tree tables of beta slot `slot`, every cost the bfloat16 selection cost of
// the all-K modes: the top levels of few nodes in one dense pass over the
// image (which also writes the patches' bfloat16 records), then each further
// level with the patches grouped by their current node and that node's
// children scored from the records, the best one kept (no fallback); the
// last level leaves a leaf, the label.
fepll_status select_tree(fepll_gmm* g, const float* x, int H, int W, int slot,
                         int32_t* labels, float* best, float* second, int32_t* flags,
                         hipStream_t st) {
  auto& T = g->tree;
  const int Np = (H - 7) * (W - 7);
  const size_t K = T.Kall;
  StageTimer tm(g, 0, st);
  if (flags) {
    hipLaunchKernelGGL(zero_i32_kernel, dim3((Np + 255) / 256), dim3(256), 0, st, flags, Np);
    HIPX(hipGetLastError());
  }
  const uint16_t* Ub = T.tb.Ub + (size_t)slot * K * kTileStride;
  const float* L = T.tb.L32 + (size_t)slot * K;
  const float* Pinv = T.tb.Pinv + (size_t)slot * K;
  const bool sparse = T.dense_levels + 1 < T.nlevels;  // levels left after the dense ones
  if (T.dense_levels > 0) {
    TreeDenseArgs a{};
    a.x = x;
    a.H = H;
    a.W = W;
    a.Ub = Ub;
    a.L = L;
    a.rk = T.tb.rk;
    a.Pinv = Pinv;
    a.node = T.dnode;
    a.par = T.dpar;
    a.lend = T.dlend;
    a.n = T.dense_n;
    a.nlev = T.dense_levels;
    a.root = T.root;
    a.labels = labels;
    a.best = sparse ? nullptr : best;
    a.second = sparse ? nullptr : second;
    a.zop = sparse ? reinterpret_cast<uint4*>(g->zop) : nullptr;
    a.znz = sparse ? g->znz : nullptr;
    HIPX(launch_tree_dense_bf16(a, st));
  } else {
    HIPX(launch_records_bf16(x, H, W, g->zop, g->znz, st));
    hipLaunchKernelGGL(fill_i32_kernel, dim3((Np + 255) / 256), dim3(256), 0, st, labels, Np,
                       T.root);
    HIPX(hipGetLastError());
  }
  for (int lev = T.dense_levels + 1; lev < T.nlevels; ++lev) {
    // (best / second: the leaf level's, among the last node's children)
    const bool last = lev == T.nlevels - 1;
    HIPX(launch_tree_level_bf16(labels, Np, g->zop, g->znz, Ub, L, T.tb.rk, Pinv, T.Kall,
                                T.children, g->cand, g->phist, g->pseg, g->psorted, labels,
                                last ? best : nullptr, last ? second : nullptr, st));
  }
  return FEPLL_OK;
}

// One float32 Gaussian selection of one image x with the tables of beta
// slot `slot`: the certified E-step, then the float64 re-selection of the
// uncertified patches.
fepll_status select_one(fepll_gmm* g, const float* x, int H, int W, int slot, double beta,
                        const fepll_options& o, int32_t* labels, float* best, float* second,
                        int32_t* flags, hipStream_t st) {
  const int Np = (H - 7) * (W - 7);
  const size_t K = g->K;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, g->count, 1);
  HIPX(hipGetLastError());
  {
    StageTimer tm(g, 0, st);
    HIPX(launch_estep_f32(x, H, W, g->tb.Ut + (size_t)slot * K * kTileStride,
                          g->tb.L32 + (size_t)slot * K, g->K, beta, labels, best, second, flags,
                          g->count, o.recheck ? g->list : nullptr, st));
  }
  if (o.recheck) {
    StageTimer tm(g, 1, st);
    HIPX(launch_recheck_f64(x, H, W, g->U64, g->tb.invnu64 + (size_t)slot * K * kP,
                            g->tb.L64 + (size_t)slot * K, g->K, g->count, g->list, labels, Np,
                            st));
  }
  return FEPLL_OK;
}

// Selection of every image of the planned batch at iteration t.  The
// all-K reduced-precision modes run as one persistent launch over the
// batch, the proposal path as one launch per stage over the batch; float32
// (with its recheck) runs image by image.  best / second / flags: packed
// like labels, or NULL.
// The jittered subsets' flag set, list and counts of iteration t (float32
// uses set 0 throughout), and the clearing of both flag sets.
int32_t* jflags_of(fepll_gmm* g, int t) { return g->jflags + (size_t)(t % 3) * g->np_cap; }
int32_t* jlist_of(fepll_gmm* g, int t) { return g->jlist + (size_t)(t % 3) * g->np_cap; }
int32_t* jcount_of(fepll_gmm* g, int t) { return g->jcount + (size_t)(t % 4) * g->batch.n; }
fepll_status clear_jflags(fepll_gmm* g, hipStream_t st) {
  const size_t m = 3 * g->np_cap;
  hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                     g->jflags, (int)m);
  HIPX(hipGetLastError());
  return FEPLL_OK;
}

// Jittered subsampling (Sec. 3.3) at iteration t: the chosen patches of every
// image (flags, then the list and the label K for the others), and their
// selection; float32 selects every patch first (its certification and
// recheck are per patch) and marks the others after.
fepll_status select_jitter(fepll_gmm* g, int t, const fepll_options& o, const float* x,
                           int32_t* labels, hipStream_t st) {
  const Batch& b = g->batch;
  const int n = (int)b.n_patches;
  const size_t K = g->K;
  fepll_status s;
  if (o.precision == FEPLL_FP32) {
    for (int i = 0; i < b.n; ++i) {
      const ImgDesc& d = g->hd[i];
      const int slot = d.slot0 + t;
      if ((s = select_one(g, x + d.px, d.H, d.W, slot, g->cbeta[slot], o, labels + d.np, nullptr,
                          nullptr, nullptr, st)) != FEPLL_OK)
        return s;
    }
  }
  // the reduced-precision paths append each iteration's list to its own
  // count, flag set and list (the previous iteration's are undone by the
  // same launch)
  const bool fp32 = o.precision == FEPLL_FP32;
  int32_t* cnt = fp32 ? g->jcount : jcount_of(g, t);
  // the one-pass e4m3 list selection adds its label counts to the list
  // sort's histogram (cleared by the drawing) when every image runs in one
  // pass
  bool sel_hist = o.precision == FEPLL_FP8 && g->jit_nbl > 0;
  for (int i = 0; i < b.n && sel_hist; ++i) {
    const ImgDesc& d = g->hd[i];
    const int64_t Np = (int64_t)(d.H - 7) * (d.W - 7);
    if (fp8_list_split(std::min<int64_t>(jitter_points_max(d.H, d.W, o.jitter), Np), g->K) > 1)
      sel_hist = false;
  }
  g->jit_hist = sel_hist;
  const size_t hist_n = K * (size_t)g->jit_nbl;
  int32_t* jflags = fp32 ? g->jflags : jflags_of(g, t);
  int32_t* jlist = fp32 ? g->jlist : jlist_of(g, t);
  {
    // the chosen patches of every image (stage 8: subset).  The position
    // flags are all zero between calls; after a new allocation or an
    // interrupted call they are cleared first.
    StageTimer tm(g, 8, st);
    if (o.precision == FEPLL_FP32) {
      // every patch was selected: flag the subset, then list it and give the
      // others the label K (the compaction clears the flags again)
      if (g->jflags_dirty && (s = clear_jflags(g, st)) != FEPLL_OK) return s;
      g->jflags_dirty = true;
      for (int i = 0; i < b.n; ++i) {
        const ImgDesc& d = g->hd[i];
        const int Np = (d.H - 7) * (d.W - 7);
        HIPX(launch_jitter_mark(d.H, d.W, o.jitter, o.seed, t, jflags + d.np, cnt + i, nullptr,
                                JitterPrev{}, st));
        HIPX(launch_jitter_compact(Np, g->K, jflags + d.np, labels + d.np, cnt + i,
                                   jlist + d.np, st));
      }
      g->jflags_dirty = false;
    } else if (!(g->jit_fused && t > 0)) {
      // every label not on the previous list is K here (run_hqs): list the
      // subset as it is drawn, and undo the previous list (t > 0).  (Drawn
      // by the previous reprojection when run_hqs fuses them.)
      for (int i = 0; i < b.n; ++i) {
        const ImgDesc& d = g->hd[i];
        JitterPrev prev;
        if (t > 0) {
          prev.list = jlist_of(g, t - 1) + d.np;
          prev.count = jcount_of(g, t - 1) + i;
          prev.flags = jflags_of(g, t - 1) + d.np;
          prev.labels = labels + d.np;
          prev.K = g->K;
          prev.zero = jcount_of(g, t + 1) + i;
        }
        if (sel_hist) {
          prev.clear = g->hist + hist_n * i;
          prev.nclear = (int)hist_n;
        }
        HIPX(launch_jitter_mark(d.H, d.W, o.jitter, o.seed, t, jflags + d.np, cnt + i,
                                jlist + d.np, prev, st));
      }
    }
  }
  if (o.precision == FEPLL_FP32) return FEPLL_OK;
  for (int i = 0; i < b.n; ++i) {
    const ImgDesc& d = g->hd[i];
    const int Np = (d.H - 7) * (d.W - 7);
    const int slot = d.slot0 + t;
    if (o.precision == FEPLL_FP8) {
      const int64_t lmax = std::min<int64_t>(jitter_points_max(d.H, d.W, o.jitter), Np);
      // the split needs its scratch (sized by ensure_jitter); without it, one pass
      float4* part =
          (!sel_hist && g->jpart && (size_t)(fp8_list_split(lmax, g->K) * lmax) <= g->jpart_cap)
              ? g->jpart
              : nullptr;
      int ns = 1;
      {
        StageTimer tm(g, 0, st, true);  // the selection kernel alone
        HIPX(launch_estep_fp8_list(g->d + i, lmax, t, x, g->tb.Uf, g->tb.Ue, g->tb.L32,
                                   g->tb.rk, g->tb.Pinv, g->K, cnt + i, jlist + d.np,
                                   labels, nullptr, nullptr, part, &ns,
                                   sel_hist ? g->hist + hist_n * i : nullptr, g->jit_nbl, st));
      }
      StageTimer tm(g, 8, st);  // the merge of the component ranges
      HIPX(launch_fp8_merge(g->d + i, lmax, cnt + i, jlist + d.np, part, ns, labels, nullptr,
                            nullptr, st));
    } else {
      StageTimer tm(g, 0, st);
      BF16Args a{};
      a.x = x + d.px;
      a.H = d.H;
      a.W = d.W;
      a.Ub = g->tb.Ub + (size_t)slot * K * kTileStride;
      a.L = g->tb.L32 + (size_t)slot * K;
      a.K = g->K;
      a.labels = labels + d.np;
      a.list_count = cnt + i;
      a.list = jlist + d.np;
      a.rk = g->tb.rk;
      a.Pinv = g->tb.Pinv + (size_t)slot * K;
      HIPX(launch_estep_bf16_mode(kModeListFull, a, st));
    }
  }
  return FEPLL_OK;
}

// Scratch of the jittered selection for the planned batch (allocated before
// any capture).
fepll_status ensure_jitter(fepll_gmm* g, const fepll_options& o) {
  if (!o.jitter || o.precision != FEPLL_FP8) return FEPLL_OK;
  size_t need = 0;
  for (const ImgDesc& d : g->hd) {
    const int64_t Np = (int64_t)(d.H - 7) * (d.W - 7);
    const int64_t lmax = std::min<int64_t>(jitter_points_max(d.H, d.W, o.jitter), Np);
    need = std::max(need, (size_t)(fp8_list_split(lmax, g->K) * lmax));
  }
  if (need > g->jpart_cap || !g->jpart) {
    if (g->used) HIPX(hipStreamSynchronize(g->last_stream));
    dfree(g->jpart);
    g->jpart_cap = 0;
    HIPX(dalloc(&g->jpart, need));
    g->jpart_cap = need;
  }
  return FEPLL_OK;
}

// The proposal path over the planned batch at iteration t: the network's
// top-m candidates of every patch (one launch over the batch's selection
// tiles), their exact rescoring with the fallback decisions (one launch over
// the rescoring tiles), then the full-K search of every image's fallback
// list (one launch over the items of all lists).  flags (or NULL): 1 on the
// patches that fell back, 0 elsewhere.
fepll_status select_proposal(fepll_gmm* g, int t, const fepll_options& o, const float* x,
                             int32_t* labels, float* best, float* second, int32_t* flags,
                             hipStream_t st) {
  const Batch& b = g->batch;
  {
    StageTimer tm(g, 6, st);
    ProposeArgs p{};
    p.x = x;
    p.d = b.d;
    p.est_img = b.est_img;
    p.n_est = b.n_est;
    p.logsb_slot = g->dlogsb;
    p.t = t;
    p.Wb = g->pWb;
    p.bias = g->pbias;
    p.K = g->K;
    p.m = o.top_m;
    p.cand = g->cand;
    p.zero = g->fbcnt;  // the fallback counts the rescoring appends to
    p.n_zero = b.n;
    HIPX(launch_propose(p, st));
  }
  {
    StageTimer tm(g, 0, st);
    RescoreArgs r{};
    r.d = b.d;
    r.tile_img = b.resc_img;
    r.x = x;
    r.cand = g->cand;
    r.m = o.top_m;
    r.K = g->K;
    r.t = t;
    r.Ub = g->tb.Ub;
    r.L = g->tb.L32;
    r.rk = g->tb.rk;
    r.Pinv = g->tb.Pinv;
    r.margin = (float)o.margin_nats;
    r.labels = labels;
    r.best = best;
    r.second = second;
    r.fb_count = g->fbcnt;
    r.fb_list = g->fb_list;
    HIPX(launch_rescore_batch(r, b.n_resc, st));
    HIPX(launch_fallback_items(g->fbcnt, b.n, g->fbitems, st));
  }
  {
    StageTimer tm(g, 7, st);
    BF16Args a{};
    a.x = x;
    a.Ub = g->tb.Ub;
    a.L = g->tb.L32;
    a.K = g->K;
    a.labels = labels;
    a.best = best;
    a.second = second;
    a.list_count = g->fbcnt;
    a.list = g->fb_list;
    a.d = b.d;
    a.t = t;
    a.rk = g->tb.rk;
    a.Pinv = g->tb.Pinv;
    a.item_pre = g->fbitems;
    a.n_img = b.n;
    a.ksplit = kFallbackSplit;
    a.part_out = g->fbpart;
    a.part_stride = g->np_cap;
    // a fixed grid walking the items (at most every patch falls back)
    int64_t items = 0;
    for (const ImgDesc& d : g->hd) items += ((int64_t)(d.H - 7) * (d.W - 7) + 511) / 512;
    a.blocks = (int)std::max<int64_t>(1, std::min<int64_t>(items * kFallbackSplit, 1024));
    HIPX(launch_estep_bf16_mode(kModeListBatch, a, st));
    a.blocks = (int)std::max<int64_t>(1, std::min<int64_t>(items, 1024));
    HIPX(launch_fallback_merge(a, st));
  }
  if (flags) {
    const int n = (int)b.n_patches;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, st, flags, n);
    HIPX(hipGetLastError());
    for (int i = 0; i < b.n; ++i) {
      const ImgDesc& d = g->hd[i];
      const int Np = (d.H - 7) * (d.W - 7);
      hipLaunchKernelGGL(mark_kernel, dim3((Np + 255) / 256), dim3(256), 0, st, g->fbcnt + i,
                         g->fb_list + d.np, flags + d.np);
      HIPX(hipGetLastError());
    }
  }
  return FEPLL_OK;
}

fepll_status select_batch(fepll_gmm* g, int t, const fepll_options& o, const float* x,
                          int32_t* labels, float* best, float* second, int32_t* flags,
                          hipStream_t st) {
  const Batch& b = g->batch;
  const int blocks = g->tune.est_blocks;
  if (o.jitter) return select_jitter(g, t, o, x, labels, st);
  if (o.use_tree) {
    fepll_status s;
    for (int i = 0; i < b.n; ++i) {
      const ImgDesc& d = g->hd[i];
      if ((s = select_tree(g, x + d.px, d.H, d.W, d.slot0 + t, labels + d.np,
                           best ? best + d.np : nullptr, second ? second + d.np : nullptr,
                           flags ? flags + d.np : nullptr, st)) != FEPLL_OK)
        return s;
    }
    return FEPLL_OK;
  }
  if (o.precision == FEPLL_BF16 && o.use_proposal)
    return select_proposal(g, t, o, x, labels, best, second, flags, st);
  if (o.precision == FEPLL_FP8 || o.precision == FEPLL_BF16) {
    if (flags) {
      const int n = (int)b.n_patches;
      hipLaunchKernelGGL(zero_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, st, flags, n);
      HIPX(hipGetLastError());
    }
    StageTimer tm(g, 0, st);
    if (o.precision == FEPLL_FP8)
      HIPX(launch_estep_fp8_batch(b, x, g->tb.Uf, g->tb.Ue, g->tb.L32, g->tb.rk, g->tb.Pinv,
                                  g->K, t, labels, best, second, blocks, st));
    else
      HIPX(launch_estep_bf16_batch(b, x, g->tb.Ub, g->tb.L32, g->tb.rk, g->tb.Pinv, g->K, t,
                                   labels, best, second, blocks, st));
    return FEPLL_OK;
  }
  fepll_status s;
  for (int i = 0; i < b.n; ++i) {
    const ImgDesc& d = g->hd[i];
    const int slot = d.slot0 + t;
    if ((s = select_one(g, x + d.px, d.H, d.W, slot, g->cbeta[slot], o, labels + d.np,
                        best ? best + d.np : nullptr, second ? second + d.np : nullptr,
                        flags ? flags + d.np : nullptr, st)) != FEPLL_OK)
      return s;
  }
  return FEPLL_OK;
}

// T iterations of Alg. 1 over the planned batch, from g->xa (y in g->ybuf);
// *result receives the buffer holding the restored images.  labels_out
// (single image only): per-iteration copies of the labels.
// Image estimation of a periodic convolution A on the single image of the
// plan: x (float, H x W) holds x~ on entry and the estimate on return.
fepll_status deblur_update(fepll_gmm* g, float* x, double b, hipStream_t st) {
  auto& D = g->db;
  const int n = D.H * D.W, m = D.H * (D.W / 2 + 1);
  HIPX(launch_f2d(x, D.r, n, st));
  if (hipfftExecD2Z(D.fwd, D.r, reinterpret_cast<hipfftDoubleComplex*>(D.X)) != HIPFFT_SUCCESS)
    return fail(FEPLL_EDEVICE, "hipfftExecD2Z failed");
  HIPX(launch_spec_update(D.AtY, D.a2, D.X, m, b, st));
  if (hipfftExecZ2D(D.inv, reinterpret_cast<hipfftDoubleComplex*>(D.X), D.r) != HIPFFT_SUCCESS)
    return fail(FEPLL_EDEVICE, "hipfftExecZ2D failed");
  HIPX(launch_d2f_scale(D.r, x, n, 1.0 / n, st));
  return FEPLL_OK;
}

fepll_status run_hqs(fepll_gmm* g, int T, const fepll_options& o, int32_t* labels_out,
                     hipMemcpyKind lkind, float** result, hipStream_t st,
                     const std::vector<double>* deblur_b = nullptr) {
  const Batch& b = g->batch;
  float* xc = g->xa;
  float* xn = g->xb;
  fepll_status s;
  // bound of any image's Wiener tile count (a jittered subset: its points)
  int64_t max_tiles_image = 0;
  for (const ImgDesc& d : g->hd) {
    int64_t n = (int64_t)(d.H - 7) * (d.W - 7);
    if (o.jitter) n = std::min<int64_t>(n, jitter_points_max(d.H, d.W, o.jitter));
    max_tiles_image = std::max<int64_t>(max_tiles_image, n / kWienerTile + g->K);
  }
  // jittered subsets in a reduced precision: each iteration lists its
  // patches as it draws them, and the patches off the list keep the label K
  // (set here for all, restored for the listed ones by the next iteration's
  // drawing, and after the last iteration)
  const bool jit_list = o.jitter && o.precision != FEPLL_FP32;
  // ... and sorts by label over those lists when their counts fit the
  // histogram (chunks of kListChunk list entries per image)
  int list_chunks = 0;
  for (const ImgDesc& d : g->hd) {
    const int64_t lmax = std::min<int64_t>(jitter_points_max(d.H, d.W, std::max(o.jitter, 1)),
                                           (int64_t)(d.H - 7) * (d.W - 7));
    list_chunks = std::max<int>(list_chunks, (int)((lmax + kListChunk - 1) / kListChunk));
  }
  const bool list_sort = jit_list && max_tiles_image <= kSmallTiles &&
                         (size_t)list_chunks * b.n <= g->h_sort.size();
  g->jit_nbl = list_sort ? list_chunks : 0;
  g->jit_hist = false;
  // one image, its list sorted, no labels returned: the reprojection of
  // iteration t also draws the subset of t + 1 (it then takes its patches
  // from the flags, and the drawing gives the patches of the list of t - 1
  // flag 0 and label K again)
  g->jit_fused = list_sort && b.n == 1 && labels_out == nullptr;
  if (jit_list) {
    const int n = (int)b.n_patches;
    if (g->jflags_dirty && (s = clear_jflags(g, st)) != FEPLL_OK) return s;
    g->jflags_dirty = true;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, st, g->labels, n,
                       g->K);
    HIPX(hipGetLastError());
    hipLaunchKernelGGL(zero_i32_kernel, dim3((4 * b.n + 255) / 256), dim3(256), 0, st, g->jcount,
                       4 * b.n);
    HIPX(hipGetLastError());
  }
  for (int t = 0; t < T; ++t) {
    TraceRange tr("fepll HQS iteration", t);
    if ((s = select_batch(g, t, o, xc, g->labels, nullptr, nullptr, nullptr, st)) != FEPLL_OK)
      return s;
    if (labels_out)
      HIPX(hipMemcpyAsync(labels_out + (size_t)t * b.n_patches, g->labels,
                          sizeof(int32_t) * b.n_patches, lkind, st));
    {
      StageTimer tm(g, 2, st, labels_out == nullptr);
      if (list_sort)
        HIPX(launch_bucket_list(b, g->labels, jlist_of(g, t), jcount_of(g, t), g->K,
                                list_chunks, g->hist, g->seg, g->perm, g->wbase, g->jit_hist,
                                st));
      else
        HIPX(launch_bucket_batch(b, g->labels, g->K, g->hist, g->seg, g->perm, g->wbase,
                                 max_tiles_image, st));
    }
    {
      StageTimer tm(g, 3, st, true);
      HIPX(launch_wiener_batch(b, xc, g->tb.Wt, o.precision == FEPLL_FP32 ? nullptr : g->tb.Wh,
                               g->K, t, g->seg, g->perm, g->wbase, g->Zhat,
                               g->tune.wiener_blocks, st));
    }
    {
      StageTimer tm(g, 4, st, true);
      if (g->jit_fused && t + 1 < T) {
        // the drawing of t + 1: undoes the list of t - 1 (flags and labels;
        // this reprojection reads neither), zeroes the count t + 2 appends
        // to, clears the selection's histogram
        const ImgDesc& d = g->hd[0];
        JitterPrev prev;
        if (t >= 1) {
          prev.list = jlist_of(g, t - 1) + d.np;
          prev.count = jcount_of(g, t - 1);
          prev.flags = jflags_of(g, t - 1) + d.np;
          prev.labels = g->labels + d.np;
          prev.K = g->K;
        }
        prev.zero = jcount_of(g, t + 2);
        if (g->jit_hist) {
          prev.clear = g->hist;
          prev.nclear = g->K * g->jit_nbl;
        }
        int blocks = 0;
        const JitterDraw dr =
            make_jitter_draw(d.H, d.W, o.jitter, o.seed, t + 1, jflags_of(g, t + 1) + d.np,
                             jcount_of(g, t + 1), jlist_of(g, t + 1) + d.np, prev, &blocks);
        HIPX(launch_ola_batch(b, g->Zhat, g->ybuf, g->bvals, t, xn, jflags_of(g, t), 0,
                              deblur_b ? 1 : 0, &dr, st));
      } else if (g->jit_fused) {
        HIPX(launch_ola_batch(b, g->Zhat, g->ybuf, g->bvals, t, xn, jflags_of(g, t), 0,
                              deblur_b ? 1 : 0, nullptr, st));
      } else {
        HIPX(launch_ola_batch(b, g->Zhat, g->ybuf, g->bvals, t, xn,
                              o.jitter ? g->labels : nullptr, g->K, deblur_b ? 1 : 0, nullptr,
                              st));
      }
      if (deblur_b) {
        fepll_status s2 = deblur_update(g, xn, (*deblur_b)[t], st);
        if (s2 != FEPLL_OK) return s2;
      }
    }
    std::swap(xc, xn);
  }
  if (jit_list && T > 0) {
    // the last list's patches (the last two when fused) back to flag 0 and
    // label K
    StageTimer tm(g, 8, st);
    for (int u = (g->jit_fused && T >= 2) ? T - 2 : T - 1; u < T; ++u)
      for (int i = 0; i < b.n; ++i) {
        const ImgDesc& d = g->hd[i];
        const int64_t lmax = std::min<int64_t>(jitter_points_max(d.H, d.W, o.jitter),
                                               (int64_t)(d.H - 7) * (d.W - 7));
        HIPX(launch_jitter_reset(jlist_of(g, u) + d.np, lmax, jcount_of(g, u) + i, nullptr,
                                 jflags_of(g, u) + d.np, g->labels + d.np, g->K, st));
      }
  }
  if (jit_list) g->jflags_dirty = false;
  *result = xc;
  return FEPLL_OK;
}

template <class V>
void put(std::vector<uint8_t>& k, const V& v) {
  const uint8_t* p = reinterpret_cast<const uint8_t*>(&v);
  k.insert(k.end(), p, p + sizeof(V));
}

// run_hqs through a captured graph: the launch sequence depends only on
// the plan, the beta slots, the options, the launch shapes and the
// buffers, so it is captured once and replayed while those stay the same.
fepll_status run_hqs_graph(fepll_gmm* g, int T, const fepll_options& o, float** result,
                           hipStream_t st) {
  std::vector<uint8_t> key;
  put(key, T);
  put(key, g->K);
  put(key, o.precision);
  put(key, o.recheck);
  put(key, o.use_proposal);
  put(key, o.top_m);
  put(key, o.margin_nats);
  put(key, o.jitter);
  put(key, o.seed);
  put(key, o.use_tree);
  put(key, g->tree.Kall);
  put(key, g->tune);
  put(key, g->rho);
  for (const ImgDesc& d : g->hd) put(key, d);
  for (double v : g->cbeta) put(key, v);
  for (float v : g->hbvals) put(key, v);
  const void* ptrs[] = {g->tb.Ut, g->tb.Ub, g->tb.Wt, g->tb.Wh, g->tb.L32, g->tb.L64, g->tb.invnu64,
                        g->tb.Uf, g->tb.Ue,   g->d,     g->est_img, g->sort_img, g->ola_img,
                        g->wbase, g->bvals,   g->labels, g->list,  g->count,  g->hist,
                        g->seg,   g->perm,    g->Zhat,  g->ybuf,   g->xa,     g->xb,
                        g->pWb,   g->pbias,   g->cand,  g->fb_list, g->fbpart,
                        g->fbcnt, g->resc_img, g->dlogsb, g->dbeta,
                        g->psorted, g->phist, g->pseg,
                        g->tb.rk,   g->tb.Pinv, g->zop,  g->znz,
                        g->jflags,  g->jlist,   g->jcount, g->jpart,
                        g->tree.tb.Ub, g->tree.tb.L32, g->tree.tb.Pinv, g->tree.rk,
                        g->tree.children, g->tree.dnode, g->tree.dpar, g->tree.dlend};
  for (const void* p : ptrs) put(key, p);
  put(key, g->tree_gen);  // a new tree may reuse the old one's addresses
  if (g->gexec && key == g->gkey) {
    // the graph starts from clear subset flags: after an interrupted eager
    // call they are cleared here first
    if (o.jitter && g->jflags_dirty) {
      fepll_status s = clear_jflags(g, st);
      if (s != FEPLL_OK) return s;
      g->jflags_dirty = false;
    }
    *result = (T % 2) ? g->xb : g->xa;
    HIPX(hipGraphLaunch(g->gexec, st));
    return FEPLL_OK;
  }
  if (g->gexec) {
    HIPX(hipStreamSynchronize(st));
    (void)hipGraphExecDestroy(g->gexec);
    g->gexec = nullptr;
    g->gkey.clear();
  }
  if (!g->cap_stream) HIPX(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
  HIPX(hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal));
  float* res = nullptr;
  const fepll_status s = run_hqs(g, T, o, nullptr, hipMemcpyDefault, &res, g->cap_stream);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(g->cap_stream, &graph);
  if (s != FEPLL_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  HIPX(e);
  const hipError_t ei = hipGraphInstantiate(&g->gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    g->gexec = nullptr;
    HIPX(ei);
  }
  g->gkey = std::move(key);
  *result = res;
  HIPX(hipGraphLaunch(g->gexec, st));
  return FEPLL_OK;
}

// Plans and spectrum buffers of the deblurring for an H x W image.
fepll_status ensure_deblur(fepll_gmm* g, int H, int W, hipStream_t st) {
  auto& D = g->db;
  const size_t n = (size_t)H * W, m = (size_t)H * (W / 2 + 1);
  if (g->used) HIPX(hipStreamSynchronize(g->last_stream));
  if (!D.plans || D.H != H || D.W != W) {
    if (D.plans) {
      (void)hipfftDestroy(D.fwd);
      (void)hipfftDestroy(D.inv);
      D.plans = false;
    }
    if (hipfftPlan2d(&D.fwd, H, W, HIPFFT_D2Z) != HIPFFT_SUCCESS)
      return fail(FEPLL_EDEVICE, "hipfftPlan2d (D2Z) failed");
    if (hipfftPlan2d(&D.inv, H, W, HIPFFT_Z2D) != HIPFFT_SUCCESS) {
      (void)hipfftDestroy(D.fwd);
      return fail(FEPLL_EDEVICE, "hipfftPlan2d (Z2D) failed");
    }
    D.plans = true;
    D.H = H;
    D.W = W;
  }
  if (hipfftSetStream(D.fwd, st) != HIPFFT_SUCCESS || hipfftSetStream(D.inv, st) != HIPFFT_SUCCESS)
    return fail(FEPLL_EDEVICE, "hipfftSetStream failed");
  if (n > D.n_cap || !D.r) {
    dfree(D.r);
    D.n_cap = 0;
    HIPX(dalloc(&D.r, n));
    D.n_cap = n;
  }
  if (m > D.m_cap || !D.Hh) {
    dfree(D.Hh);
    dfree(D.AtY);
    dfree(D.a2);
    dfree(D.X);
    D.m_cap = 0;
    HIPX(dalloc(&D.Hh, m));
    HIPX(dalloc(&D.AtY, m));
    HIPX(dalloc(&D.a2, m));
    HIPX(dalloc(&D.X, m));
    D.m_cap = m;
  }
  return FEPLL_OK;
}

// The kernel's spectrum (into D.Hh) and lambda = min(|A^t A|_F^2 /
// (N |A|_2^2), 250 sigma^2) over the full spectrum (Hermitian half:
// the columns other than 0 and W/2 stand for two), on the host in float64.
fepll_status deblur_spectrum(fepll_gmm* g, const fepll_operator* op, double sigma,
                             double* lambda, hipStream_t st) {
  auto& D = g->db;
  const int H = D.H, W = D.W, Wh = W / 2 + 1;
  std::vector<double> e((size_t)H * W, 0.0);
  for (int u = 0; u < op->kh; ++u)
    for (int v = 0; v < op->kw; ++v) {
      const int r = ((u - op->kh / 2) % H + H) % H, c = ((v - op->kw / 2) % W + W) % W;
      e[(size_t)r * W + c] += (double)op->kernel[u * op->kw + v];
    }
  HIPX(hipMemcpyAsync(D.r, e.data(), sizeof(double) * e.size(), hipMemcpyHostToDevice, st));
  if (hipfftExecD2Z(D.fwd, D.r, reinterpret_cast<hipfftDoubleComplex*>(D.Hh)) != HIPFFT_SUCCESS)
    return fail(FEPLL_EDEVICE, "hipfftExecD2Z failed");
  std::vector<double2> h((size_t)H * Wh);
  HIPX(hipMemcpyAsync(h.data(), D.Hh, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, st));
  HIPX(hipStreamSynchronize(st));
  double s4 = 0.0, mx = 0.0;
  for (int k = 0; k < H; ++k)
    for (int l = 0; l < Wh; ++l) {
      const double2 z = h[(size_t)k * Wh + l];
      const double a = z.x * z.x + z.y * z.y;
      const double wgt = (l == 0 || 2 * l == W) ? 1.0 : 2.0;
      s4 += wgt * a * a;
      mx = std::max(mx, a);
    }
  if (!(mx > 0.0)) return fail(FEPLL_EINVAL, "H: the blur kernel's spectrum is zero");
  *lambda = std::min(s4 / ((double)H * W) / mx, 250.0 * sigma * sigma);
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

const char* fepll_version(void) { return "fepll-gfx950 0.2"; }

fepll_status fepll_set_memory_limit(size_t limit_bytes) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_mem_limit = limit_bytes;
  return FEPLL_OK;
}

size_t fepll_memory_in_use(void) {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  return g_mem_in_use;
}

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
  default_tuning(&g->tune);
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
  g->lam_h.assign(lambda, lambda + (size_t)K * d);
  g->U_h.assign(U, U + (size_t)K * d * d);
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
    if (m.own_a) g->pool.push_back(m.a);
    g->pool.push_back(m.b);
  }
  g->marks.clear();
  g->chain_ev = nullptr;
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
    if (m.own_a) (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  for (auto e : g->pool) (void)hipEventDestroy(e);
  if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  dfree(g->U64);
  dfree(g->lam64);
  dfree(g->w64);
  dfree(g->rk);
  dfree(g->tb.Pinv);
  dfree(g->dbeta);
  dfree(g->tb.Ut);
  dfree(g->tb.Ub);
  dfree(g->tb.Wh);
  dfree(g->tb.Wt);
  dfree(g->tb.L32);
  dfree(g->tb.L64);
  dfree(g->tb.invnu64);
  dfree(g->tb.Uf);
  dfree(g->tb.Ue);
  dfree(g->d);
  dfree(g->est_img);
  dfree(g->sort_img);
  dfree(g->ola_img);
  dfree(g->wbase);
  dfree(g->bvals);
  dfree(g->labels);
  dfree(g->list);
  dfree(g->count);
  dfree(g->hist);
  dfree(g->seg);
  dfree(g->perm);
  dfree(g->Zhat);
  dfree(g->cand);
  dfree(g->fb_list);
  dfree(g->fbpart);
  dfree(g->psorted);
  dfree(g->fbcnt);
  dfree(g->resc_img);
  dfree(g->dlogsb);
  dfree(g->zop);
  dfree(g->znz);
  dfree(g->jflags);
  dfree(g->jlist);
  dfree(g->jcount);
  dfree(g->jpart);
  if (g->db.plans) {
    (void)hipfftDestroy(g->db.fwd);
    (void)hipfftDestroy(g->db.inv);
  }
  dfree(g->tree.U64);
  dfree(g->tree.lam64);
  dfree(g->tree.w64);
  dfree(g->tree.rk);
  dfree(g->tree.children);
  dfree(g->tree.dnode);
  dfree(g->tree.dpar);
  dfree(g->tree.dlend);
  dfree(g->tree.dbeta);
  dfree(g->tree.tb.Ub);
  dfree(g->tree.tb.Wt);
  dfree(g->tree.tb.L32);
  dfree(g->tree.tb.Pinv);
  dfree(g->db.r);
  dfree(g->db.Hh);
  dfree(g->db.AtY);
  dfree(g->db.a2);
  dfree(g->db.X);
  dfree(g->phist);
  dfree(g->pseg);
  dfree(g->pWb);
  dfree(g->pbias);
  dfree(g->ybuf);
  dfree(g->xa);
  dfree(g->xb);
  delete g;
}

fepll_status fepll_restore(fepll_gmm* g, const fepll_image* y, const fepll_operator* Hop,
                           double sigma, const double* beta_schedule, int32_t T,
                           fepll_image* out, const fepll_options* opt, int32_t* labels_out) {
  g_err.clear();
  TraceRange tr("fepll_restore");
  if (!g) return fail(FEPLL_EINVAL, "gmm handle is NULL");
  fepll_status s;
  if ((s = check_image(y, "y")) != FEPLL_OK) return s;
  if ((s = check_image(out, "out")) != FEPLL_OK) return s;
  const bool conv = Hop && Hop->kind == FEPLL_OP_CONVOLUTION;
  if (Hop && Hop->kind != FEPLL_OP_IDENTITY && !conv)
    return fail(FEPLL_EINVAL, "H->kind must be FEPLL_OP_IDENTITY or FEPLL_OP_CONVOLUTION");
  if (conv) {
    if (!Hop->kernel) return fail(FEPLL_EINVAL, "H->kernel is NULL");
    if (Hop->kh < 1 || Hop->kw < 1 || Hop->kh % 2 == 0 || Hop->kw % 2 == 0 ||
        Hop->kh > y->height || Hop->kw > y->width)
      return fail(FEPLL_EINVAL, "H: kernel sizes must be odd and at most the image's");
    for (int i = 0; i < Hop->kh * Hop->kw; ++i)
      if (!std::isfinite(Hop->kernel[i])) return fail(FEPLL_EINVAL, "H: non-finite kernel entry");
  }
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(FEPLL_EINVAL, "sigma must be > 0");
  if (out->height != y->height || out->width != y->width)
    return fail(FEPLL_EINVAL, "out must have the shape of y");
  fepll_options o;
  fepll_options_default(&o);
  if (opt) o = *opt;
  if ((s = check_opt(g, &o)) != FEPLL_OK) return s;
  const int H = y->height, W = y->width;
  hipStream_t st = (hipStream_t)o.stream;
  // deblurring: the kernel's spectrum and lambda (Sec. 5) before the schedule
  double lambda = 1.0;
  if (conv) {
    if ((s = use_stream(g, st)) != FEPLL_OK) return s;
    if ((s = ensure_deblur(g, H, W, st)) != FEPLL_OK) return s;
    if ((s = deblur_spectrum(g, Hop, sigma, &lambda, st)) != FEPLL_OK) return s;
  }
  std::vector<double> betas;
  if (!beta_schedule) {
    if (T != 0 && T != kDefaultT) return fail(FEPLL_EINVAL, "default schedule has T = 5");
    for (int t = 0; t < kDefaultT; ++t) betas.push_back(lambda * kDefaultB[t] / (sigma * sigma));
  } else {
    if (T < 1 || T > kMaxT) return fail(FEPLL_EINVAL, "T must be in 1..16");
    for (int t = 0; t < T; ++t) {
      if (!(beta_schedule[t] > 0.0) || !std::isfinite(beta_schedule[t]))
        return fail(FEPLL_EINVAL, "beta values must be finite and > 0");
      betas.push_back(beta_schedule[t]);
    }
  }
  T = (int32_t)betas.size();
  if (o.init) {
    if ((s = check_image(o.init, "options.init")) != FEPLL_OK) return s;
    if (o.init->height != y->height || o.init->width != y->width)
      return fail(FEPLL_EINVAL, "options.init must have the shape of y");
    if ((s = host_finite(o.init, "options.init")) != FEPLL_OK) return s;
  }
  if ((s = host_finite(y, "y")) != FEPLL_OK) return s;

  if ((s = use_stream(g, st)) != FEPLL_OK) return s;
  g->profiling = profile_mask(o.profile);
  std::vector<float> bvals;
  for (double b : betas) bvals.push_back((float)(b * sigma * sigma));
  if ((s = make_plan(g, 1, &H, &W, T, bvals, st)) != FEPLL_OK) return s;
  if ((s = ensure_consts(g, betas, table_mask(o), st)) != FEPLL_OK) return s;
  if ((s = ensure_jitter(g, o)) != FEPLL_OK) return s;
  if (o.use_tree && (s = ensure_tree_consts(g, betas, st)) != FEPLL_OK) return s;

  HIPX(copy_in(g->ybuf, y, st));
  if (o.init) HIPX(copy_in(g->xa, o.init, st));
  else if (!conv)
    HIPX(hipMemcpyAsync(g->xa, g->ybuf, sizeof(float) * H * W, hipMemcpyDeviceToDevice, st));

  float* res = nullptr;
  if (conv) {
    // A^t y once; the Sec. 5 start unless options.init is given; then the
    // iterations with the Fourier image estimation (eager: no capture)
    auto& D = g->db;
    const int n = H * W, m = H * (W / 2 + 1);
    HIPX(launch_f2d(g->ybuf, D.r, n, st));
    if (hipfftExecD2Z(D.fwd, D.r, reinterpret_cast<hipfftDoubleComplex*>(D.X)) != HIPFFT_SUCCESS)
      return fail(FEPLL_EDEVICE, "hipfftExecD2Z failed");
    HIPX(launch_spec_prep(D.Hh, D.X, D.AtY, D.a2, m, st));
    if (!o.init) {
      HIPX(launch_spec_init(D.AtY, D.a2, D.X, H, W, 0.2 * sigma * sigma / lambda, st));
      if (hipfftExecZ2D(D.inv, reinterpret_cast<hipfftDoubleComplex*>(D.X), D.r) !=
          HIPFFT_SUCCESS)
        return fail(FEPLL_EDEVICE, "hipfftExecZ2D failed");
      HIPX(launch_d2f_scale(D.r, g->xa, n, 1.0 / n, st));
    }
    std::vector<double> bb;
    for (double bt : betas) bb.push_back(bt * sigma * sigma);
    s = run_hqs(g, T, o, labels_out,
                y->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, &res, st, &bb);
  } else if (o.profile || labels_out)
    s = run_hqs(g, T, o, labels_out,
                y->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, &res, st);
  else
    s = run_hqs_graph(g, T, o, &res, st);
  if (s != FEPLL_OK) return s;
  HIPX(copy_out(out, res, st));
  if (!out->on_device || !y->on_device || (labels_out && !y->on_device))
    HIPX(hipStreamSynchronize(st));
  return FEPLL_OK;
}

fepll_status fepll_restore_batch(fepll_gmm* g, int32_t n, const fepll_image* y,
                                 const double* sigma, fepll_image* out,
                                 const fepll_options* opt) {
  g_err.clear();
  TraceRange tr("fepll_restore_batch");
  if (!g) return fail(FEPLL_EINVAL, "gmm handle is NULL");
  if (n < 1 || n > kMaxBatch) return fail(FEPLL_EINVAL, "n must be in 1..65536");
  if (!y || !sigma || !out) return fail(FEPLL_EINVAL, "y, sigma and out must be non-NULL");
  fepll_options o;
  fepll_options_default(&o);
  if (opt) o = *opt;
  fepll_status s;
  if ((s = check_opt(g, &o)) != FEPLL_OK) return s;
  if (o.init) return fail(FEPLL_EINVAL, "options.init is not taken by fepll_restore_batch");
  std::vector<int> Hs(n), Ws(n);
  std::vector<double> betas;
  std::vector<float> bvals;
  bool host = false;
  for (int i = 0; i < n; ++i) {
    const std::string yi = "y[" + std::to_string(i) + "]";
    const std::string oi = "out[" + std::to_string(i) + "]";
    if ((s = check_image(&y[i], yi.c_str())) != FEPLL_OK) return s;
    if ((s = check_image(&out[i], oi.c_str())) != FEPLL_OK) return s;
    if (out[i].height != y[i].height || out[i].width != y[i].width)
      return fail(FEPLL_EINVAL, oi + " must have the shape of " + yi);
    if (!(sigma[i] > 0.0) || !std::isfinite(sigma[i]))
      return fail(FEPLL_EINVAL, "sigma[" + std::to_string(i) + "] must be > 0");
    if ((s = host_finite(&y[i], yi.c_str())) != FEPLL_OK) return s;
    Hs[i] = y[i].height;
    Ws[i] = y[i].width;
    for (int t = 0; t < kDefaultT; ++t) {
      betas.push_back(kDefaultB[t] / (sigma[i] * sigma[i]));
      bvals.push_back((float)kDefaultB[t]);  // beta sigma^2
    }
    host = host || !y[i].on_device || !out[i].on_device;
  }
  hipStream_t st = (hipStream_t)o.stream;
  if ((s = use_stream(g, st)) != FEPLL_OK) return s;
  g->profiling = profile_mask(o.profile);
  if ((s = make_plan(g, n, Hs.data(), Ws.data(), kDefaultT, bvals, st)) != FEPLL_OK) return s;
  if ((s = ensure_consts(g, betas, table_mask(o), st)) != FEPLL_OK) return s;
  if ((s = ensure_jitter(g, o)) != FEPLL_OK) return s;
  if (o.use_tree && (s = ensure_tree_consts(g, betas, st)) != FEPLL_OK) return s;
  for (int i = 0; i < n; ++i) HIPX(copy_in(g->ybuf + g->hd[i].px, &y[i], st));
  const int64_t px = g->hd[n - 1].px + (int64_t)Hs[n - 1] * Ws[n - 1];
  HIPX(hipMemcpyAsync(g->xa, g->ybuf, sizeof(float) * px, hipMemcpyDeviceToDevice, st));
  float* res = nullptr;
  if (o.profile) s = run_hqs(g, kDefaultT, o, nullptr, hipMemcpyDefault, &res, st);
  else s = run_hqs_graph(g, kDefaultT, o, &res, st);
  if (s != FEPLL_OK) return s;
  for (int i = 0; i < n; ++i) HIPX(copy_out(&out[i], res + g->hd[i].px, st));
  if (host) HIPX(hipStreamSynchronize(st));
  return FEPLL_OK;
}

fepll_status fepll_set_tuning(fepll_gmm* g, const fepll_tuning* t) {
  g_err.clear();
  if (!g) return fail(FEPLL_EINVAL, "gmm handle is NULL");
  fepll_tuning v;
  default_tuning(&v);
  if (t) v = *t;
  if (v.est_blocks < 0) return fail(FEPLL_EINVAL, "tuning.est_blocks must be >= 0");
  if (v.wiener_blocks < 8 || v.wiener_blocks % 8)
    return fail(FEPLL_EINVAL, "tuning.wiener_blocks must be a positive multiple of 8");
  if (v.ola_rows != 16 && v.ola_rows != 32 && v.ola_rows != 64)
    return fail(FEPLL_EINVAL, "tuning.ola_rows must be 16, 32 or 64");
  v.reserved = 0;
  g->tune = v;
  g->plan_valid = false;  // the reprojection tiles depend on ola_rows
  return FEPLL_OK;
}

fepll_status fepll_get_tuning(fepll_gmm* g, fepll_tuning* t) {
  g_err.clear();
  if (!g || !t) return fail(FEPLL_EINVAL, "NULL argument");
  *t = g->tune;
  return FEPLL_OK;
}

fepll_status fepll_autotune(fepll_gmm* g, int32_t n, const fepll_image* y, const double* sigma,
                            const fepll_options* opt, fepll_tuning* best) {
  g_err.clear();
  if (!g) return fail(FEPLL_EINVAL, "gmm handle is NULL");
  if (n < 1 || n > kMaxBatch || !y || !sigma)
    return fail(FEPLL_EINVAL, "1..65536 images with their sigma are needed");
  fepll_options o;
  fepll_options_default(&o);
  if (opt) o = *opt;
  o.profile = 1;
  fepll_status s;
  int64_t total = 0, largest = 0;
  for (int i = 0; i < n; ++i) {
    if ((s = check_image(&y[i], "y")) != FEPLL_OK) return s;
    total += (int64_t)y[i].height * y[i].width;
    largest = std::max<int64_t>(largest, (int64_t)y[i].height * y[i].width);
  }
  // a result kept for this kind of workload in the tuning cache
  const std::string ckey = tuning_key(g, o, n, total, largest);
  const char* cpath = std::getenv("FEPLL_TUNING_CACHE");
  fepll_tuning cached;
  if (cpath && *cpath && tuning_lookup(cpath, ckey, &cached)) {
    if ((s = fepll_set_tuning(g, &cached)) != FEPLL_OK) return s;
    if (best) *best = cached;
    return FEPLL_OK;
  }
  // every image is restored into a device scratch image
  float* scratch = nullptr;
  HIPX(dalloc(&scratch, (size_t)total));
  std::vector<fepll_image> outs(y, y + n);
  int64_t off = 0;
  for (int i = 0; i < n; ++i) {
    outs[i].data = scratch + off;
    outs[i].row_stride = y[i].width;
    outs[i].on_device = 1;
    off += (int64_t)y[i].height * y[i].width;
  }
  // Candidates per stage.  A stage's time does not depend on the other
  // stages' shapes, so trial r takes candidate r mod (count) of every stage:
  // 12 trials cover every candidate of every stage; each is kept at its
  // fastest trial.
  const int est_c[] = {0, 512, 768, 1024};
  const int wie_c[] = {1024, 2048, 4096, 8192};
  const int ola_c[] = {16, 32, 64};
  const int ne = 4, nw = 4, no = 3, trials = 12;
  std::vector<double> te(ne, 1e300), tw(nw, 1e300), to(no, 1e300);
  const fepll_tuning saved = g->tune;
  s = FEPLL_OK;
  for (int r = -1; r < trials && s == FEPLL_OK; ++r) {
    const int rr = r < 0 ? 0 : r;  // r = -1: warm-up (constants, scratch, code objects)
    const fepll_tuning t{est_c[rr % ne], wie_c[rr % nw], ola_c[rr % no], 0};
    if ((s = fepll_set_tuning(g, &t)) != FEPLL_OK) break;
    double ms[kStages];
    (void)fepll_profile(g, nullptr, nullptr, 0);
    if ((s = fepll_restore_batch(g, n, y, sigma, outs.data(), &o)) != FEPLL_OK) break;
    if ((s = fepll_profile(g, ms, nullptr, kStages)) != FEPLL_OK) break;
    if (r < 0) continue;
    te[rr % ne] = std::min(te[rr % ne], ms[0]);
    tw[rr % nw] = std::min(tw[rr % nw], ms[3]);
    to[rr % no] = std::min(to[rr % no], ms[4]);
  }
  (void)hipStreamSynchronize((hipStream_t)o.stream);
  dfree(scratch);
  if (s != FEPLL_OK) {
    const std::string msg = g_err;
    (void)fepll_set_tuning(g, &saved);
    return fail(s, msg);
  }
  const fepll_tuning t{est_c[std::min_element(te.begin(), te.end()) - te.begin()],
                       wie_c[std::min_element(tw.begin(), tw.end()) - tw.begin()],
                       ola_c[std::min_element(to.begin(), to.end()) - to.begin()], 0};
  if ((s = fepll_set_tuning(g, &t)) != FEPLL_OK) return s;
  if (best) *best = t;
  if (cpath && *cpath) tuning_store(cpath, ckey, t);
  return FEPLL_OK;
}

fepll_status fepll_gmm_flat_tail(fepll_gmm* g, double rho, int32_t* ranks) {
  g_err.clear();
  if (!g) return fail(FEPLL_EINVAL, "gmm handle is NULL");
  if (!(rho > 0.0 && rho <= 1.0)) return fail(FEPLL_EINVAL, "rho must be in (0, 1]");
  const int K = g->K;
  // Sec. 3.1: r_k is the smallest rank whose leading eigenvalues hold rho of
  // the trace; the eigenvalues after it are replaced by their average.  The
  // trace, the partial sums and the tail sum are taken in index order.
  std::vector<double> lam = g->lam_h;
  std::vector<int32_t> rk;
  flat_tail_host(lam, K, rho, rk);
  // tables and captured work of earlier calls read the spectra: let them end
  HIPX(hipDeviceSynchronize());
  if (!g->rk) HIPX(dalloc(&g->rk, (size_t)K));
  HIPX(hipMemcpy(g->lam64, lam.data(), sizeof(double) * lam.size(), hipMemcpyHostToDevice));
  HIPX(hipMemcpy(g->rk, rk.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice));
  g->tb.rk = (rho < 1.0) ? g->rk : nullptr;
  g->rho = rho;
  g->h_rk = rk;
  g->cbeta.clear();  // every per-beta table is rebuilt on next use
  g->cmask = 0;
  if (g->tree.Kall) {
    fepll_status s = tree_upload_spectra(g);
    if (s != FEPLL_OK) return s;
  }
  if (ranks) std::memcpy(ranks, rk.data(), sizeof(int32_t) * K);
  return FEPLL_OK;
}

fepll_status fepll_gmm_set_tree(fepll_gmm* g, int32_t nlevels, const int32_t* sizes,
                                const int32_t* parents) {
  g_err.clear();
  if (!g) return fail(FEPLL_EINVAL, "gmm handle is NULL");
  auto& T = g->tree;
  const int K = g->K;
  HIPX(hipDeviceSynchronize());
  ++g->tree_gen;
  auto clear = [&]() {
    dfree(T.U64);
    dfree(T.lam64);
    dfree(T.w64);
    dfree(T.rk);
    dfree(T.children);
    dfree(T.dnode);
    dfree(T.dpar);
    dfree(T.dlend);
    T = fepll_gmm::Tree{};
  };
  if (nlevels == 0) {
    dfree(T.dbeta);
    dfree(T.tb.Ub);
    dfree(T.tb.Wt);
    dfree(T.tb.L32);
    dfree(T.tb.Pinv);
    clear();
    return FEPLL_OK;
  }
  if (nlevels < 2 || nlevels > 16) return fail(FEPLL_EINVAL, "nlevels must be in 2..16");
  if (!sizes || !parents) return fail(FEPLL_EINVAL, "sizes and parents must be non-NULL");
  if (sizes[0] != 1) return fail(FEPLL_EINVAL, "sizes[0] must be 1 (the root)");
  if (sizes[nlevels - 1] != K) return fail(FEPLL_EINVAL, "the last level must have the K leaves");
  int64_t total = 0;
  for (int n = 0; n < nlevels; ++n) {
    if (sizes[n] < 1) return fail(FEPLL_EINVAL, "every level needs a node");
    total += sizes[n];
  }
  if (total > kMaxK) return fail(FEPLL_EUNSUPPORTED, "more than 1024 nodes in all");
  // parents per level, and every node above the leaves with 1..8 children
  std::vector<const int32_t*> par(nlevels, nullptr);
  {
    const int32_t* p = parents;
    for (int n = 1; n < nlevels; ++n) {
      par[n] = p;
      std::vector<int> cnt(sizes[n - 1], 0);
      for (int i = 0; i < sizes[n]; ++i) {
        if (p[i] < 0 || p[i] >= sizes[n - 1])
          return fail(FEPLL_EINVAL, "a parent index is out of its level");
        cnt[p[i]]++;
      }
      for (int c : cnt)
        if (c < 1 || c > 8) return fail(FEPLL_EINVAL, "every inner node needs 1..8 children");
      p += sizes[n];
    }
  }
  // node ids: leaves 0..K-1, then the levels nlevels-2 .. 0
  std::vector<int> base(nlevels, 0);
  int next = K;
  for (int n = nlevels - 2; n >= 0; --n) {
    base[n] = next;
    next += sizes[n];
  }
  const int Kall = next;
  // moment matching, leaves upwards, in float64
  std::vector<double> w((size_t)Kall, 0.0), Sg((size_t)Kall * kP * kP, 0.0);
  {
    std::vector<double> wl(K);
    HIPX(hipMemcpy(wl.data(), g->w64, sizeof(double) * K, hipMemcpyDeviceToHost));
    for (int k = 0; k < K; ++k) {
      w[k] = wl[k];
      const double* U = g->U_h.data() + (size_t)k * kP * kP;
      const double* l = g->lam_h.data() + (size_t)k * kP;
      double* S = Sg.data() + (size_t)k * kP * kP;
      for (int p = 0; p < kP; ++p)
        for (int q = 0; q < kP; ++q) {
          double a = 0.0;
          for (int j = 0; j < kP; ++j) a += U[p * kP + j] * l[j] * U[q * kP + j];
          S[p * kP + q] = a;
        }
    }
  }
  auto id = [&](int n, int i) { return (n == nlevels - 1) ? i : base[n] + i; };
  // an inner node first holds sum_{leaves below} w_l Sigma_l (its children's
  // weighted covariances for leaves, their sums for inner nodes), divided by
  // its weight once every level below is in
  for (int n = nlevels - 1; n >= 1; --n)
    for (int i = 0; i < sizes[n]; ++i) {
      const int c = id(n, i), q = id(n - 1, par[n][i]);
      w[q] += w[c];
      const double f = (n == nlevels - 1) ? w[c] : 1.0;
      const double* Sc = Sg.data() + (size_t)c * kP * kP;
      double* Sq = Sg.data() + (size_t)q * kP * kP;
      for (int e = 0; e < kP * kP; ++e) Sq[e] += f * Sc[e];
    }
  for (int n = nlevels - 2; n >= 0; --n)
    for (int i = 0; i < sizes[n]; ++i) {
      const int q = id(n, i);
      double* Sq = Sg.data() + (size_t)q * kP * kP;
      for (int e = 0; e < kP * kP; ++e) Sq[e] /= w[q];
    }
  // eigendecomposition of the inner nodes (leaves keep their own)
  std::vector<double> Uall((size_t)Kall * kP * kP), lall((size_t)Kall * kP);
  std::copy(g->U_h.begin(), g->U_h.end(), Uall.begin());
  std::copy(g->lam_h.begin(), g->lam_h.end(), lall.begin());
  if (Kall > K) {
    fepll_status s = fepll_cov_eig(Sg.data() + (size_t)K * kP * kP, Kall - K, kP,
                                   Uall.data() + (size_t)K * kP * kP, lall.data() + (size_t)K * kP);
    if (s != FEPLL_OK) return s;
  }
  // children table
  std::vector<uint16_t> ch((size_t)Kall * 8, 0xffffu);
  int maxch = 0;
  for (int n = nlevels - 1; n >= 1; --n)
    for (int i = 0; i < sizes[n]; ++i) {
      const int q = id(n - 1, par[n][i]);
      uint16_t* row = ch.data() + (size_t)q * 8;
      int j = 0;
      while (row[j] != 0xffffu) ++j;
      row[j] = (uint16_t)id(n, i);  // children in ascending index: ties to the lower one
      maxch = std::max(maxch, j + 1);
    }
  clear();
  T.Kall = Kall;
  T.root = id(0, 0);
  T.nlevels = nlevels;
  T.maxch = maxch;
  T.lvl_size.assign(sizes, sizes + nlevels);
  T.U_h = std::move(Uall);
  T.lam_h = std::move(lall);
  T.w_h = w;
  HIPX(dalloc(&T.U64, T.U_h.size()));
  HIPX(dalloc(&T.lam64, T.lam_h.size()));
  HIPX(dalloc(&T.w64, (size_t)Kall));
  HIPX(dalloc(&T.rk, (size_t)Kall));
  HIPX(dalloc(&T.children, ch.size()));
  HIPX(hipMemcpy(T.U64, T.U_h.data(), sizeof(double) * T.U_h.size(), hipMemcpyHostToDevice));
  HIPX(hipMemcpy(T.w64, w.data(), sizeof(double) * Kall, hipMemcpyHostToDevice));
  HIPX(hipMemcpy(T.children, ch.data(), sizeof(uint16_t) * ch.size(), hipMemcpyHostToDevice));
  {
    // dense top levels: a level of few nodes costs less scored for every
    // patch in one pass than sorted into (patch, child) pairs
    std::vector<int32_t> dn, dp, de;
    int lev = 1;
    for (; lev < nlevels && sizes[lev] <= kDenseNodes; ++lev) {
      for (int i = 0; i < sizes[lev]; ++i) {
        dn.push_back(id(lev, i));
        dp.push_back(id(lev - 1, par[lev][i]));
      }
      de.push_back((int32_t)dn.size());
    }
    T.dense_levels = lev - 1;
    T.dense_n = (int)dn.size();
    if (T.dense_levels > 0) {
      HIPX(dalloc(&T.dnode, dn.size()));
      HIPX(dalloc(&T.dpar, dp.size()));
      HIPX(dalloc(&T.dlend, de.size()));
      HIPX(hipMemcpy(T.dnode, dn.data(), sizeof(int32_t) * dn.size(), hipMemcpyHostToDevice));
      HIPX(hipMemcpy(T.dpar, dp.data(), sizeof(int32_t) * dp.size(), hipMemcpyHostToDevice));
      HIPX(hipMemcpy(T.dlend, de.data(), sizeof(int32_t) * de.size(), hipMemcpyHostToDevice));
    }
  }
  g->plan_valid = false;  // the pair scratch is sized for the tree's nodes
  return tree_upload_spectra(g);
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
  const std::vector<float> bv(1, 1.f);
  if ((s = make_plan(g, 1, &H, &W, 1, bv, st)) != FEPLL_OK) return s;
  HIPX(copy_in(g->xa, x, st));
  ProposeArgs p{};
  p.x = g->xa;
  p.H = H;
  p.W = W;
  p.logsb = (float)(-0.5 * std::log(beta));
  p.Wb = g->pWb;
  p.bias = g->pbias;
  p.K = g->K;
  p.m = top_m;
  p.cand = cand;
  HIPX(launch_propose(p, st));
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
  if (o.jitter) return fail(FEPLL_EUNSUPPORTED, "fepll_select runs on every patch (jitter = 0)");
  const int H = x->height, W = x->width;
  hipStream_t st = (hipStream_t)o.stream;
  if ((s = use_stream(g, st)) != FEPLL_OK) return s;
  g->profiling = profile_mask(o.profile);
  const std::vector<float> bv(1, 1.f);
  if ((s = make_plan(g, 1, &H, &W, 1, bv, st)) != FEPLL_OK) return s;
  if ((s = ensure_consts(g, std::vector<double>(1, beta), table_mask(o), st)) != FEPLL_OK)
    return s;
  if (o.use_tree && (s = ensure_tree_consts(g, std::vector<double>(1, beta), st)) != FEPLL_OK)
    return s;
  HIPX(copy_in(g->xa, x, st));
  return select_batch(g, 0, o, g->xa, labels, best, second, flags, st);
}

}  // extern "C"
