// fepll_select_static: the float32 Gaussian selection of fepll_select
// (Alg. 1, Gaussian selection, in the eigenspace form of Sec. 2.1, every
// patch certified or re-selected in float64) with no device allocation.
// Everything the step needs beyond its inputs, its outputs and the handle's
// float64 mixture -- the per-beta tables, the count and list of uncertified
// patches -- lives in one file-scope device array of fixed size, one copy per
// GPU, kept until the process ends.  Its device address is taken once per
// device (hipGetSymbolAddress, with that device current) and only that
// address reaches the kernels.  The count is cleared by a kernel, so the
// call records no memset and allocates nothing under graph capture.  Every
// call on a device shares that device's array: calls that overlap on one
// GPU (other streams, other threads) race and must be serialised by the
// caller.
#include <mutex>

#include "common.h"
#include "fepll.h"
#include "internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per GPU
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices];  // device address of scratch on each GPU

// The device address of this device's array (taken on first use, with the
// device current).
fepll_status scratch_on(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fepll::fail(FEPLL_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                            hipGetErrorString(e));
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[dev];
  return FEPLL_OK;
}

size_t up256(size_t n) { return (n + 255) & ~size_t(255); }

// Offsets of the regions of the array for K components and Np patches.
struct Layout {
  size_t beta, Ut, Wt, L32, L64, invnu, count, list, end;
  Layout(size_t K, size_t Np) {
    size_t o = 0;
    beta = o;
    o += up256(sizeof(double));
    Ut = o;
    o += up256(K * fepll::kTileStride * sizeof(float));
    Wt = o;
    o += up256(K * fepll::kTileStride * sizeof(float));
    L32 = o;
    o += up256(K * sizeof(float));
    L64 = o;
    o += up256(K * sizeof(double));
    invnu = o;
    o += up256(K * fepll::kP * sizeof(double));
    count = o;
    o += 256;
    list = o;
    o += up256(Np * 4 * sizeof(int32_t));  // int4 entries
    end = o;
  }
};

__global__ void put_beta_kernel(double* b, double beta, int32_t* count) {
  b[0] = beta;
  count[0] = 0;
}

}  // namespace

extern "C" {

fepll_status fepll_select_static(fepll_gmm* g, const fepll_image* x, double beta,
                                 int32_t* labels, float* best, float* second, int32_t* flags,
                                 void* stream) {
  using namespace fepll;
  clear_error();
  if (!g) return fail(FEPLL_EINVAL, "gmm handle is NULL");
  if (!x || !x->data) return fail(FEPLL_EINVAL, "x is NULL");
  if (!labels) return fail(FEPLL_EINVAL, "labels is NULL");
  if (!x->on_device) return fail(FEPLL_EINVAL, "fepll_select_static takes a device image");
  if (x->height < 8 || x->width < 8)
    return fail(FEPLL_EINVAL, "x: height and width must be >= 8");
  if (x->row_stride != 0 && x->row_stride != x->width)
    return fail(FEPLL_EINVAL, "fepll_select_static takes a contiguous image (row_stride = width)");
  if (!(beta > 0.0) || !std::isfinite(beta)) return fail(FEPLL_EINVAL, "beta must be > 0");
  const GmmView v = gmm_view(g);
  const int H = x->height, W = x->width;
  const size_t Np = (size_t)(H - 7) * (W - 7);
  const Layout L((size_t)v.K, Np);
  if (L.end > kScratchBytes)
    return fail(FEPLL_EINVAL, "fepll_select_static: K = " + std::to_string(v.K) + " and " +
                                  std::to_string(Np) + " patches need " +
                                  std::to_string(L.end) + " bytes of scratch, above its " +
                                  std::to_string(kScratchBytes));
  int dev = -1;
  HIPX(hipGetDevice(&dev));
  if (dev != v.device)
    return fail(FEPLL_EINVAL, "fepll_select_static: the current device is not the handle's");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(FEPLL_EUNSUPPORTED, "fepll_select_static: device index out of range");
  unsigned char* base = nullptr;
  fepll_status s;
  if ((s = scratch_on(dev, &base)) != FEPLL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  double* dbeta = reinterpret_cast<double*>(base + L.beta);
  int32_t* count = reinterpret_cast<int32_t*>(base + L.count);
  int32_t* list = reinterpret_cast<int32_t*>(base + L.list);
  ConstTables tb{};
  tb.Ut = reinterpret_cast<float*>(base + L.Ut);
  tb.Wt = reinterpret_cast<float*>(base + L.Wt);
  tb.L32 = reinterpret_cast<float*>(base + L.L32);
  tb.L64 = reinterpret_cast<double*>(base + L.L64);
  tb.invnu64 = reinterpret_cast<double*>(base + L.invnu);
  hipLaunchKernelGGL(put_beta_kernel, dim3(1), dim3(1), 0, st, dbeta, beta, count);
  HIPX(hipGetLastError());
  HIPX(launch_prep(v.U64, v.lam64, v.w64, v.K, dbeta, 1, kTabF32, tb, st));
  HIPX(launch_estep_f32(x->data, H, W, tb.Ut, tb.L32, v.K, beta, labels, best, second, flags,
                        count, list, st));
  HIPX(launch_recheck_f64(x->data, H, W, v.U64, tb.invnu64, tb.L64, v.K, count, list, labels,
                          (int)Np, st));
  return FEPLL_OK;
}

}  // extern "C"
