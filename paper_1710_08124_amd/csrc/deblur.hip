// Image estimation of Alg. 1 for a periodic convolution A (deblurring):
// x = (A^t A + b I)^-1 (A^t y + b x~), b = beta sigma^2, is a pointwise
// division in the Fourier basis (A's eigenvalues are the DFT of its kernel,
// Sec. 2.1's remark on fast transforms); the start of Sec. 5,
// x = (A^t A + c Lap)^-1 A^t y with c = 0.2 sigma^2 / lambda and Lap the
// positive semidefinite periodic 5-point Laplacian, is the same division
// with c Lap's eigenvalues in place of b.
//
// The transforms are float64 (hipFFT D2Z / Z2D on the half spectrum,
// H x (W/2 + 1)): the update adds nothing measurable to the float32
// rounding of the patch steps.  Kernels here are elementwise over the image
// or the half spectrum.
#include <hip/hip_runtime.h>

#include "common.h"

namespace fepll {

namespace {

__global__ void f2d_kernel(const float* __restrict__ in, double* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

__global__ void d2f_scale_kernel(const double* __restrict__ in, float* __restrict__ out, int n,
                                 double scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)(in[i] * scale);
}

// AtY = conj(Hh) Yh, a2 = |Hh|^2 (half spectrum, m entries)
__global__ void spec_prep_kernel(const double2* __restrict__ Hh, const double2* __restrict__ Yh,
                                 double2* __restrict__ AtY, double* __restrict__ a2, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double2 h = Hh[i], y = Yh[i];
  AtY[i] = make_double2(h.x * y.x + h.y * y.y, h.x * y.y - h.y * y.x);
  a2[i] = h.x * h.x + h.y * h.y;
}

// X = (AtY + b Xt) / (a2 + b), in place on Xt
__global__ void spec_update_kernel(const double2* __restrict__ AtY, const double* __restrict__ a2,
                                   double2* __restrict__ X, int m, double b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double2 t = X[i], a = AtY[i];
  const double inv = 1.0 / (a2[i] + b);
  X[i] = make_double2((a.x + b * t.x) * inv, (a.y + b * t.y) * inv);
}

// X = AtY / (a2 + c (4 - 2 cos(2 pi k / H) - 2 cos(2 pi l / W))) on the half
// spectrum (row k, column l < W/2 + 1)
__global__ void spec_init_kernel(const double2* __restrict__ AtY, const double* __restrict__ a2,
                                 double2* __restrict__ X, int H, int W, double c) {
  const int Wh = W / 2 + 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H * Wh) return;
  const int k = i / Wh, l = i - k * Wh;
  const double two_pi = 6.283185307179586476925286766559;
  const double lap = 4.0 - 2.0 * cos(two_pi * k / H) - 2.0 * cos(two_pi * l / W);
  const double den = a2[i] + c * lap;
  const double2 a = AtY[i];
  X[i] = make_double2(a.x / den, a.y / den);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_f2d(const float* in, double* out, int n, hipStream_t st) {
  hipLaunchKernelGGL(f2d_kernel, dim3(blocks_for(n)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

hipError_t launch_d2f_scale(const double* in, float* out, int n, double scale, hipStream_t st) {
  hipLaunchKernelGGL(d2f_scale_kernel, dim3(blocks_for(n)), dim3(256), 0, st, in, out, n, scale);
  return hipGetLastError();
}

hipError_t launch_spec_prep(const void* Hh, const void* Yh, void* AtY, double* a2, int m,
                            hipStream_t st) {
  hipLaunchKernelGGL(spec_prep_kernel, dim3(blocks_for(m)), dim3(256), 0, st,
                     static_cast<const double2*>(Hh), static_cast<const double2*>(Yh),
                     static_cast<double2*>(AtY), a2, m);
  return hipGetLastError();
}

hipError_t launch_spec_update(const void* AtY, const double* a2, void* X, int m, double b,
                              hipStream_t st) {
  hipLaunchKernelGGL(spec_update_kernel, dim3(blocks_for(m)), dim3(256), 0, st,
                     static_cast<const double2*>(AtY), a2, static_cast<double2*>(X), m, b);
  return hipGetLastError();
}

hipError_t launch_spec_init(const void* AtY, const double* a2, void* X, int H, int W, double c,
                            hipStream_t st) {
  hipLaunchKernelGGL(spec_init_kernel, dim3(blocks_for((int64_t)H * (W / 2 + 1))), dim3(256), 0,
                     st, static_cast<const double2*>(AtY), a2, static_cast<double2*>(X), H, W, c);
  return hipGetLastError();
}

}  // namespace fepll
