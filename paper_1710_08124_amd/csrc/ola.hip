// Patch reprojection + image estimation (Alg. 1), fused:
//   x~ = (sum_i P_i^t P_i)^-1 sum_i P_i^t z^_i      (average of overlapping patches)
//   x  = (y + b x~) / (1 + b),  b = beta sigma^2     (A = identity)
//
// A gather, not a scatter: each output pixel sums the (up to 64) patch
// entries that cover it in a fixed order -- patch rows ascending, then
// columns descending inside a row -- so the result is bitwise reproducible
// and needs no atomics.  A workgroup owns a 32 x 64 block of output pixels;
// it walks the 39 patch rows that touch the block, stages each row's z^
// vectors (71 patches x 64 floats, one contiguous stretch of memory) in LDS
// with a 65-float pitch (consecutive lanes then hit consecutive banks), and
// every thread accumulates the row's contribution to its 8 pixels.
//
// The per-pixel patch count of the valid patch set is the product of a row
// and a column factor, cnt(y, x) = n(y, H) n(x, W) with
// n(v, S) = min(v, S-8) - max(0, v-7) + 1.
#include "common.h"

namespace fepll {

namespace {
constexpr int TX = 64;
constexpr int TY = 32;
constexpr int PITCH = 65;
}  // namespace

__global__ __launch_bounds__(256) void ola_update_kernel(const float* __restrict__ Zhat,
                                                         const float* __restrict__ y, int H,
                                                         int W, float b,
                                                         float* __restrict__ xnew) {
  __shared__ float buf[(TX + 7) * PITCH];
  const int Hp = H - 7, Wp = W - 7;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  float acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = 0.f;
  const int cfirst = x0 - 7;
  const int rlo = max(0, y0 - 7), rhi = min(Hp - 1, y0 + TY - 1);
  for (int r = rlo; r <= rhi; ++r) {
    __syncthreads();
    for (int e = threadIdx.x; e < (TX + 7) * 16; e += blockDim.x) {
      const int slot = e >> 4, q4 = e & 15;
      const int c = cfirst + slot;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (c >= 0 && c < Wp)
        v = reinterpret_cast<const float4*>(Zhat + ((size_t)r * Wp + c) * kP)[q4];
      float* d = buf + slot * PITCH + q4 * 4;
      d[0] = v.x;
      d[1] = v.y;
      d[2] = v.z;
      d[3] = v.w;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int dy = y0 + ty * 8 + i - r;
      if (dy >= 0 && dy < 8) {
        float s = 0.f;
#pragma unroll
        for (int dx = 0; dx < 8; ++dx) s += buf[(tx + 7 - dx) * PITCH + 8 * dy + dx];
        acc[i] += s;
      }
    }
  }
  const int xx = x0 + tx;
  if (xx >= W) return;
  const float ncol = (float)(min(xx, W - 8) - max(0, xx - 7) + 1);
  const float onepb = 1.f + b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int yy = y0 + ty * 8 + i;
    if (yy < H) {
      const float nrow = (float)(min(yy, H - 8) - max(0, yy - 7) + 1);
      const float xt = acc[i] / (nrow * ncol);
      const size_t o = (size_t)yy * W + xx;
      xnew[o] = (y[o] + b * xt) / onepb;
    }
  }
}

hipError_t launch_ola_update(const float* Zhat, const float* y, int H, int W, double b,
                             float* xnew, hipStream_t st) {
  dim3 grid((W + TX - 1) / TX, (H + TY - 1) / TY);
  hipLaunchKernelGGL(ola_update_kernel, grid, dim3(256), 0, st, Zhat, y, H, W, (float)b, xnew);
  return hipGetLastError();
}

}  // namespace fepll
