// Patch reprojection + image estimation (Alg. 1), fused:
//   x~ = (sum_i P_i^t P_i)^-1 sum_i P_i^t z^_i      (average of overlapping patches)
//   x  = (y + b x~) / (1 + b),  b = beta sigma^2     (A = identity)
//
// A gather, not a scatter: each output pixel sums the (up to 64) patch
// entries that cover it in a fixed order -- dy ascending (patch rows
// descending), dx ascending -- so the result is bitwise reproducible and
// needs no atomics.
//
// z^ is stored in row planes, Zhat[dy][patch][dx]: output row y takes row
// dy of the patches of patch row y - dy, so every (plane, patch row)
// segment is read by exactly one output row and only the 7-column halo of a
// tile is read twice.  A workgroup owns 16 output rows x 64 columns and
// walks 2 groups of 8 rows x 8 planes; each round stages the 8 segments of
// a group (8 x 71 patches x 8 floats) in LDS with a 9-float pitch
// (conflict-free reads), while the next round's segments are already in
// flight in registers.
//
// The per-pixel patch count of the valid patch set is the product of a row
// and a column factor, cnt(y, x) = n(y, H) n(x, W) with
// n(v, S) = min(v, S-8) - max(0, v-7) + 1.
#include "common.h"

namespace fepll {

namespace {
constexpr int TX = 64;
constexpr int TY = 16;
constexpr int NP = TX + 7;      // patches per segment
constexpr int PITCH = 9;        // floats per staged patch row
constexpr int SEG = NP * PITCH;
constexpr int F4 = 8 * NP * 2;  // float4 of one round (8 segments x NP patches x 2)
constexpr int PER = (F4 + 255) / 256;
}  // namespace

__global__ __launch_bounds__(256) void ola_update_kernel(const float* __restrict__ Zhat,
                                                         const float* __restrict__ y, int H,
                                                         int W, float b,
                                                         float* __restrict__ xnew) {
  __shared__ float buf[2][8 * SEG];
  const int Hp = H - 7, Wp = W - 7;
  const size_t Np8 = (size_t)Hp * Wp * 8;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int cfirst = x0 - 7;

  // round q = (group, dy): segments j = 0..7 are (plane dy, patch row y0 + 8 group + j - dy)
  float4 pre[PER];
  auto fetch = [&](int q) {
    const int grp = q >> 3, dy = q & 7;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + 256 * u;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < F4) {
        const int j = e / (2 * NP), rem = e - j * 2 * NP;
        const int p = rem >> 1, h = rem & 1;
        const int r = y0 + 8 * grp + j - dy, c = cfirst + p;
        if (r >= 0 && r < Hp && c >= 0 && c < Wp)
          v = *reinterpret_cast<const float4*>(Zhat + dy * Np8 + ((size_t)r * Wp + c) * 8 +
                                               4 * h);
      }
      pre[u] = v;
    }
  };
  auto stash = [&](int q) {
    float* B = buf[q & 1];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < F4) {
        const int j = e / (2 * NP), rem = e - j * 2 * NP;
        const int p = rem >> 1, h = rem & 1;
        float* d = B + j * SEG + p * PITCH + 4 * h;
        d[0] = pre[u].x;
        d[1] = pre[u].y;
        d[2] = pre[u].z;
        d[3] = pre[u].w;
      }
    }
  };

  const int nq = 2 * 8;
  fetch(0);
  float acc[2][2] = {{0.f, 0.f}, {0.f, 0.f}};  // [group][row of the pair]
  for (int q = 0; q < nq; ++q) {
    stash(q);
    __syncthreads();
    if (q + 1 < nq) fetch(q + 1);
    const float* B = buf[q & 1];
    const int grp = q >> 3;
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      const int j = 2 * ty + jj;
      const float* S = B + j * SEG + (tx + 7) * PITCH;
      const int dy = q & 7;
      float s = 0.f;
#pragma unroll
      for (int dx = 0; dx < 8; ++dx) s += S[dx - dx * PITCH];
      // the segment row is zero where the patch does not exist
      (void)dy;
      if (grp == 0) acc[0][jj] += s;
      else acc[1][jj] += s;
    }
    __syncthreads();
  }
  const int xx = x0 + tx;
  if (xx >= W) return;
  const float ncol = (float)(min(xx, W - 8) - max(0, xx - 7) + 1);
  const float onepb = 1.f + b;
#pragma unroll
  for (int grp = 0; grp < 2; ++grp)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      const int yy = y0 + 8 * grp + 2 * ty + jj;
      if (yy < H) {
        const float nrow = (float)(min(yy, H - 8) - max(0, yy - 7) + 1);
        const float xt = acc[grp][jj] / (nrow * ncol);
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
