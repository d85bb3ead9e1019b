// Patch reprojection + image estimation (Alg. 1), fused:
//   x~ = (sum_i P_i^t P_i)^-1 sum_i P_i^t z^_i      (average of overlapping patches)
//   x  = (y + b x~) / (1 + b),  b = beta sigma^2     (A = identity)
//
// A gather, not a scatter: each output pixel sums the (up to 64) patch
// entries that cover it in a fixed order -- patch rows ascending (dy
// descending), and within a patch row dx ascending -- so the result is
// bitwise reproducible and needs no atomics.
//
// z^ is stored patch-major, Zhat[patch][dy][dx] (256 contiguous bytes per
// patch), so one patch row of a tile (71 patches) is one contiguous 18 KB
// run.  A workgroup owns TY output rows x 64 columns (TY = 16, 32 or 64, a
// tuning choice) and walks the TY + 7 patch rows that touch them, top to
// bottom: each patch row is staged in LDS (odd
// pitch, conflict-free reads) while the next one is in flight in registers,
// and every pixel row in flight keeps a running sum in a register of the
// thread that owns it (thread row j owns pixel rows = j mod 4, two of them
// in flight).  A pixel row is final once patch row y (dy = 0) is added.
//
// Tiles are numbered across the batch, image after image and column-strip-
// major within an image, and dealt so that consecutive tiles of a strip run
// on the same XCD at about the same time: the 7 patch rows a tile shares
// with the tile below are then read from that XCD's L2.
//
// The per-pixel patch count of the valid patch set is the product of a row
// and a column factor, cnt(y, x) = n(y, H) n(x, W) with
// n(v, S) = min(v, S-8) - max(0, v-7) + 1.
//
// SUB: a subset of the patches (the jittered subsampling of Sec. 3.3; a
// patch is in it when its label is below K).  Patches outside it are
// neither read nor counted: the spare slot of each staged patch (entry 64
// of its pitch) holds 1 or 0, summed like the entries into the pixel's
// count, and the average divides by that count (at least 1: the subset
// covers every pixel).  With every patch in the subset the sums, counts and
// results are the same bits as the full-set kernel's.
#include "common.h"

namespace fepll {

namespace {
constexpr int TX = kOlaX;
constexpr int NP = TX + 7;       // patches of one staged patch row
constexpr int PITCH = 65;        // floats per staged patch
constexpr int ROW = NP * PITCH;  // floats per staged patch row
constexpr int F4 = NP * 16;      // float4 of one patch row
constexpr int PER = (F4 + 255) / 256;
}  // namespace

template <int TY, bool SUB>
__global__ __launch_bounds__(256) void ola_update_kernel(Batch bt,
                                                         const float* __restrict__ Zhat_b,
                                                         const float* __restrict__ y_b,
                                                         const float* __restrict__ bvals, int it,
                                                         float* __restrict__ xnew_b,
                                                         const int32_t* __restrict__ labels_b,
                                                         int K) {
  __shared__ float buf[2][ROW];
  const int G8 = gridDim.x;  // a multiple of 8
  const int lin = (blockIdx.x & 7) * (G8 >> 3) + (blockIdx.x >> 3);
  if (lin >= bt.n_ola) return;
  const ImgDesc d = bt.d[bt.ola_img[lin]];
  const int H = d.H, W = d.W;
  const int Hp = H - 7, Wp = W - 7;
  const float b = bvals[d.slot0 + it];
  const float* Zhat = Zhat_b + (size_t)d.np * kP;
  const int32_t* labels = SUB ? labels_b + d.np : nullptr;
  const float* y = y_b + d.px;
  float* xnew = xnew_b + d.px;
  const int nty = (H + TY - 1) / TY;
  const int lt = lin - d.ola0;
  const int x0 = (lt / nty) * TX, y0 = (lt % nty) * TY;
  const int tx = threadIdx.x & 63, j = threadIdx.x >> 6;
  const int cfirst = x0 - 7;

  float4 pre[PER];
  float pin[SUB ? PER : 1];      // SUB: 1 when the patch is in the subset
  int32_t lnext[SUB ? PER : 1];  // SUB: the labels of the next patch row, loaded a row ahead
  // SUB: labels of patch row r for this thread's entries (K outside the image)
  auto fetch_labels = [&](int r) {
    if (!SUB) return;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int c = cfirst + (e >> 4);
      const bool in = e < F4 && r >= 0 && r < Hp && c >= 0 && c < Wp;
      lnext[u] = in ? labels[(size_t)r * Wp + c] : K;
    }
  };
  auto fetch = [&](int r) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + 256 * u;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      const int p = e >> 4, f = e & 15;
      const int c = cfirst + p;
      bool ok = e < F4 && r >= 0 && r < Hp && c >= 0 && c < Wp;
      if (SUB) {
        ok = ok && lnext[u] < K;
        pin[u] = ok ? 1.f : 0.f;
      }
      if (ok) v = *reinterpret_cast<const float4*>(Zhat + ((size_t)r * Wp + c) * kP + 4 * f);
      pre[u] = v;
    }
    fetch_labels(r + 1);  // (SUB) ready by the next fetch
  };
  auto stash = [&](float* B) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < F4) {
        float* q = B + (e >> 4) * PITCH + 4 * (e & 15);
        q[0] = pre[u].x;
        q[1] = pre[u].y;
        q[2] = pre[u].z;
        q[3] = pre[u].w;
        if (SUB && (e & 15) == 15) q[4] = pin[u];  // entry 64: in the subset
      }
    }
  };

  const int xx = x0 + tx;
  const float ncol = (float)(min(xx, W - 8) - max(0, xx - 7) + 1);
  const float onepb = 1.f + b;
  const int rb = y0 - 7, re = y0 + TY - 1;  // patch rows touching the tile
  // pixel rows in flight of this thread: ya (closer to final) and ya + 4
  int ya = rb + ((j - rb) & 3);
  float acc_a = 0.f, acc_b = 0.f;
  float cnt_a = 0.f, cnt_b = 0.f;  // SUB: subset patches covering rows ya, ya + 4
  fetch_labels(rb);
  fetch(rb);
  for (int r = rb; r <= re; ++r) {
    float* B = buf[(r - rb) & 1];
    stash(B);
    __syncthreads();
    if (r < re) fetch(r + 1);
    const int da = ya - r;  // 0..3
    const float* S = B + (tx + 7) * PITCH;
    float sa = 0.f, sb = 0.f;
#pragma unroll
    for (int dx = 0; dx < 8; ++dx) {
      sa += S[8 * da + dx - dx * PITCH];
      sb += S[8 * (da + 4) + dx - dx * PITCH];
    }
    acc_a += sa;
    acc_b += sb;
    if (SUB) {
      float n = 0.f;
#pragma unroll
      for (int dx = 0; dx < 8; ++dx) n += S[64 - dx * PITCH];
      cnt_a += n;
      cnt_b += n;
    }
    if (da == 0) {  // row ya has all its patch rows
      if (ya >= y0 && ya < H && xx < W) {
        const float nrow = (float)(min(ya, H - 8) - max(0, ya - 7) + 1);
        const float xt = acc_a / (SUB ? cnt_a : nrow * ncol);
        const size_t o = (size_t)ya * W + xx;
        xnew[o] = (y[o] + b * xt) / onepb;
      }
      ya += 4;
      acc_a = acc_b;
      acc_b = 0.f;
      cnt_a = cnt_b;
      cnt_b = 0.f;
    }
  }
}

template <bool SUB>
static void launch_ola_rows(const Batch& b, int blocks, const float* Zhat, const float* y,
                            const float* bvals, int t, float* xnew, const int32_t* labels, int K,
                            hipStream_t st) {
  if (b.ola_rows == 16)
    hipLaunchKernelGGL((ola_update_kernel<16, SUB>), dim3(blocks), dim3(256), 0, st, b, Zhat, y,
                       bvals, t, xnew, labels, K);
  else if (b.ola_rows == 64)
    hipLaunchKernelGGL((ola_update_kernel<64, SUB>), dim3(blocks), dim3(256), 0, st, b, Zhat, y,
                       bvals, t, xnew, labels, K);
  else
    hipLaunchKernelGGL((ola_update_kernel<32, SUB>), dim3(blocks), dim3(256), 0, st, b, Zhat, y,
                       bvals, t, xnew, labels, K);
}

hipError_t launch_ola_batch(const Batch& b, const float* Zhat, const float* y,
                            const float* bvals, int t, float* xnew, const int32_t* subset_labels,
                            int K, hipStream_t st) {
  const int blocks = (b.n_ola + 7) & ~7;  // whole rounds over the 8 XCDs
  if (subset_labels)
    launch_ola_rows<true>(b, blocks, Zhat, y, bvals, t, xnew, subset_labels, K, st);
  else
    launch_ola_rows<false>(b, blocks, Zhat, y, bvals, t, xnew, nullptr, K, st);
  return hipGetLastError();
}

}  // namespace fepll
