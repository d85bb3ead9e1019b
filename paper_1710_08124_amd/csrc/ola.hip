// Patch reprojection + image estimation (Alg. 1), fused:
//   x~ = (sum_i P_i^t P_i)^-1 sum_i P_i^t z^_i      (average of overlapping patches)
//   x  = (y + b x~) / (1 + b),  b = beta sigma^2     (A = identity)
// (raw: x~ itself, for an operator A whose image estimation follows in the
// Fourier basis, deblur.hip)
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

template <int TY>
__global__ __launch_bounds__(256) void ola_update_kernel(Batch bt,
                                                         const float* __restrict__ Zhat_b,
                                                         const float* __restrict__ y_b,
                                                         const float* __restrict__ bvals, int it,
                                                         float* __restrict__ xnew_b, int raw) {
  __shared__ float buf[2][ROW];
  const int G8 = gridDim.x;  // a multiple of 8
  const int lin = (blockIdx.x & 7) * (G8 >> 3) + (blockIdx.x >> 3);
  if (lin >= bt.n_ola) return;
  const ImgDesc d = bt.d[bt.ola_img[lin]];
  const int H = d.H, W = d.W;
  const int Hp = H - 7, Wp = W - 7;
  const float b = bvals[d.slot0 + it];
  const float* Zhat = Zhat_b + (size_t)d.np * kP;
  const float* y = y_b + d.px;
  float* xnew = xnew_b + d.px;
  const int nty = (H + TY - 1) / TY;
  const int lt = lin - d.ola0;
  const int x0 = (lt / nty) * TX, y0 = (lt % nty) * TY;
  const int tx = threadIdx.x & 63, j = threadIdx.x >> 6;
  const int cfirst = x0 - 7;

  float4 pre[PER];
  auto fetch = [&](int r) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + 256 * u;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      const int p = e >> 4, f = e & 15;
      const int c = cfirst + p;
      if (e < F4 && r >= 0 && r < Hp && c >= 0 && c < Wp)
        v = *reinterpret_cast<const float4*>(Zhat + ((size_t)r * Wp + c) * kP + 4 * f);
      pre[u] = v;
    }
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
    if (da == 0) {  // row ya has all its patch rows
      if (ya >= y0 && ya < H && xx < W) {
        const float nrow = (float)(min(ya, H - 8) - max(0, ya - 7) + 1);
        const float xt = acc_a / (nrow * ncol);
        const size_t o = (size_t)ya * W + xx;
        xnew[o] = raw ? xt : (y[o] + b * xt) / onepb;
      }
      ya += 4;
      acc_a = acc_b;
      acc_b = 0.f;
    }
  }
}

// ---- subset reprojection (jittered subsampling, Sec. 3.3).  The same
// tiles; a tile first lists the chosen patches of its window (the
// (TY + 7) x 71 patches that touch it; a patch is chosen when its label is
// below K) in raster order, by a ballot compaction into LDS, then stages
// their estimates 64 patches at a time in LDS, and every thread adds, to the
// pixels it owns (column tx, rows j, j + 4, ...), the entries of the listed
// patches that cover them, in list order, counting them: a fixed order, no
// atomics, and work in proportion to the chosen patches, not to all.
template <int TY>
__global__ __launch_bounds__(256) void ola_subset_kernel(Batch bt, const float* __restrict__ Zhat_b,
                                                         const float* __restrict__ y_b,
                                                         const float* __restrict__ bvals, int it,
                                                         float* __restrict__ xnew_b,
                                                         const int32_t* __restrict__ labels_b,
                                                         int K, int raw) {
  constexpr int WR = TY + 7;          // patch rows of the window
  constexpr int WIN = WR * NP;        // patches of the window
  constexpr int CH = 64;              // patches staged at a time
  constexpr int NR = TY / 4;          // pixel rows per thread
  __shared__ int16_t plist[WIN];      // chosen patches: window row * NP + column
  __shared__ float zs[CH * PITCH];
  __shared__ int wcnt[4];
  const int G8 = gridDim.x;
  const int lin = (blockIdx.x & 7) * (G8 >> 3) + (blockIdx.x >> 3);
  if (lin >= bt.n_ola) return;
  const ImgDesc d = bt.d[bt.ola_img[lin]];
  const int H = d.H, W = d.W;
  const int Hp = H - 7, Wp = W - 7;
  const float b = bvals[d.slot0 + it];
  const float* Zhat = Zhat_b + (size_t)d.np * kP;
  const int32_t* labels = labels_b + d.np;
  const float* y = y_b + d.px;
  float* xnew = xnew_b + d.px;
  const int nty = (H + TY - 1) / TY;
  const int lt = lin - d.ola0;
  const int x0 = (lt / nty) * TX, y0 = (lt % nty) * TY;
  const int tx = threadIdx.x & 63, j = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rfirst = y0 - 7, cfirst = x0 - 7;

  // 1. the window's chosen patches, raster order: thread t tests window
  // entries t * PT .. t * PT + PT - 1 (all its label loads in flight at
  // once), then a block-wide exclusive scan of the counts places them
  constexpr int PT = (WIN + 255) / 256;
  bool in[PT];
  int mine = 0;
#pragma unroll
  for (int u = 0; u < PT; ++u) {
    const int w = threadIdx.x * PT + u;
    const int r = rfirst + w / NP, c = cfirst + w % NP;
    in[u] = w < WIN && r >= 0 && r < Hp && c >= 0 && c < Wp &&
            labels[(size_t)r * Wp + c] < K;
  }
#pragma unroll
  for (int u = 0; u < PT; ++u) mine += in[u] ? 1 : 0;
  int incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wcnt[wave] = incl;
  __syncthreads();
  int pos = incl - mine;
#pragma unroll
  for (int v = 0; v < 4; ++v) pos += (v < wave) ? wcnt[v] : 0;
  const int n = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
#pragma unroll
  for (int u = 0; u < PT; ++u)
    if (in[u]) plist[pos++] = (int16_t)(threadIdx.x * PT + u);
  __syncthreads();

  // 2. accumulate, CH patches at a time
  float acc[NR], cnt[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) acc[i] = cnt[i] = 0.f;
  const int xx = x0 + tx;
  for (int c0 = 0; c0 < n; c0 += CH) {
    const int m = min(CH, n - c0);
    // stage: 16 float4 per patch
    for (int e = threadIdx.x; e < m * 16; e += 256) {
      const int q = e >> 4, f = e & 15;
      const int w = plist[c0 + q];
      const int r = rfirst + w / NP, c = cfirst + w % NP;
      const float4 v = *reinterpret_cast<const float4*>(Zhat + ((size_t)r * Wp + c) * kP + 4 * f);
      float* zp = zs + q * PITCH + 4 * f;
      zp[0] = v.x;
      zp[1] = v.y;
      zp[2] = v.z;
      zp[3] = v.w;
    }
    __syncthreads();
    for (int q = 0; q < m; ++q) {
      const int w = plist[c0 + q];
      const int r = rfirst + w / NP, c = cfirst + w % NP;
      const int dx = xx - c;
      if (dx < 0 || dx >= 8) continue;
      const float* zp = zs + q * PITCH + dx;
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int dy = y0 + j + 4 * i - r;
        if (dy >= 0 && dy < 8) {
          acc[i] += zp[8 * dy];
          cnt[i] += 1.f;
        }
      }
    }
    __syncthreads();  // zs is restaged
  }

  // 3. average and image update
  const float onepb = 1.f + b;
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int yy = y0 + j + 4 * i;
    if (yy < H && xx < W) {
      const size_t o = (size_t)yy * W + xx;
      const float xt = acc[i] / cnt[i];
      xnew[o] = raw ? xt : (y[o] + b * xt) / onepb;
    }
  }
}

template <bool SUB>
static void launch_ola_rows(const Batch& b, int blocks, const float* Zhat, const float* y,
                            const float* bvals, int t, float* xnew, const int32_t* labels, int K,
                            int raw, hipStream_t st) {
  if (SUB) {
    if (b.ola_rows == 16)
      hipLaunchKernelGGL(ola_subset_kernel<16>, dim3(blocks), dim3(256), 0, st, b, Zhat, y, bvals,
                         t, xnew, labels, K, raw);
    else if (b.ola_rows == 64)
      hipLaunchKernelGGL(ola_subset_kernel<64>, dim3(blocks), dim3(256), 0, st, b, Zhat, y, bvals,
                         t, xnew, labels, K, raw);
    else
      hipLaunchKernelGGL(ola_subset_kernel<32>, dim3(blocks), dim3(256), 0, st, b, Zhat, y, bvals,
                         t, xnew, labels, K, raw);
    return;
  }
  if (b.ola_rows == 16)
    hipLaunchKernelGGL(ola_update_kernel<16>, dim3(blocks), dim3(256), 0, st, b, Zhat, y, bvals, t,
                       xnew, raw);
  else if (b.ola_rows == 64)
    hipLaunchKernelGGL(ola_update_kernel<64>, dim3(blocks), dim3(256), 0, st, b, Zhat, y, bvals, t,
                       xnew, raw);
  else
    hipLaunchKernelGGL(ola_update_kernel<32>, dim3(blocks), dim3(256), 0, st, b, Zhat, y, bvals, t,
                       xnew, raw);
}

hipError_t launch_ola_batch(const Batch& b, const float* Zhat, const float* y,
                            const float* bvals, int t, float* xnew, const int32_t* subset_labels,
                            int K, int raw, hipStream_t st) {
  const int blocks = (b.n_ola + 7) & ~7;  // whole rounds over the 8 XCDs
  if (subset_labels)
    launch_ola_rows<true>(b, blocks, Zhat, y, bvals, t, xnew, subset_labels, K, raw, st);
  else
    launch_ola_rows<false>(b, blocks, Zhat, y, bvals, t, xnew, nullptr, K, raw, st);
  return hipGetLastError();
}

}  // namespace fepll
