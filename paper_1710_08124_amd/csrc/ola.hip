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

#include "jitter_draw.h"

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
// tiles, each cut into parts of TY rows, one workgroup per part.  A part's
// window is the (TY + 7) x 71 patches that touch it; a patch is chosen when
// its member word differs from `none` (a label below K, or a set flag).
//   1. one bit per window patch: each window row is two ballots (columns
//      0..63 and 64..70) over coalesced label loads; a wave scan of the rows'
//      popcounts gives every chosen patch its slot in raster order, and the
//      slots are listed (plist) in LDS;
//   2. the chosen patches' estimates are staged in LDS, CH slots at a time,
//      every load of a chunk in flight at once;
//   3. a thread owns column tx and pixel rows j, j + 4, ...; the patches
//      covering pixel (y, x) start in window rows y - y0 .. y - y0 + 7 and
//      window columns tx .. tx + 7, so each window row the thread touches
//      gives an 8-bit field of its mask, and a set bit's slot is the row's
//      base plus the popcount of the bits before it.  A pixel sums its
//      patches' entries in raster order of the patches (fixed, no atomics),
//      and its count is the popcount of its 8 fields.
template <int TY>
__global__ __launch_bounds__(256) void ola_subset_kernel(Batch bt, const float* __restrict__ Zhat_b,
                                                         const float* __restrict__ y_b,
                                                         const float* __restrict__ bvals, int it,
                                                         float* __restrict__ xnew_b,
                                                         const int32_t* __restrict__ member_b,
                                                         int none, int raw, int nparts,
                                                         JitterDraw draw, int draw_blocks) {
  constexpr int WR = TY + 7;          // patch rows of the window
  constexpr int WIN = WR * NP;        // patches of the window
  constexpr int CH = 128;             // patches staged at a time
  constexpr int NR = TY / 4;          // pixel rows per thread
  constexpr int RPW = (WR + 3) / 4;   // window rows per wave in step 1
  constexpr int SPT = CH * 16 / 256;  // float4 staged per thread per chunk
  static_assert(WR <= 128, "two window rows per lane in the scan");
  __shared__ uint64_t mlo[WR], mhi[WR];  // chosen: columns 0..63, 64..70
  __shared__ int rbase[WR + 1];          // chosen patches in the rows above
  __shared__ int16_t plist[WIN];         // slot -> window row * NP + column
  __shared__ float zs[CH * PITCH];
  // workgroups past the nparts of the reprojection run the drawing of the
  // next iteration (disjoint words: other flags, list and count)
  if ((int)blockIdx.x >= nparts) {
    jitter_draw_block<true>(draw, (int)blockIdx.x - nparts, draw_blocks);
    return;
  }
  // a planned tile (64 x ola_rows) is cut into ola_rows / TY workgroups of
  // TY rows (short tiles: more workgroups in flight for a sparse subset)
  const int G8 = nparts;
  const int sub = bt.ola_rows / TY;
  const int lin2 = (blockIdx.x & 7) * (G8 >> 3) + (blockIdx.x >> 3);
  if (lin2 >= bt.n_ola * sub) return;
  const int lin = lin2 / sub, part = lin2 - lin * sub;
  const ImgDesc d = bt.d[bt.ola_img[lin]];
  const int H = d.H, W = d.W;
  const int Hp = H - 7, Wp = W - 7;
  const float b = bvals[d.slot0 + it];
  const float* Zhat = Zhat_b + (size_t)d.np * kP;
  const int32_t* member = member_b + d.np;
  const float* y = y_b + d.px;
  float* xnew = xnew_b + d.px;
  const int nty = (H + bt.ola_rows - 1) / bt.ola_rows;
  const int lt = lin - d.ola0;
  const int x0 = (lt / nty) * TX, y0 = (lt % nty) * bt.ola_rows + part * TY;
  if (y0 >= H) return;  // (a part below the image)
  const int tx = threadIdx.x & 63, j = threadIdx.x >> 6;
  const int lane = tx, wave = j;
  const int rfirst = y0 - 7, cfirst = x0 - 7;
  // y of the thread's pixels, loaded now so that the update at the end does
  // not wait for them
  float yv[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int yy = y0 + j + 4 * i;
    yv[i] = (!raw && yy < H && x0 + tx < W) ? y[(size_t)yy * W + x0 + tx] : 0.f;
  }

  // 1. masks: wave w takes window rows w, w + 4, ... (all loads first)
  {
    int la[RPW], lb[RPW];
    const int c = cfirst + lane, c2 = cfirst + 64 + lane;
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
      const int rw = wave + 4 * u, r = rfirst + rw;
      const bool row = rw < WR && r >= 0 && r < Hp;
      la[u] = (row && c >= 0 && c < Wp) ? member[(size_t)r * Wp + c] : none;
      lb[u] = (row && lane < NP - 64 && c2 >= 0 && c2 < Wp) ? member[(size_t)r * Wp + c2] : none;
    }
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
      const int rw = wave + 4 * u;
      const uint64_t A = __ballot(la[u] != none), B = __ballot(lb[u] != none);
      if (rw < WR && lane == 0) {
        mlo[rw] = A;
        mhi[rw] = B;
      }
    }
  }
  __syncthreads();
  if (wave == 0) {
    const int c0 = lane < WR ? __popcll(mlo[lane]) + __popcll(mhi[lane]) : 0;
    const int c1 = lane + 64 < WR ? __popcll(mlo[lane + 64]) + __popcll(mhi[lane + 64]) : 0;
    int s0 = c0, s1 = c1;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v0 = __shfl_up(s0, off), v1 = __shfl_up(s1, off);
      if (lane >= off) {
        s0 += v0;
        s1 += v1;
      }
    }
    const int t0 = __shfl(s0, 63), t1 = __shfl(s1, 63);
    if (lane < WR) rbase[lane] = s0 - c0;
    if (lane + 64 < WR) rbase[lane + 64] = t0 + s1 - c1;
    if (lane == 0) rbase[WR] = t0 + t1;
  }
  __syncthreads();
  for (int rw = wave; rw < WR; rw += 4) {
    const uint64_t A = mlo[rw], B = mhi[rw];
    const uint64_t below = (1ull << lane) - 1ull;
    if ((A >> lane) & 1ull) plist[rbase[rw] + __popcll(A & below)] = (int16_t)(rw * NP + lane);
    if (lane < NP - 64 && ((B >> lane) & 1ull))
      plist[rbase[rw] + __popcll(A) + __popcll(B & below)] = (int16_t)(rw * NP + 64 + lane);
  }
  const int n = rbase[WR];
  __syncthreads();

  // 3. per window row the thread touches (u = 0 .. 4 NR + 3: row j + u),
  // its 8-bit field at columns tx .. tx + 7 and the slot of its first bit
  float acc[NR], cnt[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) acc[i] = cnt[i] = 0.f;
  const int xx = x0 + tx;
  for (int c0 = 0; c0 < n; c0 += CH) {
    const int m = min(CH, n - c0);
    // 2. stage slots c0 .. c0 + m - 1 (clamped loads, all in flight)
    float4 v[SPT];
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int q = min(e >> 4, m - 1), f = e & 15;
      const int w = plist[c0 + q];
      const int r = rfirst + w / NP, c = cfirst + w % NP;
      v[u] = *reinterpret_cast<const float4*>(Zhat + ((size_t)r * Wp + c) * kP + 4 * f);
    }
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const int e = threadIdx.x + 256 * u;
      if ((e >> 4) < m) {
        float* zp = zs + (e >> 4) * PITCH + 4 * (e & 15);
        zp[0] = v[u].x;
        zp[1] = v[u].y;
        zp[2] = v[u].z;
        zp[3] = v[u].w;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4 * NR + 4; ++u) {
      const int rw = j + u;  // < 4 NR + 7 = WR
      const uint64_t A = mlo[rw], B = mhi[rw];
      // bits tx .. tx + 7 of the row's 71-bit mask
      const uint32_t f8 =
          (uint32_t)((tx + 8 <= 64 ? (A >> tx) : ((A >> tx) | (B << (64 - tx)))) & 0xffull);
      if (c0 == 0) {
        const float pc = (float)__popc(f8);
        if (u / 4 < NR) cnt[u / 4] += pc;
        if (u / 4 >= 1 && u / 4 - 1 < NR) cnt[u / 4 - 1] += pc;
      }
      if (!f8) continue;
      int sl = rbase[rw] + __popcll(A & ((1ull << tx) - 1ull)) - c0;
      uint32_t bits = f8;
      while (bits) {
        const int k = __ffs(bits) - 1;  // window column tx + k: dx = 7 - k
        bits &= bits - 1u;
        if (sl >= 0 && sl < m) {
          const float* zp = zs + sl * PITCH + (7 - k);
          // pixel row i = u / 4 (dy = 7 - u % 4) and i = u / 4 - 1 (dy = 3 - u % 4)
          if (u / 4 < NR) acc[u / 4] += zp[8 * (7 - u % 4)];
          if (u / 4 >= 1 && u / 4 - 1 < NR) acc[u / 4 - 1] += zp[8 * (3 - u % 4)];
        }
        ++sl;
      }
    }
    __syncthreads();  // zs is restaged
  }

  // 4. average and image update
  const float onepb = 1.f + b;
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int yy = y0 + j + 4 * i;
    if (yy < H && xx < W) {
      const size_t o = (size_t)yy * W + xx;
      const float xt = acc[i] / cnt[i];
      xnew[o] = raw ? xt : (yv[i] + b * xt) / onepb;
    }
  }
}

template <bool SUB>
static void launch_ola_rows(const Batch& b, int blocks, const float* Zhat, const float* y,
                            const float* bvals, int t, float* xnew, const int32_t* member,
                            int none, int raw, const JitterDraw* draw, hipStream_t st) {
  if (SUB) {
    // 16-row parts of every planned tile (the planned heights are 16, 32, 64),
    // then the drawing's workgroups
    const int parts = ((int)(((int64_t)b.n_ola * (b.ola_rows / 16) + 7) & ~7));
    int dblocks = 0;
    JitterDraw a;
    if (draw) {
      a = *draw;
      dblocks = (a.amax * a.cmax + 255) / 256;
    }
    hipLaunchKernelGGL(ola_subset_kernel<16>, dim3(parts + dblocks), dim3(256), 0, st, b, Zhat, y,
                       bvals, t, xnew, member, none, raw, parts, a, dblocks);
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
                            const float* bvals, int t, float* xnew, const int32_t* member,
                            int none, int raw, const JitterDraw* draw, hipStream_t st) {
  const int blocks = (b.n_ola + 7) & ~7;  // whole rounds over the 8 XCDs
  if (draw && !member) return hipErrorInvalidValue;
  if (member)
    launch_ola_rows<true>(b, blocks, Zhat, y, bvals, t, xnew, member, none, raw, draw, st);
  else
    launch_ola_rows<false>(b, blocks, Zhat, y, bvals, t, xnew, nullptr, none, raw, nullptr, st);
  return hipGetLastError();
}

}  // namespace fepll
