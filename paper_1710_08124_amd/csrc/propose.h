// Internal declarations of the proposal path (bfloat16 selection modes and
// the fused network inference).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace fepll {

enum { kModeSpatialFull = 0, kModeListFull = 2, kModeListBatch = 3 };

struct BF16Args {
  // spatial all-K mode: x, Ub, L, labels, best, second are the packed
  // buffers / all-slot tables of a batch (see ImgDesc); other modes: one
  // image and the tables of one beta
  const float* x;         // current image, H x W contiguous
  int H, W;
  const uint16_t* Ub;     // bfloat16 operand table of this beta
  const float* L;         // L_k of this beta
  int K;
  int32_t* labels;        // Np
  float* best;            // Np or NULL
  float* second;          // Np or NULL
  const int32_t* list_count;  // list mode: list length (device)
  const int32_t* list;        // list mode: patch indices
  const ImgDesc* d;           // spatial all-K mode: the batch
  const int32_t* est_img;     // spatial all-K mode: image of each tile
  int n_est;                  // spatial all-K mode: tiles of the batch
  int t;                      // spatial all-K mode: iteration (slot0 + t)
  int blocks;                 // spatial all-K mode: workgroups (0 = one per tile)
  // flat-tail form (Sec. 3.1), or NULL: kept ranks per component, and 1/nu_P
  // per component (all-slot table in the spatial all-K mode, this beta's
  // otherwise)
  const int32_t* rk;
  const float* Pinv;
  // list mode: the patches' bfloat16 operands (8 uint4 per patch) and
  // squared norms, as written by the proposal network, or NULL (read the
  // patches from the image)
  const uint4* zop;
  const float* znz;
  // batched list mode (every image's list at list + d.np, its length
  // list_count[i]; the tables of all slots): items of 512 list entries,
  // image i's first item_pre[i], their total item_pre[n_img]; blocks is the
  // grid of the launch
  const int32_t* item_pre;
  int n_img;
  // batched list mode split over the components (ksplit >= 2): ksplit
  // workgroups per item, part p searching components [p K / ksplit,
  // (p + 1) K / ksplit) and writing, for list entry e of image d, its label
  // to part_out[p * part_stride + d.np + e], its best and second cost (float
  // bits) ksplit * part_stride and 2 ksplit * part_stride further on;
  // launch_fallback_merge then writes labels, best and second.  0 or 1: one
  // workgroup per item, outputs written directly.
  int ksplit;
  int32_t* part_out;
  size_t part_stride;
};

hipError_t launch_estep_bf16_mode(int mode, const BF16Args& args, hipStream_t st);
// The batched list mode's merge of its ksplit parts (ksplit >= 2), in
// component order: the labels, costs and second costs of one search over all
// K, bit for bit.
hipError_t launch_fallback_merge(const BF16Args& args, hipStream_t st);

// Exact rescoring of the proposal's candidates over a batch at iteration t
// (tables of all slots; one workgroup per tile of kRescPatches consecutive
// patches of one image, tile_img giving the image of each tile and
// ImgDesc::resc0 its first): every pair (patch i, candidate j < m) gets the
// bfloat16 selection cost of the all-K modes, bit for bit; per patch the best
// (ties to the lower component) and second cost, its label (0x7fffffff
// without candidates) and the fallback decision -- half the exact gap below
// margin, or fewer than two candidates -- appending the patch (local index)
// to its image's list at fb_list + d.np, fb_count[i] entries (zeroed before).
constexpr int kRescPatches = 896;
struct RescoreArgs {
  const ImgDesc* d;
  const int32_t* tile_img;
  const float* x;         // packed images
  const uint16_t* cand;   // packed, 8 per patch
  int m, K, t;
  const uint16_t* Ub;     // all slots
  const float* L;
  const int32_t* rk;      // flat tail, or NULL
  const float* Pinv;
  float margin;
  int32_t* labels;        // packed
  float* best;            // packed or NULL
  float* second;          // packed or NULL
  int32_t* fb_count;      // per image
  int32_t* fb_list;       // packed
};
hipError_t launch_rescore_batch(const RescoreArgs& a, int n_tiles, hipStream_t st);
// pre[i] = sum over images j < i of ceil(count[j] / 512), pre[n] the total:
// the items of the batched fallback search (kModeListBatch).
hipError_t launch_fallback_items(const int32_t* count, int n, int32_t* pre, hipStream_t st);

// Search-tree descent (Sec. 3.2): every patch's bfloat16 operand record and
// squared norm (as the network writes them).
hipError_t launch_records_bf16(const float* x, int H, int W, uint16_t* zop, float* znz,
                               hipStream_t st);
// One level of the descent from the current nodes cur to their best
// children (labels; may alias cur: cur is consumed first), with the pair
// sort's scratch (cand: 8 uint16 per patch; hist, seg, sorted) grouping the
// patches by node; records zop / znz as launch_records_bf16 writes them.
hipError_t launch_tree_level_bf16(const int32_t* cur, int Np, const uint16_t* zop,
                                  const float* znz, const uint16_t* Ub_t, const float* L32_t,
                                  const int32_t* rk, const float* Pinv_t, int K,
                                  const uint16_t* children, uint16_t* cand, int32_t* hist,
                                  int32_t* seg, int32_t* sorted, int32_t* labels, float* best,
                                  float* second, hipStream_t st);

// The top levels of the descent in one pass over the image: positions
// 0..n-1 list the nodes of those levels in order (node: node id, par: its
// parent's id, lend: the end position of each of the nlev levels); every
// patch starts at root, scores each node whose parent is its current node
// (the bfloat16 selection cost of the tree tables Ub / L / rk / Pinv of one
// beta, indexed by node id) and moves to the best at each level's end.
// labels: the node reached; best / second (or NULL): the last level's; zop /
// znz (or NULL): the patches' operand records, as launch_records_bf16 writes
// them.
struct TreeDenseArgs {
  const float* x;
  int H, W;
  const uint16_t* Ub;
  const float* L;
  const int32_t* rk;  // NULL: plain form
  const float* Pinv;
  const int32_t* node;
  const int32_t* par;
  const int32_t* lend;
  int n, nlev, root;
  int32_t* labels;
  float* best;
  float* second;
  uint4* zop;
  float* znz;
};
hipError_t launch_tree_dense_bf16(const TreeDenseArgs& a, hipStream_t st);

// Network inference + top-m over selection tiles (4 patch rows x kEstCols
// columns, two workgroups each): one image (d NULL: x, H, W, logsb, cand
// indexed by the image's patch) or a planned batch at iteration t (d,
// est_img, n_est; log sigma_beta of each image from logsb_slot[d.slot0 + t];
// cand packed like the labels).  cand gets, for every patch, its m best
// classes in decreasing logit order (ties to the lower class), 0xffff after
// the m-th.  Wb / bias: see propose.hip.
struct ProposeArgs {
  const float* x;
  int H, W;
  float logsb;
  const ImgDesc* d;
  const int32_t* est_img;
  int n_est;
  const float* logsb_slot;
  int t;
  const uint16_t* Wb;
  const float* bias;
  int K, m;
  uint16_t* cand;
  // n_zero int32 set to 0 by the launch before any later kernel runs (the
  // rescoring's per-image fallback counts), or NULL
  int32_t* zero;
  int n_zero;
};
hipError_t launch_propose(const ProposeArgs& a, hipStream_t st);

// Host-side packing of float32 parameters into the inference layouts.
// Returns the number of uint16 entries of Wb and fills wb / bias.
void pack_proposal(const float* params, int K, uint16_t* wb, float* bias);
size_t proposal_wb_count(int K);
size_t proposal_bias_count(int K);

}  // namespace fepll
