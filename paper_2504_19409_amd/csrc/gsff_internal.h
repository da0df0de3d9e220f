// Internal declarations shared by the HIP translation units of libgsff:
// workspace layout, device-side views, and the host launchers each .hip file
// provides to the C ABI in capi.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsff.h"

namespace gsff {

constexpr int kTile = GSFF_TILE;           // 16x16 pixel screen tiles
constexpr int kBlock = kTile * kTile;      // one thread per pixel of a tile
constexpr int kRadixIpt = 16;              // keys per lane in a pair-sort radix chunk
constexpr int kRadixChunk = 64 * kRadixIpt;  // keys per wave chunk (pair sort)
constexpr int kSortIptMax = 16;            // depth sort: most keys per lane
// Depth sort keys per lane (4, 8 or 16; a workgroup sorts 256 times as many):
// the fewest that keep the chunks to about 256, so that small frames get
// many short chunks and large ones no more chunks than the chip holds.
inline int sort_ipt_for(int64_t P) {
  return P <= 256 * 256 * 4 ? 4 : (P <= 256 * 256 * 8 ? 8 : kSortIptMax);
}
constexpr int kSortHistBlocks = 64;        // workgroups of the 4-digit histogram
constexpr int kSortLbGroup = 8;            // depth sort: chunks per look-back group
constexpr uint32_t kSortWaitPolls = 2048;  // depth sort: polls before a workgroup counts itself
constexpr int kScanBlock = 1024;           // elements per block in the count scan
constexpr int kPoseBlock = 256;            // Gaussians per preprocess-adjoint block
constexpr int kMaxDirectTiles = 4096;      // tile grids binned without a pair sort
constexpr int kBinBands = 2;               // tile-row bands of the direct scatter
constexpr int kSuper = GSFF_SUPER;         // bin-grid cell: kSuper x kSuper tiles (16-bit masks)
static_assert(kSuper == 4, "pair masks are 16 bits");
constexpr int kBinBlock = 256;             // depth ranks per direct-binning block
constexpr int kSegBatches = 4;             // adjoint segment: batches of 16 walked entries
constexpr int kSegLen = 16 * kSegBatches;  // walked-list entries per adjoint segment
constexpr int kMaxSeg = 8;                 // adjoint segments per tile (the last one takes the rest)

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// ---- checked build --------------------------------------------------------
// Compiled with -DGSFF_CHECKED=1 (libgsff_checked.so), the kernels test every
// index that comes from data (a sort destination, a listed id, a tile range,
// an adjoint row or slot) against what it addresses.  A failed test skips the
// access, raises GSFF_FLAG_CHECK, counts the failure and records the first
// one (site, index, limit) in the status words below.  `guard` tests in both
// builds (the release build needs the test for well-formed inputs too);
// GSFF_CHECK tests only in the checked build (the release build relies on the
// index being in range by construction).
#ifndef GSFF_CHECKED
#define GSFF_CHECKED 0
#endif
constexpr int kStatusChkSite = 4, kStatusChkIndex = 5, kStatusChkLimit = 6, kStatusChkCount = 7;

__device__ __forceinline__ void check_failed(uint32_t* status, uint32_t site, uint64_t idx,
                                             uint64_t lim) {
  atomicOr(&status[0], GSFF_FLAG_CHECK);
  if (atomicAdd(&status[kStatusChkCount], 1u) == 0u) {
    status[kStatusChkSite] = site;
    status[kStatusChkIndex] = (uint32_t)(idx < 0xFFFFFFFFull ? idx : 0xFFFFFFFFull);
    status[kStatusChkLimit] = (uint32_t)(lim < 0xFFFFFFFFull ? lim : 0xFFFFFFFFull);
  }
}

// (the comparison is made in the operands' own types, as unchecked code would)
template <typename I, typename L>
__device__ __forceinline__ bool guard(uint32_t* status, uint32_t site, I idx, L lim) {
  const bool ok = idx < lim;
#if GSFF_CHECKED
  if (!ok) check_failed(status, site, (uint64_t)idx, (uint64_t)lim);
#else
  (void)status;
  (void)site;
#endif
  return ok;
}

// (a macro: the release build evaluates none of the arguments)
#define GSFF_CHECK(status, site, idx, lim) \
  (!GSFF_CHECKED || ::gsff::guard((status), (site), (idx), (lim)))

inline int ceil_log2(uint64_t v) {
  int b = 0;
  while ((uint64_t(1) << b) < v) ++b;
  return b;
}

// Byte offsets of every workspace region; computed identically on the host
// for gsff_workspace_size / gsff_workspace_layout and for every launch.
struct Layout {
  int64_t P = 0, max_pairs = 0;
  int32_t C = 0;
  int64_t row_cap = 0;      // adjoint partial rows (one per walked pair)
  int32_t row_width = 0;    // floats per row: 10 image-space terms + C features
  int64_t item_cap = 0;     // adjoint reduction work items (64-row chunks)
  int64_t slot_cap = 0;     // adjoint slots: one per tile of every Gaussian's rectangle
  int32_t W = 0, H = 0, tiles_x = 0, tiles_y = 0, ntiles = 0;
  int32_t super_x = 0, super_y = 0, nsuper = 0;  // bin grid: kSuper x kSuper tiles per cell
  int32_t rank_bits = 0, tile_bits = 0;
  bool direct_bin = false;  // bin by coverage masks (else by sorting (super-tile, rank) keys)
  bool sort_fits = false;   // (super-tile, rank) keys fit 32 bits
  int64_t sort_ipt = 0;  // depth sort keys per lane (sort_ipt_for)
  int64_t sort_blocks = 0, pair_chunks = 0, scan_blocks = 0, pose_blocks = 0, bin_blocks = 0;
  uint64_t status = 0, records = 0, rects = 0, pmask = 0, clist = 0, crange = 0, dkeys_a = 0, dkeys_b = 0, dids_a = 0,
           dids_b = 0, offsets = 0, pkeys_a = 0, pkeys_b = 0, tile_ranges = 0, pix_T = 0,
           pix_end = 0, grad2d = 0, hist = 0, hist_tot = 0, scan_part = 0, pose_part = 0,
           binhist = 0, tile_tot = 0, curbase = 0, rows = 0, tile_walk = 0, walk_off = 0,
           slot_local = 0, slot_cnt = 0, slot_blk = 0, nslot = 0, slots = 0, item_n = 0, items = 0,
           seg_order = 0, seg_n = 0, seg_state = 0, seg_final = 0, l1_codes = 0, loss_part = 0, sort_part = 0, sort_lb = 0, total = 0;
};

// Returns false if the sizes are not representable (key bits, negative sizes).
bool compute_layout(int64_t P, int32_t C, int64_t max_pairs, int32_t W, int32_t H, Layout* L);

// Device-side view of a workspace.
struct WsView {
  uint32_t* status;      // [0] flags, [1] pair count, [2] pairs in use, [4-7] checks
  float4* rec;           // [3][P]
  ushort4* rects;        // [P]
  uint32_t* dkeys_a;     // [P]  depth keys (sorted result lands here)
  uint32_t* dkeys_b;
  uint32_t* dids_a;      // [P]  Gaussian ids in depth order
  uint32_t* dids_b;
  uint32_t* offsets;     // [P+1] exclusive scan of tile counts in depth order
  uint32_t* pkeys_a;     // [max_pairs] pair keys (sorted result lands here)
  uint32_t* pkeys_b;
  uint2* tile_ranges;    // [nsuper] [start, end) of every super-tile's list in pkeys_a / pmask
  uint16_t* pmask;       // [max_pairs] tiles of the super-tile the pair's rectangle covers
                         //   (bit 4 (ty % 4) + (tx % 4))
  uint32_t* clist;       // per-tile lists the forward walked (capacity: the super-tile's
                         //   list length for each of its 16 tiles)
  uint2* crange;         // [ntiles] [start, walk end) of every tile's walked list in clist
  float* pix_T;          // [H*W]
  uint32_t* pix_end;     // [H*W]
  float* grad2d;         // [P][10]
  uint32_t* hist;        // radix chunk histograms [bins][chunks]
  uint32_t* hist_tot;    // radix digit totals [256]
  uint32_t* sort_part;   // depth sort: per-workgroup 4-digit histograms [kSortHistBlocks][4][256]
  uint32_t* sort_lb;     // depth sort look-back words [4 passes][chunks + groups][256]
  uint32_t* scan_part;   // count-scan block partials
  double* pose_part;     // [pose_blocks][6]
  uint32_t* binhist;     // direct binning: per-tile counts per rank block [ntiles][blocks]
  uint32_t* tile_tot;    // direct binning: pairs per tile [ntiles]
  uint32_t* curbase;     // direct binning: pairs of earlier blocks per tile [blocks][ntiles]
  // Adjoint partial sums: the compositing adjoint writes one row per walked
  // (tile, Gaussian) pair and files the row index in the Gaussian's slots
  // (slot range = the Gaussian's rectangle tile count, counted by nslot); the
  // adjoint reduction sums every Gaussian's rows, one work item per 64 slots.
  float* rows;           // [row_cap][row_width]
  uint32_t* tile_walk;   // [ntiles] end of the forward's walk of every tile list
  uint32_t* walk_off;    // [ntiles] first row of every tile
  uint4* seg_order;      // [ntiles * kMaxSeg] adjoint work items, longest first: tile |
                         // segment << 24 | inner << 30 | rows fit << 31, q1, q2, row base
  uint32_t* seg_n;       // [1] adjoint work items
  float* seg_state;      // [ntiles][kMaxSeg - 1][5][256] per-pixel state at the segment
                         // ends: T, then the colour and depth blended in front of the end
  float* seg_final;      // [ntiles][4][256] final colour and depth of the split tiles
  uint32_t* l1_codes;    // [1 + ceil(C / 16)][H*W] the L1 upstream in 2-bit codes
  float* loss_part;      // [ceil(H*W / 256)] the L1 loss per 256 pixels
  uint32_t* slot_local;  // [P] first slot of each Gaussian inside its 256-Gaussian block
  uint32_t* slot_cnt;    // [P/256]: slot count of each 256-Gaussian block (preprocess)
  uint32_t* slot_blk;    // [P/256]: first slot of each block (scanned by the adjoint's set-up)
  uint32_t* nslot;       // [P] slots filled per Gaussian
  uint32_t* slots;       // [slot_cap] row index per filed (tile, Gaussian) pair
  uint32_t* item_n;      // [1] work items filed
  uint2* items;          // [item_cap] (Gaussian, first slot) of every 64-slot chunk
  uint32_t row_cap;
  int32_t row_width;
  uint32_t item_cap;
  uint32_t slot_cap;
};

WsView make_view(void* ws, const Layout& L);

// Device copy of the settings with derived constants.
struct DevSettings {
  float near_plane, guard, dilation, alpha_min, alpha_max, t_min;
  int32_t render_features;
  int32_t deterministic;  // fixed-order adjoint reduction
};

struct DevCamera {
  int32_t W, H;
  float fx, fy, cx, cy;
  const float* viewmat;
};

struct DevGaussians {
  int64_t P;
  int32_t C;
  int32_t feat_dtype;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* logit;
  const float* rgb;
  const void* feat;
};

// Sets the message gsff_last_error() returns and passes the code through.
gsff_status record_error(gsff_status code, const char* msg);

// ---- host launchers (each returns the first HIP error, or hipSuccess) ----
hipError_t launch_preprocess(const DevGaussians& g, const DevCamera& cam,
                             const DevSettings& st, const Layout& L, const WsView& w,
                             hipStream_t s);
hipError_t launch_sort_depth(const Layout& L, const WsView& w, hipStream_t s);
void set_sort_wait_limit(uint32_t polls);
hipError_t launch_bin(const Layout& L, const WsView& w, hipStream_t s);
hipError_t launch_sort_tiles(const Layout& L, const WsView& w, hipStream_t s);
hipError_t launch_tile_ranges(const Layout& L, const WsView& w, hipStream_t s);
hipError_t launch_composite_fwd(const DevGaussians& g, const DevSettings& st,
                                const Layout& L, const WsView& w, float* out_rgb,
                                float* out_depth, float* out_alpha, void* out_feat,
                                int32_t out_feat_dtype, hipStream_t s);
// The adjoint's work items (tile list segments, longest first) and the first
// adjoint row of every tile, from the walks the last forward recorded.
hipError_t launch_adjoint_items(const Layout& L, const WsView& w, hipStream_t s);
hipError_t launch_visibility(const DevSettings& st, const DevGaussians& g, const Layout& L,
                             const WsView& w, float t_vis, uint8_t* visible, hipStream_t s);
hipError_t launch_covisibility(const uint8_t* a, const uint8_t* b, int64_t n, uint32_t* counts,
                               hipStream_t s);
hipError_t launch_keyframe_decide(const uint32_t* counts, float tau, uint32_t* keyframe,
                                  hipStream_t s);
hipError_t launch_composite_bwd(const DevGaussians& g, const DevSettings& st,
                                const Layout& L, const WsView& w, const float* g_rgb,
                                const float* g_depth, const float* g_alpha,
                                const float* g_feat, bool geometry, float* d_feat,
                                int32_t accumulate, hipStream_t s);
// L1-loss upstream (see gsff_backward_l1): forward outputs, targets (NULL =
// group not in the loss), group weights, and an optional loss accumulator.
struct L1Args {
  const float *out_rgb, *out_depth, *out_alpha, *out_feat;
  const float *t_rgb, *t_depth, *t_alpha, *t_feat;
  double w_rgb, w_depth, w_alpha, w_feat;
  float* loss;
  // per-pixel masks of the tracking loss (NULL: every pixel): mask_v gates
  // the colour and depth terms, mask_e the colour term
  const uint8_t* mask_v = nullptr;
  const uint8_t* mask_e = nullptr;
};
hipError_t launch_composite_bwd_l1(const DevGaussians& g, const DevSettings& st,
                                   const Layout& L, const WsView& w, const L1Args& a,
                                   bool geometry, float* d_feat, int32_t accumulate,
                                   hipStream_t s);
hipError_t launch_preprocess_bwd(const DevGaussians& g, const DevCamera& cam,
                                 const DevSettings& st, const Layout& L, const WsView& w,
                                 const gsff_grads& out, int32_t accumulate, hipStream_t s);
hipError_t launch_l1_grad(const float* x, const float* y, int64_t n, float scale,
                          float* grad, float* loss, hipStream_t s);

}  // namespace gsff
