// Host side of the C ABI declared in include/gsff.h: argument checks,
// workspace layout, and the launch sequence of every stage.  No allocation,
// no host/device synchronisation (except gsff_read_status).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "gsff_internal.h"

namespace gsff {

static thread_local std::string g_last_error;

static gsff_status fail(gsff_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

gsff_status record_error(gsff_status code, const char* msg) { return fail(code, msg); }

static gsff_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return GSFF_OK;
  return fail(GSFF_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool compute_layout(int64_t P, int32_t C, int64_t max_pairs, int32_t W, int32_t H, Layout* L) {
  if (P < 0 || C < 0 || C > 4096 || max_pairs < 0 || W <= 0 || H <= 0) return false;
  // the depth sort's look-back words carry 30-bit counts
  if (P >= ((int64_t)1 << 30) || max_pairs > (int64_t)0xFFFFFFFEu) return false;
  Layout l;
  l.C = C;
  l.P = P;
  l.max_pairs = max_pairs;
  l.W = W;
  l.H = H;
  l.tiles_x = (W + kTile - 1) / kTile;
  l.tiles_y = (H + kTile - 1) / kTile;
  if (l.tiles_x > 65535 || l.tiles_y > 65535) return false;
  l.ntiles = l.tiles_x * l.tiles_y;
  l.super_x = (l.tiles_x + kSuper - 1) / kSuper;
  l.super_y = (l.tiles_y + kSuper - 1) / kSuper;
  l.nsuper = l.super_x * l.super_y;
  l.rank_bits = ceil_log2((uint64_t)(P < 2 ? 2 : P));
  l.tile_bits = ceil_log2((uint64_t)l.nsuper);
  // direct binning keeps per-wave cursors (16 B per super-tile), the tiles'
  // first pairs (4 B per super-tile) and coverage masks (32 B per super-tile
  // column and row) of a block in 64 KiB of LDS
  l.direct_bin = l.nsuper <= kMaxDirectTiles &&
                 20ll * l.nsuper + 32ll * (l.super_x + l.super_y) <= 65536 - 64;
  // the fallback path packs (super-tile, rank) into 32-bit keys
  l.sort_fits = l.rank_bits + l.tile_bits <= 32;
  if (!l.direct_bin && !l.sort_fits) return false;
  l.sort_ipt = sort_ipt_for(P);
  l.sort_blocks = (P + 256 * l.sort_ipt - 1) / (256 * l.sort_ipt);
  l.pair_chunks = (max_pairs + kRadixChunk - 1) / kRadixChunk;
  l.scan_blocks = (P + kScanBlock - 1) / kScanBlock;
  l.pose_blocks = (P + kPoseBlock - 1) / kPoseBlock;
  l.bin_blocks = (P + kBinBlock - 1) / kBinBlock;
  const uint64_t HW = (uint64_t)W * H;
  const uint64_t A = 256;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o = align_up(o + bytes, A);
    return at;
  };
  l.status = take(32);
  l.records = take(48ull * P);
  l.rects = take(8ull * P);
  l.dkeys_a = take(4ull * P);
  l.dkeys_b = take(4ull * P);
  l.dids_a = take(4ull * P);
  l.dids_b = take(4ull * P);
  l.offsets = take(4ull * (P + 1));
  l.pkeys_a = take(4ull * max_pairs);
  l.pkeys_b = take(l.sort_fits ? 4ull * max_pairs : 0ull);  // key-sort binning (bin_mode 1 or large grids)
  l.pmask = take(2ull * max_pairs);
  l.tile_ranges = take(8ull * l.nsuper);
  l.clist = take(4ull * kSuper * kSuper * (uint64_t)max_pairs);
  l.crange = take(8ull * l.ntiles);
  l.pix_T = take(4ull * HW);
  l.pix_end = take(4ull * HW);
  l.grad2d = take(40ull * P);
  // radix histograms of the (tile, rank) pair sort (larger tile grids only)
  const int64_t chunks = !l.sort_fits ? 1 : (l.pair_chunks > 0 ? l.pair_chunks : 1);
  l.hist = take(4ull * 256 * (uint64_t)chunks);
  l.hist_tot = take(4ull * 256);
  l.sort_part = take(4ull * kSortHistBlocks * 1024);
  {  // per pass: a word per digit for every chunk and every group of kSortLbGroup chunks
    const uint64_t ch = (uint64_t)(l.sort_blocks > 0 ? l.sort_blocks : 1);
    l.sort_lb = take(4ull * 4 * 256 * (ch + (ch + kSortLbGroup - 1) / kSortLbGroup));
  }
  l.scan_part = take(4ull * (uint64_t)(l.scan_blocks + 1));
  l.pose_part = take(8ull * 6 * (uint64_t)(l.pose_blocks + 1));
  l.binhist = take(l.direct_bin ? 4ull * l.nsuper * (uint64_t)l.bin_blocks : 0ull);
  l.tile_tot = take(l.direct_bin ? 4ull * l.nsuper : 0ull);
  l.curbase = take(l.direct_bin ? 4ull * l.nsuper * (uint64_t)l.bin_blocks : 0ull);
  // adjoint partial rows: room for two walked pairs per Gaussian (a tile whose
  // rows do not fit falls back to atomic accumulation)
  l.row_width = 10 + C;
  l.row_cap = 2 * P + 4096;
  if (l.row_cap > kSuper * kSuper * max_pairs + 4096) l.row_cap = kSuper * kSuper * max_pairs + 4096;
  if (l.row_cap > 0xFFFFFFFFll) l.row_cap = 0xFFFFFFFFll;  // 32-bit row indices
  l.rows = take(4ull * (uint64_t)l.row_cap * (uint64_t)l.row_width);
  l.tile_walk = take(4ull * l.ntiles);
  l.walk_off = take(4ull * l.ntiles);
  l.seg_order = take(16ull * l.ntiles * kMaxSeg);
  l.seg_n = take(4);
  l.seg_state = take(4ull * l.ntiles * (kMaxSeg - 1) * 5 * kBlock);
  l.seg_final = take(4ull * l.ntiles * 4 * kBlock);
  l.l1_codes = take(4ull * (1 + (C + 15) / 16) * HW);
  l.loss_part = take(4ull * ((HW + 255) / 256));
  l.slot_local = take(4ull * P);
  l.slot_cnt = take(4ull * (uint64_t)(l.pose_blocks + 1));
  l.slot_blk = take(4ull * (uint64_t)(l.pose_blocks + 1));
  l.nslot = take(4ull * P);
  // slots: a Gaussian's range is its rectangle's tile count, so all of them
  // together are the tile pairs: at most kSuper^2 per super-tile pair
  l.slot_cap = (int64_t)kSuper * kSuper * max_pairs;
  if (l.slot_cap > 0xFFFFFFFFll) l.slot_cap = 0xFFFFFFFFll;
  l.slots = take(4ull * (uint64_t)l.slot_cap);
  // a work item per Gaussian with rows, plus one per further full 64 rows
  l.item_cap = P + l.row_cap / 64 + 1;
  if (l.item_cap > 0xFFFFFFFFll) l.item_cap = 0xFFFFFFFFll;
  l.item_n = take(4ull);
  l.items = take(8ull * (uint64_t)l.item_cap);

  l.total = o;
  *L = l;
  return true;
}

WsView make_view(void* ws, const Layout& L) {
  char* b = (char*)ws;
  WsView w;
  w.status = (uint32_t*)(b + L.status);
  w.rec = (float4*)(b + L.records);
  w.rects = (ushort4*)(b + L.rects);
  w.dkeys_a = (uint32_t*)(b + L.dkeys_a);
  w.dkeys_b = (uint32_t*)(b + L.dkeys_b);
  w.dids_a = (uint32_t*)(b + L.dids_a);
  w.dids_b = (uint32_t*)(b + L.dids_b);
  w.offsets = (uint32_t*)(b + L.offsets);
  w.pkeys_a = (uint32_t*)(b + L.pkeys_a);
  w.pkeys_b = (uint32_t*)(b + L.pkeys_b);
  w.tile_ranges = (uint2*)(b + L.tile_ranges);
  w.pmask = (uint16_t*)(b + L.pmask);
  w.clist = (uint32_t*)(b + L.clist);
  w.crange = (uint2*)(b + L.crange);
  w.pix_T = (float*)(b + L.pix_T);
  w.pix_end = (uint32_t*)(b + L.pix_end);
  w.grad2d = (float*)(b + L.grad2d);
  w.hist = (uint32_t*)(b + L.hist);
  w.hist_tot = (uint32_t*)(b + L.hist_tot);
  w.sort_part = (uint32_t*)(b + L.sort_part);
  w.sort_lb = (uint32_t*)(b + L.sort_lb);
  w.scan_part = (uint32_t*)(b + L.scan_part);
  w.pose_part = (double*)(b + L.pose_part);
  w.binhist = (uint32_t*)(b + L.binhist);
  w.tile_tot = (uint32_t*)(b + L.tile_tot);
  w.curbase = (uint32_t*)(b + L.curbase);
  w.rows = (float*)(b + L.rows);
  w.tile_walk = (uint32_t*)(b + L.tile_walk);
  w.walk_off = (uint32_t*)(b + L.walk_off);
  w.slot_local = (uint32_t*)(b + L.slot_local);
  w.slot_cnt = (uint32_t*)(b + L.slot_cnt);
  w.slot_blk = (uint32_t*)(b + L.slot_blk);
  w.nslot = (uint32_t*)(b + L.nslot);
  w.slots = (uint32_t*)(b + L.slots);
  w.seg_order = (uint4*)(b + L.seg_order);
  w.seg_n = (uint32_t*)(b + L.seg_n);
  w.seg_state = (float*)(b + L.seg_state);
  w.seg_final = (float*)(b + L.seg_final);
  w.l1_codes = (uint32_t*)(b + L.l1_codes);
  w.loss_part = (float*)(b + L.loss_part);
  w.item_n = (uint32_t*)(b + L.item_n);
  w.items = (uint2*)(b + L.items);
  w.row_cap = (uint32_t)L.row_cap;
  w.row_width = L.row_width;
  w.item_cap = (uint32_t)L.item_cap;
  w.slot_cap = (uint32_t)L.slot_cap;
  return w;
}

namespace {

struct Ctx {
  Layout L;
  WsView w;
  DevGaussians g;
  DevCamera cam;
  DevSettings st;
  hipStream_t s;
};

gsff_status check_common(const gsff_gaussians* g, const gsff_camera* cam, const gsff_settings* st,
                         void* ws, size_t ws_bytes, int64_t max_pairs, void* stream, Ctx* c) {
  if (!g || !cam || !st) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL gaussians/camera/settings");
  if (g->P < 0) return fail(GSFF_ERR_INVALID_ARGUMENT, "P < 0");
  if (g->C < 0 || g->C > 4096) return fail(GSFF_ERR_INVALID_ARGUMENT, "C out of range [0, 4096]");
  if (g->feat_dtype != GSFF_DTYPE_F32 && g->feat_dtype != GSFF_DTYPE_BF16 &&
      g->feat_dtype != GSFF_DTYPE_F16)
    return fail(GSFF_ERR_UNSUPPORTED, "feature dtype");
  if (g->P > 0 && (!g->means || !g->log_scales || !g->quats || !g->logit_opacity || !g->rgb))
    return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL Gaussian parameter pointer");
  if (g->P > 0 && g->C > 0 && !g->feat)
    return fail(GSFF_ERR_INVALID_ARGUMENT, "C > 0 but feat is NULL");
  if (cam->width <= 0 || cam->height <= 0) return fail(GSFF_ERR_INVALID_ARGUMENT, "image size");
  if (!(cam->fx > 0.f) || !(cam->fy > 0.f) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy))
    return fail(GSFF_ERR_INVALID_ARGUMENT, "intrinsics");
  if (!cam->viewmat) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL viewmat");
  if (!(st->alpha_min > 0.f) || !(st->alpha_max <= 1.f) || !(st->alpha_min < st->alpha_max) ||
      !(st->t_min > 0.f) || !(st->t_min < 1.f) || !(st->dilation >= 0.f) || !(st->guard > 0.f) ||
      !std::isfinite(st->near_plane))
    return fail(GSFF_ERR_INVALID_ARGUMENT, "settings out of range");
  if (!ws) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL workspace");
  if (((uintptr_t)ws & 255u) != 0) return fail(GSFF_ERR_INVALID_ARGUMENT, "workspace not 256-byte aligned");
  if (!compute_layout(g->P, g->C, max_pairs, cam->width, cam->height, &c->L))
    return fail(GSFF_ERR_INVALID_ARGUMENT,
                "sizes not representable (P, max_pairs, image, or rank+tile bits > 32)");
  if (ws_bytes < c->L.total) return fail(GSFF_ERR_INVALID_ARGUMENT, "workspace too small");
  c->w = make_view(ws, c->L);
  c->g = DevGaussians{g->P, g->C, g->feat_dtype, g->means, g->log_scales, g->quats,
                      g->logit_opacity, g->rgb, g->feat};
  c->cam = DevCamera{cam->width, cam->height, cam->fx, cam->fy, cam->cx, cam->cy, cam->viewmat};
  if (st->bin_mode != 0 && st->bin_mode != 1)
    return fail(GSFF_ERR_INVALID_ARGUMENT, "bin_mode must be 0 or 1");
  if (st->bin_mode == 1) {
    if (!c->L.sort_fits)
      return fail(GSFF_ERR_INVALID_ARGUMENT, "bin_mode 1: rank + super-tile bits exceed 32");
    c->L.direct_bin = false;
  }
  if (st->deterministic != 0 && st->deterministic != 1)
    return fail(GSFF_ERR_INVALID_ARGUMENT, "deterministic must be 0 or 1");
  c->st = DevSettings{st->near_plane, st->guard, st->dilation,        st->alpha_min,
                      st->alpha_max,  st->t_min,   st->render_features ? 1 : 0,
                      st->deterministic};
  c->s = (hipStream_t)stream;
  return GSFF_OK;
}

gsff_status check_outputs(const Ctx& c, float* out_rgb, float* out_depth, float* out_alpha,
                          void* out_feat, int32_t out_feat_dtype) {
  if (!out_rgb || !out_depth || !out_alpha) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL output image");
  if (out_feat_dtype != GSFF_DTYPE_F32 && out_feat_dtype != GSFF_DTYPE_BF16)
    return fail(GSFF_ERR_UNSUPPORTED, "output feature dtype");
  if (c.st.render_features && c.g.C > 0 && !out_feat)
    return fail(GSFF_ERR_INVALID_ARGUMENT, "features on but out_feat is NULL");
  return GSFF_OK;
}

bool any_geometry(const gsff_grads* o) {
  return o->means || o->log_scales || o->quats || o->logit_opacity || o->rgb || o->pose;
}

}  // namespace
}  // namespace gsff

using namespace gsff;

extern "C" {

gsff_status gsff_version(int32_t* major, int32_t* minor) {
  if (!major || !minor) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL version pointer");
  *major = 0;
  *minor = 1;
  return GSFF_OK;
}

gsff_status gsff_is_checked_build(int32_t* checked) {
  if (!checked) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL output");
  *checked = GSFF_CHECKED ? 1 : 0;
  return GSFF_OK;
}

gsff_status gsff_set_sort_wait_limit(uint32_t polls) {
  set_sort_wait_limit(polls);
  return GSFF_OK;
}

const char* gsff_last_error(void) { return g_last_error.c_str(); }

gsff_status gsff_default_settings(gsff_settings* st) {
  if (!st) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL settings");
  st->near_plane = 0.2f;
  st->guard = 1.3f;
  st->dilation = 0.3f;
  st->alpha_min = 1.0f / 255.0f;
  st->alpha_max = 0.99f;
  st->t_min = 1e-4f;
  st->render_features = 1;
  st->bin_mode = 0;
  st->deterministic = 0;
  return GSFF_OK;
}

gsff_status gsff_workspace_size(int64_t P, int32_t channels, int64_t max_pairs, int32_t width,
                                int32_t height, size_t* bytes) {
  if (!bytes) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL bytes");
  Layout L;
  if (!compute_layout(P, channels, max_pairs, width, height, &L))
    return fail(GSFF_ERR_INVALID_ARGUMENT, "sizes not representable");
  *bytes = (size_t)L.total;
  return GSFF_OK;
}

gsff_status gsff_workspace_layout(int64_t P, int32_t channels, int64_t max_pairs, int32_t width,
                                  int32_t height, gsff_ws_layout* out) {
  if (!out) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL layout");
  Layout L;
  if (!compute_layout(P, channels, max_pairs, width, height, &L))
    return fail(GSFF_ERR_INVALID_ARGUMENT, "sizes not representable");
  out->status = L.status;
  out->records = L.records;
  out->rects = L.rects;
  out->depth_keys = L.dkeys_a;
  out->depth_ids = L.dids_a;
  out->pair_keys = L.pkeys_a;
  out->pair_masks = L.pmask;
  out->tile_ranges = L.tile_ranges;
  out->tile_lists = L.clist;
  out->tile_list_ranges = L.crange;
  out->pix_T = L.pix_T;
  out->pix_end = L.pix_end;
  out->grad2d = L.grad2d;
  out->total_bytes = L.total;
  out->rank_bits = L.rank_bits;
  out->tiles_x = L.tiles_x;
  out->tiles_y = L.tiles_y;
  out->super_x = L.super_x;
  out->super_y = L.super_y;
  return GSFF_OK;
}

#define GSFF_PRELUDE                                                                \
  Ctx c;                                                                            \
  {                                                                                 \
    gsff_status rc_ = check_common(g, cam, st, ws, ws_bytes, max_pairs, stream, &c); \
    if (rc_ != GSFF_OK) return rc_;                                                 \
  }

gsff_status gsff_preprocess(const gsff_gaussians* g, const gsff_camera* cam,
                            const gsff_settings* st, void* ws, size_t ws_bytes,
                            int64_t max_pairs, void* stream) {
  GSFF_PRELUDE
  return hip_check(launch_preprocess(c.g, c.cam, c.st, c.L, c.w, c.s), "preprocess");
}

gsff_status gsff_sort_depth(const gsff_gaussians* g, const gsff_camera* cam,
                            const gsff_settings* st, void* ws, size_t ws_bytes,
                            int64_t max_pairs, void* stream) {
  GSFF_PRELUDE
  return hip_check(launch_sort_depth(c.L, c.w, c.s), "sort_depth");
}

gsff_status gsff_bin(const gsff_gaussians* g, const gsff_camera* cam, const gsff_settings* st,
                     void* ws, size_t ws_bytes, int64_t max_pairs, void* stream) {
  GSFF_PRELUDE
  return hip_check(launch_bin(c.L, c.w, c.s), "bin");
}

gsff_status gsff_sort_tiles(const gsff_gaussians* g, const gsff_camera* cam,
                            const gsff_settings* st, void* ws, size_t ws_bytes,
                            int64_t max_pairs, void* stream) {
  GSFF_PRELUDE
  return hip_check(launch_sort_tiles(c.L, c.w, c.s), "sort_tiles");
}

gsff_status gsff_tile_ranges(const gsff_gaussians* g, const gsff_camera* cam,
                             const gsff_settings* st, void* ws, size_t ws_bytes,
                             int64_t max_pairs, void* stream) {
  GSFF_PRELUDE
  return hip_check(launch_tile_ranges(c.L, c.w, c.s), "tile_ranges");
}

gsff_status gsff_composite_fwd(const gsff_gaussians* g, const gsff_camera* cam,
                               const gsff_settings* st, void* ws, size_t ws_bytes,
                               int64_t max_pairs, float* out_rgb, float* out_depth,
                               float* out_alpha, void* out_feat, int32_t out_feat_dtype,
                               void* stream) {
  GSFF_PRELUDE
  gsff_status rc = check_outputs(c, out_rgb, out_depth, out_alpha, out_feat, out_feat_dtype);
  if (rc != GSFF_OK) return rc;
  return hip_check(launch_composite_fwd(c.g, c.st, c.L, c.w, out_rgb, out_depth, out_alpha,
                                        out_feat, out_feat_dtype, c.s),
                   "composite_fwd");
}

gsff_status gsff_forward(const gsff_gaussians* g, const gsff_camera* cam, const gsff_settings* st,
                         void* ws, size_t ws_bytes, int64_t max_pairs, float* out_rgb,
                         float* out_depth, float* out_alpha, void* out_feat,
                         int32_t out_feat_dtype, void* stream) {
  GSFF_PRELUDE
  gsff_status rc = check_outputs(c, out_rgb, out_depth, out_alpha, out_feat, out_feat_dtype);
  if (rc != GSFF_OK) return rc;
  if ((rc = hip_check(launch_preprocess(c.g, c.cam, c.st, c.L, c.w, c.s), "preprocess")) != GSFF_OK)
    return rc;
  if ((rc = hip_check(launch_sort_depth(c.L, c.w, c.s), "sort_depth")) != GSFF_OK) return rc;
  if ((rc = hip_check(launch_bin(c.L, c.w, c.s), "bin")) != GSFF_OK) return rc;
  if ((rc = hip_check(launch_sort_tiles(c.L, c.w, c.s), "sort_tiles")) != GSFF_OK) return rc;
  if ((rc = hip_check(launch_tile_ranges(c.L, c.w, c.s), "tile_ranges")) != GSFF_OK) return rc;
  return hip_check(launch_composite_fwd(c.g, c.st, c.L, c.w, out_rgb, out_depth, out_alpha,
                                        out_feat, out_feat_dtype, c.s),
                   "composite_fwd");
}

gsff_status gsff_adjoint_items(const gsff_gaussians* g, const gsff_camera* cam,
                               const gsff_settings* st, void* ws, size_t ws_bytes,
                               int64_t max_pairs, void* stream) {
  GSFF_PRELUDE
  return hip_check(launch_adjoint_items(c.L, c.w, c.s), "adjoint_items");
}

gsff_status gsff_composite_bwd(const gsff_gaussians* g, const gsff_camera* cam,
                               const gsff_settings* st, void* ws, size_t ws_bytes,
                               int64_t max_pairs, const float* g_rgb, const float* g_depth,
                               const float* g_alpha, const float* g_feat, const gsff_grads* out,
                               int32_t accumulate, void* stream) {
  GSFF_PRELUDE
  if (!out) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL grads");
  const bool geo = any_geometry(out);
  if (geo && (!g_rgb || !g_depth || !g_alpha))
    return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL upstream gradient");
  if (out->feat && g->C == 0) return fail(GSFF_ERR_INVALID_ARGUMENT, "feat grad with C == 0");
  return hip_check(launch_composite_bwd(c.g, c.st, c.L, c.w, g_rgb, g_depth, g_alpha, g_feat, geo,
                                        out->feat, accumulate, c.s),
                   "composite_bwd");
}

gsff_status gsff_preprocess_bwd(const gsff_gaussians* g, const gsff_camera* cam,
                                const gsff_settings* st, void* ws, size_t ws_bytes,
                                int64_t max_pairs, const gsff_grads* out, int32_t accumulate,
                                void* stream) {
  GSFF_PRELUDE
  if (!out) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL grads");
  if (!any_geometry(out)) return GSFF_OK;
  return hip_check(launch_preprocess_bwd(c.g, c.cam, c.st, c.L, c.w, *out, accumulate, c.s),
                   "preprocess_bwd");
}

gsff_status gsff_backward(const gsff_gaussians* g, const gsff_camera* cam,
                          const gsff_settings* st, void* ws, size_t ws_bytes, int64_t max_pairs,
                          const float* g_rgb, const float* g_depth, const float* g_alpha,
                          const float* g_feat, const gsff_grads* out, int32_t accumulate,
                          void* stream) {
  GSFF_PRELUDE
  if (!out) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL grads");
  const bool geo = any_geometry(out);
  if (geo && (!g_rgb || !g_depth || !g_alpha))
    return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL upstream gradient");
  if (out->feat && g->C == 0) return fail(GSFF_ERR_INVALID_ARGUMENT, "feat grad with C == 0");
  gsff_status rc = hip_check(launch_adjoint_items(c.L, c.w, c.s), "adjoint_items");
  if (rc != GSFF_OK) return rc;
  rc = hip_check(launch_composite_bwd(c.g, c.st, c.L, c.w, g_rgb, g_depth, g_alpha, g_feat, geo,
                                      out->feat, accumulate, c.s),
                 "composite_bwd");
  // the preprocess adjoint also turns the adjoint's rows into out->feat, so it
  // runs for a feature-only gradient too
  if (rc != GSFF_OK) return rc;
  return hip_check(launch_preprocess_bwd(c.g, c.cam, c.st, c.L, c.w, *out, accumulate, c.s),
                   "preprocess_bwd");
}

static gsff_status backward_l1_impl(const gsff_gaussians* g, const gsff_camera* cam,
                                    const gsff_settings* st, void* ws, size_t ws_bytes,
                                    int64_t max_pairs, const float* out_rgb,
                                    const float* out_depth, const float* out_alpha,
                                    const float* out_feat, const float* t_rgb,
                                    const float* t_depth, const float* t_alpha,
                                    const float* t_feat, const float* weights, float* loss,
                                    const gsff_grads* out, int32_t accumulate, void* stream,
                                    bool with_preprocess, const uint8_t* mask_v = nullptr,
                                    const uint8_t* mask_e = nullptr) {
  GSFF_PRELUDE
  if (!out) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL grads");
  if (!weights) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL weights");
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(weights[k])) return fail(GSFF_ERR_INVALID_ARGUMENT, "weights not finite");
  if ((t_rgb && !out_rgb) || (t_depth && !out_depth) || (t_alpha && !out_alpha) ||
      (t_feat && !out_feat))
    return fail(GSFF_ERR_INVALID_ARGUMENT, "target given without the forward output");
  if (out->feat && g->C == 0) return fail(GSFF_ERR_INVALID_ARGUMENT, "feat grad with C == 0");
  const bool geo = any_geometry(out);
  L1Args a{out_rgb, out_depth, out_alpha, out_feat, t_rgb, t_depth, t_alpha, t_feat,
           (double)weights[0], (double)weights[1], (double)weights[2], (double)weights[3], loss,
           mask_v, mask_e};
  // the L1 code pass builds the adjoint's work items itself
  gsff_status rc = hip_check(
      launch_composite_bwd_l1(c.g, c.st, c.L, c.w, a, geo, out->feat, accumulate, c.s),
      "composite_bwd_l1");
  if (rc != GSFF_OK || !with_preprocess) return rc;
  return hip_check(launch_preprocess_bwd(c.g, c.cam, c.st, c.L, c.w, *out, accumulate, c.s),
                   "preprocess_bwd");
}

gsff_status gsff_backward_l1(const gsff_gaussians* g, const gsff_camera* cam,
                             const gsff_settings* st, void* ws, size_t ws_bytes,
                             int64_t max_pairs, const float* out_rgb, const float* out_depth,
                             const float* out_alpha, const float* out_feat, const float* t_rgb,
                             const float* t_depth, const float* t_alpha, const float* t_feat,
                             const float* weights, float* loss, const gsff_grads* out,
                             int32_t accumulate, void* stream) {
  return backward_l1_impl(g, cam, st, ws, ws_bytes, max_pairs, out_rgb, out_depth, out_alpha,
                          out_feat, t_rgb, t_depth, t_alpha, t_feat, weights, loss, out,
                          accumulate, stream, true);
}

gsff_status gsff_backward_tracking(const gsff_gaussians* g, const gsff_camera* cam,
                                   const gsff_settings* st, void* ws, size_t ws_bytes,
                                   int64_t max_pairs, const float* out_rgb,
                                   const float* out_depth, const float* t_rgb,
                                   const float* t_depth, const uint8_t* mask_v,
                                   const uint8_t* mask_e, float lambda_t, float* loss,
                                   float* d_pose, int32_t accumulate, void* stream) {
  if (!d_pose) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL d_pose");
  if (!std::isfinite(lambda_t)) return fail(GSFF_ERR_INVALID_ARGUMENT, "lambda_t not finite");
  // the Gaussians are frozen: the pose is the only gradient
  gsff_grads out{};
  out.pose = d_pose;
  const float weights[4] = {lambda_t, 1.f - lambda_t, 0.f, 0.f};
  return backward_l1_impl(g, cam, st, ws, ws_bytes, max_pairs, out_rgb, out_depth, nullptr,
                          nullptr, t_rgb, t_depth, nullptr, nullptr, weights, loss, &out,
                          accumulate, stream, true, mask_v, mask_e);
}

gsff_status gsff_visibility(const gsff_gaussians* g, const gsff_camera* cam,
                            const gsff_settings* st, void* ws, size_t ws_bytes,
                            int64_t max_pairs, float t_vis, uint8_t* visible, void* stream) {
  GSFF_PRELUDE
  if (g->P > 0 && !visible) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL visible");
  if (!std::isfinite(t_vis)) return fail(GSFF_ERR_INVALID_ARGUMENT, "t_vis not finite");
  return hip_check(launch_visibility(c.st, c.g, c.L, c.w, t_vis, visible, c.s), "visibility");
}

gsff_status gsff_covisibility(const uint8_t* a, const uint8_t* b, int64_t n, uint32_t* counts,
                              void* stream) {
  if (n < 0 || !counts || (n > 0 && (!a || !b)))
    return fail(GSFF_ERR_INVALID_ARGUMENT, "covisibility arguments");
  if (n > (int64_t)0xFFFFFFFFu) return fail(GSFF_ERR_INVALID_ARGUMENT, "n above 2^32 - 1");
  return hip_check(launch_covisibility(a, b, n, counts, (hipStream_t)stream), "covisibility");
}

gsff_status gsff_keyframe_test(const uint8_t* frame_vis, const uint8_t* keyframe_vis, int64_t n,
                               float tau_thresh, uint32_t* counts, uint32_t* keyframe,
                               void* stream) {
  if (!keyframe || !std::isfinite(tau_thresh))
    return fail(GSFF_ERR_INVALID_ARGUMENT, "keyframe test arguments");
  const gsff_status rc = gsff_covisibility(frame_vis, keyframe_vis, n, counts, stream);
  if (rc != GSFF_OK) return rc;
  return hip_check(launch_keyframe_decide(counts, tau_thresh, keyframe, (hipStream_t)stream),
                   "keyframe decision");
}

gsff_status gsff_composite_bwd_l1(const gsff_gaussians* g, const gsff_camera* cam,
                                  const gsff_settings* st, void* ws, size_t ws_bytes,
                                  int64_t max_pairs, const float* out_rgb, const float* out_depth,
                                  const float* out_alpha, const float* out_feat,
                                  const float* t_rgb, const float* t_depth, const float* t_alpha,
                                  const float* t_feat, const float* weights, float* loss,
                                  const gsff_grads* out, int32_t accumulate, void* stream) {
  return backward_l1_impl(g, cam, st, ws, ws_bytes, max_pairs, out_rgb, out_depth, out_alpha,
                          out_feat, t_rgb, t_depth, t_alpha, t_feat, weights, loss, out,
                          accumulate, stream, false);
}

gsff_status gsff_l1_grad(const float* x, const float* y, int64_t n, float scale, float* grad,
                         float* loss, void* stream) {
  if (n < 0) return fail(GSFF_ERR_INVALID_ARGUMENT, "n < 0");
  if (n > 0 && (!x || !y || !grad)) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL pointer");
  return hip_check(launch_l1_grad(x, y, n, scale, grad, loss, (hipStream_t)stream), "l1_grad");
}

gsff_status gsff_read_status(const void* ws, uint32_t* flags, int64_t* n_pairs, void* stream) {
  if (!ws) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL workspace");
  gsff_status rc = hip_check(hipStreamSynchronize((hipStream_t)stream), "stream sync");
  if (rc != GSFF_OK) return rc;
  uint32_t h[4];
  rc = hip_check(hipMemcpy(h, ws, sizeof(h), hipMemcpyDeviceToHost), "status copy");
  if (rc != GSFF_OK) return rc;
  if (flags) *flags = h[0];
  if (n_pairs) *n_pairs = (int64_t)h[1];
  return GSFF_OK;
}

gsff_status gsff_read_checks(const void* ws, uint32_t* out, void* stream) {
  if (!ws || !out) return fail(GSFF_ERR_INVALID_ARGUMENT, "NULL workspace or output");
  gsff_status rc = hip_check(hipStreamSynchronize((hipStream_t)stream), "stream sync");
  if (rc != GSFF_OK) return rc;
  uint32_t h[8];
  rc = hip_check(hipMemcpy(h, ws, sizeof(h), hipMemcpyDeviceToHost), "status copy");
  if (rc != GSFF_OK) return rc;
  out[0] = h[kStatusChkCount];
  out[1] = h[kStatusChkSite];
  out[2] = h[kStatusChkIndex];
  out[3] = h[kStatusChkLimit];
  return GSFF_OK;
}

}  // extern "C"
