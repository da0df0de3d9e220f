/*
 * gsff.h -- C ABI of the MI355X (gfx950) feature-field Gaussian rasterizer.
 *
 * The library renders, for one pinhole camera, the RGB image, the depth image,
 * the accumulated opacity and an N-channel feature map of a set of 3D Gaussians
 * by front-to-back alpha blending (GSFF-SLAM, Sec. 3.1, Eqs. 1-3), and returns
 * the gradients of the outputs with respect to every Gaussian parameter and the
 * SE(3) camera pose (Sec. 3.2, Eq. 4).  The feature map's gradient reaches only
 * the feature embeddings, never the means, covariances, opacities or pose
 * (Sec. 3.1, last paragraph), and a flag turns feature rendering and its
 * gradient off altogether (same paragraph).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array pointers are DEVICE pointers to caller-owned memory unless stated.
 *    The library never allocates or frees device memory and keeps no pointer
 *    after a call returns.  All scratch lives in a caller-allocated workspace
 *    of gsff_workspace_size() bytes (256-byte aligned).
 *  - `stream` is a hipStream_t (passed as void*); all work is enqueued on it
 *    and the call returns without waiting.  Nothing inside the forward or
 *    backward synchronises host and device, so sequences of calls can be
 *    captured into a HIP graph.  Only gsff_read_status() waits.
 *  - Layouts: per-Gaussian vectors are planar [k, P] (component-major);
 *    features are row-major [P, C]; images are planar [k, H, W].
 *  - Calls are thread-compatible: the library holds no mutable global state
 *    (one exception, gsff_decoder_query_noalloc, keeps a fixed scratch array
 *    per GPU; see there).
 *  - Return value: GSFF_OK, or GSFF_ERR_INVALID_ARGUMENT (NULL pointer, bad
 *    size, workspace too small, unsupported size combination),
 *    GSFF_ERR_UNSUPPORTED (dtype / channel combination not built), or
 *    GSFF_ERR_HIP (a launch failed; gsff_last_error() has the text).
 *  - Conditions found on the device (too many tile pairs for the workspace)
 *    are not returned: they set bits of a status word inside the workspace that
 *    gsff_read_status() reports.  On overflow the affected frame renders as
 *    empty (zero images, T = 1) rather than reading out of bounds.
 */
#ifndef GSFF_H
#define GSFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gsff_status;
#define GSFF_OK 0
#define GSFF_ERR_INVALID_ARGUMENT (-1)
#define GSFF_ERR_UNSUPPORTED (-2)
#define GSFF_ERR_HIP (-3)

/* status-word bits set by the device */
#define GSFF_FLAG_PAIR_OVERFLOW 1u
/* a depth-sort workgroup stopped waiting for the digit counts of the
 * chunks before its own (see gsff_set_sort_wait_limit) and counted them
 * from the keys itself; the frame's results are valid */
#define GSFF_FLAG_SORT_RECOUNT 2u
/* checked build only (gsff_is_checked_build): an index that comes from data
 * (a sort destination, a listed Gaussian id, a tile range, an adjoint row or
 * slot) failed its bounds test; the access was skipped and
 * gsff_read_checks() names the first failure.  Never raised by a correct
 * library on any input. */
#define GSFF_FLAG_CHECK 4u

/* Sites of the checked build's bounds tests (gsff_read_checks) */
#define GSFF_CHECK_SORT_DEST 1u   /* depth-sort destination < P                     */
#define GSFF_CHECK_RANK_ID 2u     /* Gaussian id at a depth rank < P                */
#define GSFF_CHECK_PAIR_DEST 3u   /* binned pair position < pairs of the frame      */
#define GSFF_CHECK_TILE_RANGE 4u  /* super-tile list: start <= end <= pairs         */
#define GSFF_CHECK_LIST_ID 5u     /* id in a tile list or walked list < P           */
#define GSFF_CHECK_WALK 6u        /* walked-list entry inside the tile's segment    */
#define GSFF_CHECK_ITEM 7u        /* adjoint item: tile, segment, list range        */
#define GSFF_CHECK_ROW 8u         /* adjoint row < row capacity                     */
#define GSFF_CHECK_SLOT 9u        /* adjoint slot inside the Gaussian's slot range  */
#define GSFF_CHECK_REDUCE 10u     /* reduction item / row read from a slot          */

/* payload / output element types */
#define GSFF_DTYPE_F32 0
#define GSFF_DTYPE_BF16 1
#define GSFF_DTYPE_F16 2

/* largest channel count composited in one pass; wider payloads are rendered in
 * channel chunks of this size that recompute the blending weights (the
 * adjoint's first pass, which also carries the geometry, takes at most 32) */
#define GSFF_MAX_CHANNELS_PER_PASS 64

/* Screen tiles are GSFF_TILE x GSFF_TILE pixels; binning lists Gaussians per
 * super-tile of GSFF_SUPER x GSFF_SUPER tiles. */
#define GSFF_TILE 16
#define GSFF_SUPER 4

/* Rendering constants the paper does not print (it inherits them from the
 * 3D Gaussian splatting rasterizer it builds on, Sec. 3.1).  Defaults from
 * gsff_default_settings(): near 0.2, guard 1.3, dilation 0.3,
 * alpha_min 1/255, alpha_max 0.99, t_min 1e-4, render_features 1, bin_mode 0,
 * deterministic 0. */
typedef struct gsff_settings {
  float near_plane;       /* Gaussians with camera z <= near_plane are culled     */
  float guard;            /* cull |x/z| > guard*W/(2fx) or |y/z| > guard*H/(2fy)  */
  float dilation;         /* added to both diagonal entries of the 2D covariance */
  float alpha_min;        /* per-pixel alpha below this is skipped               */
  float alpha_max;        /* per-pixel alpha is clamped to this                  */
  float t_min;            /* blending stops before T would fall below this       */
  int32_t render_features;/* 0: feature map is zero and receives no gradient     */
  int32_t bin_mode;       /* 0: automatic; 1: bin by sorting (super-tile, rank)
                             keys even where the direct scatter applies (same
                             lists; for testing that path)                      */
  int32_t deterministic;  /* 1: the adjoint sums every Gaussian's per-tile
                             partial sums in a fixed order (each tile's sum in
                             the slot of its place in the Gaussian's rectangle,
                             one wave per Gaussian, no float atomics), so a
                             backward repeated on the same inputs gives the
                             same bits; 0 (default): slots in arrival order
                             and Gaussians of more than 64 tiles summed with
                             atomics (faster, run-to-run differences at FP32
                             rounding).  Holds while the adjoint's rows fit
                             (tiles whose rows do not fit fall back to
                             atomics in either mode).                          */
} gsff_settings;

/* Pinhole camera.  viewmat is a DEVICE pointer to 12 floats, the row-major
 * 3x4 world-to-camera transform [R | t] = T_CW (x right, y down, z forward).
 * Pixel (px, py) is sampled at (px + 1/2, py + 1/2). */
typedef struct gsff_camera {
  int32_t width, height;
  float fx, fy, cx, cy;
  const float* viewmat;
} gsff_camera;

/* Gaussian set G_i = {mean, quaternion, scale, opacity, colour, feature}
 * (Sec. 3.1).  Raw optimisation parameters: scale = exp(log_scales),
 * opacity = sigmoid(logit_opacity); the activations are fused into the
 * kernels.  Quaternions (w, x, y, z) need not be normalised.  rgb is a
 * view-independent colour.  feat is [P, C] in feat_dtype (NULL iff C == 0). */
typedef struct gsff_gaussians {
  int64_t P;
  int32_t C;
  int32_t feat_dtype;          /* GSFF_DTYPE_F32 / BF16 / F16 */
  const float* means;          /* [3, P] */
  const float* log_scales;     /* [3, P] */
  const float* quats;          /* [4, P] */
  const float* logit_opacity;  /* [P]    */
  const float* rgb;            /* [3, P] */
  const void* feat;            /* [P, C] */
} gsff_gaussians;

/* Gradient outputs, FP32, same layouts as the parameters.  Any pointer may be
 * NULL to skip that output.  pose is [6] = (rho, theta): the gradient w.r.t.
 * the left perturbation T_CW <- Exp(delta) T_CW at delta = 0 (Eq. 4),
 * summed over Gaussians in FP64.  feat is FP32 even for a BF16/FP16 payload. */
typedef struct gsff_grads {
  float* means;          /* [3, P] */
  float* log_scales;     /* [3, P] */
  float* quats;          /* [4, P] */
  float* logit_opacity;  /* [P]    */
  float* rgb;            /* [3, P] */
  float* feat;           /* [P, C] */
  float* pose;           /* [6]    */
} gsff_grads;

/* Where each workspace region starts (byte offsets from the workspace base)
 * and how big it is; used by tests to inspect intermediate stages. */
typedef struct gsff_ws_layout {
  uint64_t status;      /* uint32[8]: flags, pair count, pairs in use, reserved,
                           then (checked build) the first failed check's site,
                           index and limit, and the number of failed checks     */
  uint64_t records;     /* float4[3][P]: (u,v,A,B) (C,o,z,valid) (r,g,b,-)     */
  uint64_t rects;       /* uint16[4][P]: tile rect x0,y0,x1,y1 (inclusive); empty => x0>x1 */
  uint64_t depth_keys;  /* uint32[P]: sorted depth keys (float bits)           */
  uint64_t depth_ids;   /* uint32[P]: Gaussian index in depth order            */
  uint64_t pair_keys;   /* uint32[max_pairs]: Gaussian ids grouped by super-tile
                           (GSFF_SUPER x GSFF_SUPER tiles), in depth order inside
                           every super-tile                                     */
  uint64_t pair_masks;  /* uint16[max_pairs]: per pair, the tiles of its super-tile
                           that the Gaussian's rectangle covers: bit
                           GSFF_SUPER (ty % GSFF_SUPER) + (tx % GSFF_SUPER); a
                           tile's list is its super-tile's pairs with its bit set */
  uint64_t tile_ranges; /* uint32[2][super_x * super_y]: [start, end) into
                           pair_keys / pair_masks of every super-tile            */
  uint64_t tile_lists;  /* uint32: the per-tile lists the forward walked (ids in
                           list order), tile t at tile_list_ranges[t]           */
  uint64_t tile_list_ranges; /* uint32[2][ntiles]: [start, walk end) in tile_lists */
  uint64_t pix_T;       /* float[H*W]: final transmittance                     */
  uint64_t pix_end;     /* uint32[H*W]: 1 + tile_lists position of the last contributor */
  uint64_t grad2d;      /* float[P][10]: du dv dA dB dC do dr dg db dz; cleared by
                           gsff_preprocess, accumulated by the compositing
                           adjoint, consumed and cleared by gsff_preprocess_bwd */
  uint64_t total_bytes;
  int32_t rank_bits;    /* bits of the depth rank inside a pair key            */
  int32_t tiles_x, tiles_y;
  int32_t super_x, super_y;
} gsff_ws_layout;

/* Library version (host only, no device work). */
gsff_status gsff_version(int32_t* major, int32_t* minor);

/* *checked = 1 for the checked build of the library (libgsff_checked.so:
 * every data-dependent index of the rasterizer's kernels is tested against
 * the buffer it addresses, a failure skips the access and raises
 * GSFF_FLAG_CHECK; slower, for test runs), 0 for the release build.  Host
 * only. */
gsff_status gsff_is_checked_build(int32_t* checked);

/* The depth sort (Sec. 3.1: Gaussians blended in depth order) runs one
 * workgroup per chunk of keys.  This sets how many polls a workgroup makes
 * for the published digit counts of the chunks before its own before it
 * counts those chunks' digits from the keys itself (raising
 * GSFF_FLAG_SORT_RECOUNT); either way the sort is exact and stable, and
 * every wait ends whatever order the workgroups are dispatched in.  0 makes
 * every workgroup count (the fallback path, for tests).  Default 2048.
 * Process-wide; applies to frames enqueued afterwards.  Host only. */
gsff_status gsff_set_sort_wait_limit(uint32_t polls);

/* Text of the last GSFF_ERR_HIP / argument error raised on this thread. */
const char* gsff_last_error(void);

/* Fill *st with the defaults listed above (host only). */
gsff_status gsff_default_settings(gsff_settings* st);

/* Workspace bytes for P Gaussians with `channels` feature channels (the C of
 * the gsff_gaussians the workspace will serve; 0..4096), a pair capacity of
 * max_pairs (Gaussian / super-tile overlaps; the count a frame needs is
 * reported by gsff_read_status), and a width x height image (host only).
 * Requires P < 2^30, max_pairs < 2^32 - 1, and for tile grids binned by the
 * pair sort ceil(log2(max(P,2))) + ceil(log2(tiles)) <= 32.  The workspace
 * needs no initialisation. */
gsff_status gsff_workspace_size(int64_t P, int32_t channels, int64_t max_pairs, int32_t width,
                                int32_t height, size_t* bytes);

/* Region offsets of a workspace for these sizes (host only). */
gsff_status gsff_workspace_layout(int64_t P, int32_t channels, int64_t max_pairs, int32_t width,
                                  int32_t height, gsff_ws_layout* out);

/* Forward render (Sec. 3.1, Eqs. 1-3): preprocess, depth sort, tile binning,
 * tile sort, tile ranges and front-to-back compositing, all on `stream`.
 * Outputs (caller-owned, device): out_rgb [3,H,W] f32, out_depth [H,W] f32
 * (sum of w_i z_i, not normalised), out_alpha [H,W] f32 (= 1 - T_final),
 * out_feat [C,H,W] in out_feat_dtype (F32 or BF16; may be NULL when C == 0
 * or features are off -- when non-NULL and features are off it is zeroed).
 * The workspace keeps what the backward needs; leave it untouched between
 * the forward and the backward of the same frame. */
gsff_status gsff_forward(const gsff_gaussians* g, const gsff_camera* cam,
                         const gsff_settings* st, void* ws, size_t ws_bytes,
                         int64_t max_pairs, float* out_rgb, float* out_depth,
                         float* out_alpha, void* out_feat, int32_t out_feat_dtype,
                         void* stream);

/* Backward (Sec. 3.1 last paragraph; Sec. 3.2, Eq. 4) of the forward that
 * last used `ws`.  Upstream gradients g_rgb [3,H,W], g_depth [H,W],
 * g_alpha [H,W] (f32, none NULL) and g_feat [C,H,W] f32 (NULL = zero).
 * Geometry gradients (means, scales, rotations, opacities, colours, pose)
 * come only from g_rgb / g_depth / g_alpha; g_feat only reaches out->feat.
 * accumulate = 0 overwrites the outputs, 1 adds to them (multi-view).
 * With every geometry pointer NULL only the feature gradient is computed. */
gsff_status gsff_backward(const gsff_gaussians* g, const gsff_camera* cam,
                          const gsff_settings* st, void* ws, size_t ws_bytes,
                          int64_t max_pairs, const float* g_rgb, const float* g_depth,
                          const float* g_alpha, const float* g_feat,
                          const gsff_grads* out, int32_t accumulate, void* stream);

/* Backward of the L1 losses the method optimises (the tracking, mapping and
 * feature losses, Eqs. 6, 8 and 11, are weighted sums of L1 terms):
 *   L = w[0] mean|rgb - t_rgb| + w[1] mean|depth - t_depth|
 *     + w[2] mean|alpha - t_alpha| + w[3] mean|feat - t_feat|
 * with each mean over its group's elements (3HW, HW, HW, C*HW).  The adjoint
 * forms the upstream gradient (w_k / numel_k) sign(out - target) per pixel
 * itself, so no upstream images are materialised.  out_* are the outputs of
 * the forward that last used `ws` (f32, same layouts); t_* the targets, where
 * a NULL target leaves that group out of the loss.  weights: HOST pointer to
 * 4 floats.  loss (device, may be NULL) receives the loss terms whose
 * gradients are computed (rgb / depth / alpha only when a geometry gradient is
 * requested, feature only when out->feat is set and features are on):
 * accumulate = 0 overwrites it, 1 adds to it, as for the gradients.
 * Otherwise as gsff_backward. */
gsff_status gsff_backward_l1(const gsff_gaussians* g, const gsff_camera* cam,
                             const gsff_settings* st, void* ws, size_t ws_bytes,
                             int64_t max_pairs, const float* out_rgb, const float* out_depth,
                             const float* out_alpha, const float* out_feat, const float* t_rgb,
                             const float* t_depth, const float* t_alpha, const float* t_feat,
                             const float* weights, float* loss, const gsff_grads* out,
                             int32_t accumulate, void* stream);

/* Tracking backward (Sec. 3.2 tracking loss, Eq. 6; pose terms Eq. 4): with
 * the Gaussians frozen, the gradient of
 *   L = lambda_t mean(m_v m_e |rgb - t_rgb|) + (1 - lambda_t) mean(m_v |depth - t_depth|)
 * with respect to the pose perturbation only (d_pose [6], rho then theta, as
 * gsff_grads.pose).  The means run over all 3HW colour and HW depth elements;
 * a masked-out pixel contributes zero.  mask_v [H,W] (the visibility mask)
 * and mask_e [H,W] (the edge mask), uint8 on the device, non-zero = kept;
 * NULL keeps every pixel.  A NULL target leaves its term out.  out_rgb and
 * out_depth are the forward outputs of the same frame.  loss (device, may be
 * NULL) receives L: accumulate = 0 overwrites it and d_pose, 1 adds to them.
 * Errors: GSFF_ERR_INVALID_ARGUMENT for a NULL d_pose or a non-finite
 * lambda_t; otherwise as gsff_backward_l1. */
gsff_status gsff_backward_tracking(const gsff_gaussians* g, const gsff_camera* cam,
                                   const gsff_settings* st, void* ws, size_t ws_bytes,
                                   int64_t max_pairs, const float* out_rgb,
                                   const float* out_depth, const float* t_rgb,
                                   const float* t_depth, const uint8_t* mask_v,
                                   const uint8_t* mask_e, float lambda_t, float* loss,
                                   float* d_pose, int32_t accumulate, void* stream);

/* Scale regulariser of the mapping loss (Sec. 3.2, Eqs. 7-8):
 *   L_reg = lambda (1/N) sum_i |s_i - sbar|_1,  s_i = exp(log_scales[:, i]),
 * sbar the mean of the N = P scale vectors, |.|_1 over the three components.
 * grad_log_scales [3, P] (may be NULL) receives dL/dlog_scales and loss
 * (device, may be NULL) L: accumulate = 0 overwrites, 1 adds.  The gradient
 * takes the mean's dependence on every s_i into account; sign(0) = 0.
 * workspace: device scratch of gsff_scale_reg_workspace_size bytes, 8-byte
 * aligned.  Errors: GSFF_ERR_INVALID_ARGUMENT for P <= 0, a NULL input or
 * workspace, a small or misaligned workspace or a non-finite lambda. */
gsff_status gsff_scale_reg(const float* log_scales, int64_t P, float lambda, float* workspace,
                           size_t ws_bytes, float* grad_log_scales, float* loss,
                           int32_t accumulate, void* stream);
gsff_status gsff_scale_reg_workspace_size(int64_t P, size_t* bytes);

/* One Adam step over up to 8 parameter groups in one launch (the mapping
 * step's optimiser over the Gaussians' SoA parameters; FP32): per element
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * param -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * All pointers are device pointers; m and v start at zero; step counts from
 * 1.  Errors: GSFF_ERR_INVALID_ARGUMENT for a NULL pointer in a non-empty
 * group, 0 or more than 8 groups, step < 1, betas outside [0, 1), eps <= 0
 * or a non-finite rate. */
typedef struct gsff_adam_group {
  float* param;
  const float* grad;
  float* m;
  float* v;
  int64_t n;
  float lr;
} gsff_adam_group;
gsff_status gsff_adam_step(const gsff_adam_group* groups, int32_t ngroups, int32_t step,
                           float beta1, float beta2, float eps, void* stream);

/* Visibility record of the last forward on `ws` (Sec. 3.2 keyframe
 * selection, Eq. 5): visible [P] uint8 on the device receives 1 for every
 * Gaussian blended at some pixel while the transmittance in front of it
 * exceeds t_vis (the paper's 0.5), 0 for every other.  The decisions are the
 * forward's own (same arithmetic on the walk it recorded), so call it after
 * gsff_forward / gsff_composite_fwd with the same arguments.  Errors:
 * GSFF_ERR_INVALID_ARGUMENT for a NULL visible (P > 0) or a non-finite t_vis. */
gsff_status gsff_visibility(const gsff_gaussians* g, const gsff_camera* cam,
                            const gsff_settings* st, void* ws, size_t ws_bytes,
                            int64_t max_pairs, float t_vis, uint8_t* visible, void* stream);

/* Co-visibility of two visibility records a, b [n] (uint8, non-zero =
 * visible; Sec. 3.2): counts [2] uint32 on the device receive |a and b| and
 * |a or b|; their ratio is the IoU that the keyframe test compares with
 * tau_thresh.  Errors: GSFF_ERR_INVALID_ARGUMENT for a NULL pointer, n < 0
 * or n >= 2^32. */
gsff_status gsff_covisibility(const uint8_t* a, const uint8_t* b, int64_t n, uint32_t* counts,
                              void* stream);

/* Keyframe test (Sec. 3.2 keyframe selection): the frame becomes a keyframe
 * when the IoU of its visibility record frame_vis with the last keyframe's
 * record keyframe_vis ([n] uint8, non-zero = visible) is below tau_thresh.
 * counts [2] receive |a and b| and |a or b| (as gsff_covisibility) and
 * keyframe [1] receives 1 for a keyframe, else 0; the IoU (1 when both
 * records are empty) is formed and compared in FP64 on the device, so the
 * decision needs no host round trip.  Device pointers.  Errors:
 * GSFF_ERR_INVALID_ARGUMENT for a NULL counts or keyframe, a non-finite
 * tau_thresh, or the arguments gsff_covisibility rejects. */
gsff_status gsff_keyframe_test(const uint8_t* frame_vis, const uint8_t* keyframe_vis, int64_t n,
                               float tau_thresh, uint32_t* counts, uint32_t* keyframe,
                               void* stream);

/* The masks of the tracking loss (Sec. 3.2, Eq. 6), uint8 [H,W] on the
 * device, 1 = kept.  mask_e: the edge mask of the target colour image t_rgb
 * [3,H,W] f32: the Sobel gradient of the grey image (mean of the three
 * channels), scaled by 1/8 so that a ramp of slope a per pixel has magnitude
 * a, the border replicated; kept where the magnitude exceeds edge_threshold
 * (>= 0).  mask_v: the visibility mask, kept where alpha [H,W] f32 (the
 * accumulated opacity of the render at the frozen Gaussians) exceeds
 * vis_threshold.  Either output may be NULL (its input may then be NULL).
 * Errors: GSFF_ERR_INVALID_ARGUMENT for a non-positive size, a missing input
 * or a non-finite or negative threshold. */
gsff_status gsff_tracking_masks(const float* t_rgb, const float* alpha, int32_t width,
                                int32_t height, float edge_threshold, float vis_threshold,
                                uint8_t* mask_v, uint8_t* mask_e, void* stream);

/* Convergence test of the tracking loop (Sec. 3.2: the pose iterations of
 * a frame end when the changes of the camera-frame means and of the rotation
 * have converged).  Every `window` steps the pose step measures the net
 * motion T_now T_start^-1 over the window (T_start: the pose when the window
 * began): its rotation angle (radians) against tol_rot and the length of its
 * translation (the shift of the camera-frame position of the world origin,
 * in the units of the means) against tol_trans. */
typedef struct gsff_pose_convergence {
  int32_t window;   /* steps per test, >= 1 */
  float tol_trans;  /* >= 0 */
  float tol_rot;    /* >= 0, radians */
} gsff_pose_convergence;

/* Floats of pose-step state (Adam moments, window start, converged flag). */
#define GSFF_POSE_STATE_FLOATS 32

/* One pose step of the tracking loop (Sec. 3.2; the increment is the left
 * perturbation of Eq. 4).  d_pose [6] (rho, theta) is the gradient from
 * gsff_backward_tracking; state [GSFF_POSE_STATE_FLOATS] holds Adam's
 * moments, the pose at the start of the test window and the converged flag;
 * step counts from 1, and step 1 resets the state (a new frame).  The
 * increment delta_k = -lr_k mhat_k / (sqrt(vhat_k) + eps) (lr_trans for rho,
 * lr_rot for theta) is applied as viewmat <- Exp(delta) viewmat with the
 * closed-form SE(3) exponential, in FP64, and written to delta [6] if that is
 * not NULL.  conv (HOST pointer, may be NULL = no test) sets the convergence
 * test; converged (device, may be NULL) receives 1 when the test held at this
 * step or an earlier one of the frame, else 0.  Once it has held, later steps
 * of the frame leave viewmat and state unchanged and write a zero delta, so a
 * captured loop of a fixed number of steps ends where an early exit would.
 * All other pointers are device pointers; viewmat is updated in place.
 * Errors: GSFF_ERR_INVALID_ARGUMENT for a NULL pointer, step < 1, betas
 * outside [0, 1), eps <= 0, a non-finite rate, or a window < 1 or a negative
 * or non-finite tolerance in conv. */
gsff_status gsff_pose_adam_step(float* viewmat, const float* d_pose, float* state,
                                int32_t step, float lr_trans, float lr_rot, float beta1,
                                float beta2, float eps, const gsff_pose_convergence* conv,
                                float* delta, uint32_t* converged, void* stream);

/* Stage entry points: the forward is exactly preprocess, sort_depth, bin,
 * sort_tiles, tile_ranges, composite_fwd in this order; the backward is
 * composite_bwd then preprocess_bwd.  Same arguments and conventions as the
 * two calls above; exposed for stage-by-stage testing and timing.  Binning
 * lists Gaussians per super-tile (GSFF_SUPER x GSFF_SUPER tiles) in depth
 * order with a tile mask per entry (ws_layout.pair_keys / pair_masks); for
 * super-tile grids whose 16 bytes per super-tile plus 32 per super-tile row
 * and column fit in 64 KiB, `bin` writes the lists directly and `sort_tiles` /
 * `tile_ranges` have nothing left to do, other grids (or bin_mode 1) sort
 * (super-tile, rank) keys.  `composite_fwd` walks each tile's entries of its
 * super-tile list and records the ids it walked (ws_layout.tile_lists), which
 * the adjoint then walks back to front.  The compositing adjoints leave their
 * per-Gaussian sums (image-space terms and feature gradients) inside `ws` as
 * one row per walked (tile, Gaussian) pair, filed per Gaussian, plus direct
 * accumulation for tiles whose rows do not fit; `preprocess` resets them and
 * `preprocess_bwd` adds them up, writes the feature gradient (out->feat, +=)
 * and resets them again: each composite_bwd (or composite_bwd_l1) is followed
 * by one preprocess_bwd with the same `out`.  `adjoint_items` turns the walks
 * of the last composite_fwd into the adjoint's work items (each tile's walked
 * list in segments of 64 entries, at most 8 per tile, longest first; the
 * forward recorded each pixel's state at every segment end), the first
 * adjoint row of every tile and the first slot of every 256-Gaussian block
 * (from the counts preprocess wrote; repeating it gives the same result): it
 * runs after composite_fwd and before the
 * first composite_bwd that follows it (gsff_backward runs it itself;
 * composite_bwd_l1 and gsff_backward_l1 build the same items inside their
 * L1 upstream pass and need no adjoint_items call). */
gsff_status gsff_preprocess(const gsff_gaussians* g, const gsff_camera* cam,
                            const gsff_settings* st, void* ws, size_t ws_bytes,
                            int64_t max_pairs, void* stream);
gsff_status gsff_sort_depth(const gsff_gaussians* g, const gsff_camera* cam,
                            const gsff_settings* st, void* ws, size_t ws_bytes,
                            int64_t max_pairs, void* stream);
gsff_status gsff_bin(const gsff_gaussians* g, const gsff_camera* cam,
                     const gsff_settings* st, void* ws, size_t ws_bytes,
                     int64_t max_pairs, void* stream);
gsff_status gsff_sort_tiles(const gsff_gaussians* g, const gsff_camera* cam,
                            const gsff_settings* st, void* ws, size_t ws_bytes,
                            int64_t max_pairs, void* stream);
gsff_status gsff_tile_ranges(const gsff_gaussians* g, const gsff_camera* cam,
                             const gsff_settings* st, void* ws, size_t ws_bytes,
                             int64_t max_pairs, void* stream);
gsff_status gsff_composite_fwd(const gsff_gaussians* g, const gsff_camera* cam,
                               const gsff_settings* st, void* ws, size_t ws_bytes,
                               int64_t max_pairs, float* out_rgb, float* out_depth,
                               float* out_alpha, void* out_feat, int32_t out_feat_dtype,
                               void* stream);
gsff_status gsff_adjoint_items(const gsff_gaussians* g, const gsff_camera* cam,
                               const gsff_settings* st, void* ws, size_t ws_bytes,
                               int64_t max_pairs, void* stream);
gsff_status gsff_composite_bwd(const gsff_gaussians* g, const gsff_camera* cam,
                               const gsff_settings* st, void* ws, size_t ws_bytes,
                               int64_t max_pairs, const float* g_rgb,
                               const float* g_depth, const float* g_alpha,
                               const float* g_feat, const gsff_grads* out,
                               int32_t accumulate, void* stream);
/* The compositing part of gsff_backward_l1 alone (its stage split: follow it
 * with gsff_preprocess_bwd). */
gsff_status gsff_composite_bwd_l1(const gsff_gaussians* g, const gsff_camera* cam,
                                  const gsff_settings* st, void* ws, size_t ws_bytes,
                                  int64_t max_pairs, const float* out_rgb, const float* out_depth,
                                  const float* out_alpha, const float* out_feat,
                                  const float* t_rgb, const float* t_depth, const float* t_alpha,
                                  const float* t_feat, const float* weights, float* loss,
                                  const gsff_grads* out, int32_t accumulate, void* stream);
gsff_status gsff_preprocess_bwd(const gsff_gaussians* g, const gsff_camera* cam,
                                const gsff_settings* st, void* ws, size_t ws_bytes,
                                int64_t max_pairs, const gsff_grads* out,
                                int32_t accumulate, void* stream);

/* ---- learned 1x1 feature decoder (the lift o(.) of Eq. 11) ------------------
 * Y = GELU(X W1 + b1) W2 + b2 per pixel, GELU in its tanh form
 * 0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))), both products on BF16
 * matrix cores with FP32 accumulation; X, W1, W2 and the hidden activations
 * are rounded to BF16 (round to nearest even), everything else is FP32.
 * Maps are planar: X bf16 [16, n_px] (the rasterizer's 16-channel latent
 * output), Y / targets [512, n_px].  Weights are FP32 masters, row-major
 * W1 [16, 128], b1 [128], W2 [128, 512], b2 [512]; the library makes the BF16
 * copies in the decoder workspace.  Device pointers; ws 256-byte aligned. */

/* Decoder workspace bytes for n_px pixels (host only). */
gsff_status gsff_decoder_workspace_size(int64_t n_px, size_t* bytes);

/* Inference: Y [512, n_px] in y_dtype (F32 or BF16). */
gsff_status gsff_decoder_forward(const void* X, const float* W1, const float* b1,
                                 const float* W2, const float* b2, void* Y, int32_t y_dtype,
                                 int64_t n_px, void* ws, size_t ws_bytes, void* stream);

/* One fused training step of L = scale * sum |Y - T| (T bf16 [512, n_px]):
 * forward, L1, and the backward to the latent map and the weights.
 * loss (device, may be NULL) += L; dX f32 [16, n_px] (feed it to the
 * rasterizer's feature-only backward as the feature upstream); dW1 [16,128],
 * db1 [128], dW2 [128,512], db2 [512] f32 are overwritten.  Gradients with
 * respect to the FP32 master weights pass straight through the BF16 rounding. */
gsff_status gsff_decoder_train_step(const void* X, const float* W1, const float* b1,
                                    const float* W2, const float* b2, const void* T,
                                    int64_t n_px, float scale, float* loss, float* dX,
                                    float* dW1, float* db1, float* dW2, float* db2, void* ws,
                                    size_t ws_bytes, void* stream);

/* Decode + query (Eqs. 10 and 12): the label probabilities
 *   p(l | x) = softmax_l( o(F)(x) . q(l) ),  o(F)(x) = GELU(X W1 + b1) W2 + b2,
 * for K query vectors Q [K, 512] f32 (1 <= K <= 64), without forming the
 * 512-channel map (the queries fold into the second layer; FP32 arithmetic).
 * X bf16 [16, n_px], weights as gsff_decoder_forward.  Outputs, each may be
 * NULL: prob [K, n_px] f32; label [n_px] int32, the label of the largest
 * logit (the first of equal ones), the prediction of Eq. 10; and, with gt
 * [n_px] int32 given, ce_loss (device [1]) = the cross-entropy of Eq. 9,
 * (1/n_px) sum over the pixels whose gt lies in [0, K) of -log p(gt | x)
 * (other pixels are left out of the sum, not of n_px).  gt and ce_loss come
 * together (with n_px = 0, ce_loss alone receives 0).  ws: device scratch of
 * gsff_decoder_query_workspace_size bytes, 16-byte aligned.  Errors:
 * GSFF_ERR_INVALID_ARGUMENT for K outside [1, 64], n_px < 0, a NULL input,
 * gt without ce_loss or the reverse (n_px > 0), or a small or misaligned
 * workspace. */
gsff_status gsff_decoder_query_workspace_size(int32_t K, int64_t n_px, size_t* bytes);
gsff_status gsff_decoder_query(const void* X, const float* W1, const float* b1, const float* W2,
                               const float* b2, const float* Q, int32_t K, int64_t n_px,
                               float* prob, int32_t* label, const int32_t* gt, float* ce_loss,
                               void* ws, size_t ws_bytes, void* stream);

/* gsff_decoder_query without a workspace argument, for callers that cannot
 * allocate device memory (code under stream / graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, outputs, errors
 * and arithmetic as gsff_decoder_query, minus ws / ws_bytes; it calls no
 * allocating routine.  Its scratch (the label-folded second layer for up to
 * 64 labels and at most 1024 per-block loss partials: 37,124 bytes, enough
 * for any n_px) is a fixed device array that each GPU the library runs on
 * holds until the process ends; its device address is looked up on the
 * first call on each device.  Every call on one GPU shares that array: calls
 * that overlap on one GPU (different streams or threads without ordering)
 * race and give undefined results; calls ordered on one stream do not.
 * Nothing needs clearing between calls (a call writes every scratch word it
 * reads).  Errors: those of gsff_decoder_query (K above 64 is the scratch's
 * limit), or GSFF_ERR_HIP if the scratch address cannot be found. */
gsff_status gsff_decoder_query_noalloc(const void* X, const float* W1, const float* b1,
                                       const float* W2, const float* b2, const float* Q,
                                       int32_t K, int64_t n_px, float* prob, int32_t* label,
                                       const int32_t* gt, float* ce_loss, void* stream);

/* L1 loss of one output group (the tracking / mapping / semantic losses,
 * Eqs. 6, 8 and 11, are weighted L1 terms): grad[i] = scale * sign(x[i] - y[i])
 * (0 where equal) and, if loss != NULL, *loss += scale * sum |x - y| (FP32
 * atomics).  n elements, device pointers. */
gsff_status gsff_l1_grad(const float* x, const float* y, int64_t n, float scale,
                         float* grad, float* loss, void* stream);

/* ---- FP64 instantiation, for derivative checks ----------------------------
 * The forward and adjoint above in FP64, built from the same device code for
 * the projection (Sec. 3.1, Eq. 1 and its splat) and its adjoint with the pose
 * terms (Sec. 3.2, Eq. 4), and for the adjoint's per-pair back-to-front step
 * and per-tile moments-to-gradient step (Eqs. 2-3).  What the FP32 kernels sum
 * on the matrix cores is summed by plain FP64 loops, and every Gaussian meets
 * every pixel (the FP32 tile lists only leave out pairs below alpha_min).
 * Central finite differences of gsff_forward_f64 check gsff_backward_f64; it
 * is not a rendering path (slow by design).  Same layouts, conventions and
 * settings as the FP32 entry points, with doubles; limits P <= 4096,
 * C <= 32, 1 <= width, height <= 256.  The image is rendered from the
 * camera's pixel centres, features are FP64 [P, C]. */
typedef struct gsff_gaussians_f64 {
  int64_t P;
  int32_t C;
  const double* means;          /* [3, P] */
  const double* log_scales;     /* [3, P] */
  const double* quats;          /* [4, P] */
  const double* logit_opacity;  /* [P]    */
  const double* rgb;            /* [3, P] */
  const double* feat;           /* [P, C] */
} gsff_gaussians_f64;

/* viewmat: DEVICE pointer to 12 doubles, row-major [R | t] = T_CW. */
typedef struct gsff_camera_f64 {
  int32_t width, height;
  double fx, fy, cx, cy;
  const double* viewmat;
} gsff_camera_f64;

/* Every pointer but feat (NULL iff C == 0) is required; outputs are written,
 * not accumulated.  pose [6] as in gsff_grads (rho, theta; left
 * perturbation), summed over the Gaussians in index order. */
typedef struct gsff_grads_f64 {
  double* means;          /* [3, P] */
  double* log_scales;     /* [3, P] */
  double* quats;          /* [4, P] */
  double* logit_opacity;  /* [P]    */
  double* rgb;            /* [3, P] */
  double* feat;           /* [P, C] */
  double* pose;           /* [6]    */
} gsff_grads_f64;

/* Bytes of the FP64 workspace (256-byte aligned by the caller). */
gsff_status gsff_f64_workspace_size(int64_t P, int32_t channels, int32_t width, int32_t height,
                                    size_t* bytes);

/* FP64 forward: out_rgb [3, H, W], out_depth [H, W] (sum of w_i z_i),
 * out_alpha [H, W] (1 - final T), out_feat [C, H, W] (required when C > 0
 * and features are rendered; zeros when they are not), and, if out_n is not
 * NULL, out_n [H, W] int32: the Gaussians each pixel blended.  Leaves in ws
 * what gsff_backward_f64 of the same inputs needs.  Errors:
 * GSFF_ERR_INVALID_ARGUMENT for sizes past the limits, NULL pointers, bad
 * settings or a small or misaligned workspace. */
gsff_status gsff_forward_f64(const gsff_gaussians_f64* g, const gsff_camera_f64* cam,
                             const gsff_settings* st, void* ws, size_t ws_bytes, double* out_rgb,
                             double* out_depth, double* out_alpha, double* out_feat,
                             int32_t* out_n, void* stream);

/* FP64 adjoint of the last gsff_forward_f64 on ws (same inputs): upstream
 * g_rgb [3, H, W], g_depth, g_alpha [H, W], g_feat [C, H, W] (required when
 * C > 0).  As in the FP32 path the feature upstream reaches only out->feat.
 * Errors as gsff_forward_f64, and for a NULL upstream or gradient output. */
gsff_status gsff_backward_f64(const gsff_gaussians_f64* g, const gsff_camera_f64* cam,
                              const gsff_settings* st, void* ws, size_t ws_bytes,
                              const double* g_rgb, const double* g_depth, const double* g_alpha,
                              const double* g_feat, const gsff_grads_f64* out, void* stream);

/* Wait for `stream`, then copy the workspace status word (which starts at
 * byte 0 of every workspace) to the host: *flags receives the GSFF_FLAG_*
 * bits and *n_pairs the number of super-tile pairs the last forward needed (even
 * when it exceeded max_pairs).  Host pointers; either may be NULL. */
gsff_status gsff_read_status(const void* ws, uint32_t* flags, int64_t* n_pairs, void* stream);

/* Checked build: wait for `stream`, then copy the bounds-test record of the
 * workspace to host memory out[4] = {failed tests, site of the first failure
 * (GSFF_CHECK_*), its index, its limit} (indices saturate at 2^32 - 1).  The
 * record is cleared by every forward (gsff_forward / gsff_preprocess) and
 * collects the failures of the forward and of the adjoints that follow it.
 * The release build tests nothing and reports zeros. */
gsff_status gsff_read_checks(const void* ws, uint32_t* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GSFF_H */
