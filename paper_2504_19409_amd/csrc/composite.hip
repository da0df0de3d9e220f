// Front-to-back alpha compositing of colour, depth and a C-channel feature
// payload (Sec. 3.1, Eqs. 2-3) and its adjoint.
//
// One 256-thread workgroup per 16x16 screen tile, one thread per pixel.  The
// tile's depth-ordered Gaussian list is walked in batches staged in LDS
// (records gathered by id, features converted to FP32 on the way in); all
// blending and transmittance is FP32.  A workgroup stops as soon as every
// pixel in it has saturated (T would fall below t_min).
//
// Workgroup -> tile mapping is XCD-aware: the dispatcher hands consecutive
// workgroups to the 8 XCDs in turn, so workgroup b is sent to tile
// (b % 8) * ceil(ntiles/8) + b / 8 -- each XCD then renders a contiguous
// band of tiles and neighbouring tiles (which share most Gaussians) hit the
// same L2.
//
// The adjoint walks back to front from each pixel's last contributor,
// recovering T_i = T_{i+1} / (1 - alpha_i) instead of storing per-pixel
// lists.  Geometry gradients (dalpha and everything behind it) come only
// from the colour, depth and opacity upstream; the feature upstream only
// produces d f_i = sum_p w_ip g_F(p) (Sec. 3.1, last paragraph).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "gsff_internal.h"

namespace gsff {

constexpr int kFwdBatch = 64;
constexpr int kBwdBatch = 64;
constexpr int kNumXcd = 8;

__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  const int per = (ntiles + kNumXcd - 1) / kNumXcd;
  return (b % kNumXcd) * per + b / kNumXcd;
}

__device__ __forceinline__ float load_feat(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float load_feat(const uint16_t* p, int64_t i) {
  return __uint_as_float((uint32_t)p[i] << 16);
}
__device__ __forceinline__ float load_feat(const _Float16* p, int64_t i) { return (float)p[i]; }

__device__ __forceinline__ void store_out(float* p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void store_out(uint16_t* p, int64_t i, float v) {
  // round to nearest even
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) {
    p[i] = 0x7FC0u;
    return;
  }
  u += 0x7FFFu + ((u >> 16) & 1u);
  p[i] = (uint16_t)(u >> 16);
}

// A tile's [start, end) limited to the pair buffer.
__device__ __forceinline__ uint2 clamp_range(uint2 r, uint32_t max_pairs) {
  const uint32_t e = min(r.y, max_pairs);
  return make_uint2(min(r.x, e), e);
}

// Gaussian id of pair `idx` (the pair buffer holds ids grouped by tile);
// returns P (an out-of-range marker) for an id that is not a valid index, so
// no gather can leave the record arrays.
__device__ __forceinline__ uint32_t pair_gid(const WsView& w, uint32_t idx, uint32_t,
                                             int64_t P) {
  const uint32_t gid = w.pkeys_a[idx];
  return gid < (uint32_t)P ? gid : (uint32_t)P;
}

// Gather the three record vectors of `gid`; an out-of-range id gets zero
// opacity, so every pixel skips it.
__device__ __forceinline__ void load_record(const WsView& w, uint32_t gid, int64_t P, float4& r0,
                                            float4& r1, float4& r2) {
  if (gid < (uint32_t)P) {
    r0 = w.rec[gid];
    r1 = w.rec[P + gid];
    r2 = w.rec[2 * P + gid];
  } else {
    r0 = make_float4(0.f, 0.f, 0.f, 0.f);
    r1 = r0;
    r2 = r0;
  }
}

// alpha of one (pixel, Gaussian) pair; forward and adjoint call this same
// code so every skip decision and weight is reproduced bit for bit.
struct AlphaEval {
  float dx, dy, G, oG, alpha;
};

__device__ __forceinline__ AlphaEval eval_alpha(const float4 r0, const float4 r1, float pxc,
                                                float pyc, float alpha_max) {
#pragma clang fp contract(off)
  AlphaEval e;
  e.dx = r0.x - pxc;
  e.dy = r0.y - pyc;
  // -1/2 (A dx^2 + 2 B dx dy + C dy^2), A = r0.z, B = r0.w, C = r1.x
  const float q = __builtin_fmaf(r0.z * e.dx, e.dx,
                                 __builtin_fmaf(2.f * r0.w * e.dx, e.dy, r1.x * e.dy * e.dy));
  e.G = __expf(-0.5f * q);
  e.oG = r1.y * e.G;
  e.alpha = e.oG < alpha_max ? e.oG : alpha_max;
  return e;
}

// ------------------------------------------------------------ forward -----

template <int CP, typename FT, typename OT>
__global__ __launch_bounds__(kBlock) void k_composite_fwd(
    DevSettings st, int64_t P, int C, int c0, int W, int H, int tiles_x, int ntiles,
    int rank_bits, uint32_t max_pairs, WsView w, const FT* __restrict__ feat,
    float* __restrict__ out_rgb,
    float* __restrict__ out_depth, float* __restrict__ out_alpha, OT* __restrict__ out_feat,
    int write_geo) {
  constexpr int CPs = CP > 0 ? CP : 1;
  __shared__ float4 s_r0[kFwdBatch], s_r1[kFwdBatch], s_r2[kFwdBatch];
  __shared__ float s_f[kFwdBatch][CPs];
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int px = tx * kTile + (threadIdx.x & (kTile - 1));
  const int py = ty * kTile + (threadIdx.x / kTile);
  const bool inside = px < W && py < H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 range = clamp_range(w.tile_ranges[tile], max_pairs);
  const uint32_t rmask = (rank_bits >= 32) ? 0xFFFFFFFFu : ((1u << rank_bits) - 1u);
  const int cn = CP > 0 ? min(CP, C - c0) : 0;

  float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, dep = 0.f;
  float acc[CPs];
#pragma unroll
  for (int c = 0; c < CPs; ++c) acc[c] = 0.f;
  bool done = !inside;
  uint32_t end = range.x;

  for (uint32_t b0 = range.x; b0 < range.y; b0 += kFwdBatch) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t n = min((uint32_t)kFwdBatch, range.y - b0);
    if (threadIdx.x < n) {
      const uint32_t gid = pair_gid(w, b0 + threadIdx.x, rmask, P);
      load_record(w, gid, P, s_r0[threadIdx.x], s_r1[threadIdx.x], s_r2[threadIdx.x]);
      if (CP > 0) {
#pragma unroll
        for (int c = 0; c < CP; ++c)
          s_f[threadIdx.x][c] =
              (c < cn && gid < (uint32_t)P) ? load_feat(feat, (int64_t)gid * C + c0 + c) : 0.f;
      }
    }
    __syncthreads();
    if (!done) {
      for (uint32_t j = 0; j < n; ++j) {
        const float4 r0 = s_r0[j], r1 = s_r1[j];
        const AlphaEval e = eval_alpha(r0, r1, pxc, pyc, st.alpha_max);
        if (e.alpha < st.alpha_min) continue;
        const float Tn = T * (1.f - e.alpha);
        if (Tn < st.t_min) {
          done = true;
          break;
        }
        const float wgt = e.alpha * T;
        const float4 r2 = s_r2[j];
        cr += wgt * r2.x;
        cg += wgt * r2.y;
        cb += wgt * r2.z;
        dep += wgt * r1.z;
#pragma unroll
        for (int c = 0; c < CP; ++c) acc[c] += wgt * s_f[j][c];
        T = Tn;
        end = b0 + j + 1;
      }
    }
  }
  if (!inside) return;
  const int64_t HW = (int64_t)W * H;
  const int64_t p = (int64_t)py * W + px;
  if (write_geo) {
    out_rgb[p] = cr;
    out_rgb[HW + p] = cg;
    out_rgb[2 * HW + p] = cb;
    out_depth[p] = dep;
    out_alpha[p] = 1.f - T;
    w.pix_T[p] = T;
    w.pix_end[p] = end;
  }
  if (CP > 0 && out_feat) {
#pragma unroll
    for (int c = 0; c < CP; ++c)
      if (c < cn) store_out(out_feat, (int64_t)(c0 + c) * HW + p, acc[c]);
  }
}

template <typename OT>
__global__ void k_fill_zero(OT* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = OT(0);
}

template <int CP, typename FT, typename OT>
static void launch_fwd_t(const DevSettings& st, const DevGaussians& g, const Layout& L,
                         const WsView& w, int c0, float* out_rgb, float* out_depth,
                         float* out_alpha, void* out_feat, int write_geo, hipStream_t s) {
  const int grid = ((L.ntiles + kNumXcd - 1) / kNumXcd) * kNumXcd;
  hipLaunchKernelGGL((k_composite_fwd<CP, FT, OT>), dim3(grid), dim3(kBlock), 0, s, st, g.P, g.C,
                     c0, L.W, L.H, L.tiles_x, L.ntiles, L.rank_bits, (uint32_t)L.max_pairs, w,
                     (const FT*)g.feat, out_rgb, out_depth, out_alpha, (OT*)out_feat, write_geo);
}

template <typename FT, typename OT>
static void launch_fwd_dispatch(int cn, const DevSettings& st, const DevGaussians& g,
                                const Layout& L, const WsView& w, int c0, float* out_rgb,
                                float* out_depth, float* out_alpha, void* out_feat,
                                int write_geo, hipStream_t s) {
  if (cn <= 0)
    launch_fwd_t<0, FT, OT>(st, g, L, w, c0, out_rgb, out_depth, out_alpha, nullptr, write_geo, s);
  else if (cn <= 8)
    launch_fwd_t<8, FT, OT>(st, g, L, w, c0, out_rgb, out_depth, out_alpha, out_feat, write_geo, s);
  else if (cn <= 16)
    launch_fwd_t<16, FT, OT>(st, g, L, w, c0, out_rgb, out_depth, out_alpha, out_feat, write_geo, s);
  else if (cn <= 32)
    launch_fwd_t<32, FT, OT>(st, g, L, w, c0, out_rgb, out_depth, out_alpha, out_feat, write_geo, s);
  else
    launch_fwd_t<64, FT, OT>(st, g, L, w, c0, out_rgb, out_depth, out_alpha, out_feat, write_geo, s);
}

hipError_t launch_composite_fwd(const DevGaussians& g, const DevSettings& st, const Layout& L,
                                const WsView& w, float* out_rgb, float* out_depth,
                                float* out_alpha, void* out_feat, int32_t out_feat_dtype,
                                hipStream_t s) {
  const bool feat_on = st.render_features && g.C > 0 && out_feat != nullptr;
  const int64_t HW = (int64_t)L.W * L.H;
  if (!feat_on && out_feat && g.C > 0) {
    const int64_t n = HW * g.C;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (out_feat_dtype == GSFF_DTYPE_BF16)
      hipLaunchKernelGGL(k_fill_zero<uint16_t>, dim3(blocks), dim3(256), 0, s,
                         (uint16_t*)out_feat, n);
    else
      hipLaunchKernelGGL(k_fill_zero<float>, dim3(blocks), dim3(256), 0, s, (float*)out_feat, n);
  }
  const int nchunks = feat_on ? (g.C + GSFF_MAX_CHANNELS_PER_PASS - 1) / GSFF_MAX_CHANNELS_PER_PASS
                              : 1;
  for (int k = 0; k < nchunks; ++k) {
    const int c0 = k * GSFF_MAX_CHANNELS_PER_PASS;
    const int cn = feat_on ? min(GSFF_MAX_CHANNELS_PER_PASS, g.C - c0) : 0;
    const int wg = (k == 0);
    const bool obf = out_feat_dtype == GSFF_DTYPE_BF16;
    if (g.feat_dtype == GSFF_DTYPE_BF16) {
      if (obf)
        launch_fwd_dispatch<uint16_t, uint16_t>(cn, st, g, L, w, c0, out_rgb, out_depth,
                                                out_alpha, out_feat, wg, s);
      else
        launch_fwd_dispatch<uint16_t, float>(cn, st, g, L, w, c0, out_rgb, out_depth, out_alpha,
                                             out_feat, wg, s);
    } else if (g.feat_dtype == GSFF_DTYPE_F16) {
      if (obf)
        launch_fwd_dispatch<_Float16, uint16_t>(cn, st, g, L, w, c0, out_rgb, out_depth,
                                                out_alpha, out_feat, wg, s);
      else
        launch_fwd_dispatch<_Float16, float>(cn, st, g, L, w, c0, out_rgb, out_depth, out_alpha,
                                             out_feat, wg, s);
    } else {
      if (obf)
        launch_fwd_dispatch<float, uint16_t>(cn, st, g, L, w, c0, out_rgb, out_depth, out_alpha,
                                             out_feat, wg, s);
      else
        launch_fwd_dispatch<float, float>(cn, st, g, L, w, c0, out_rgb, out_depth, out_alpha,
                                          out_feat, wg, s);
    }
  }
  return hipGetLastError();
}

// ----------------------------------------------------------- backward -----

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// v + (v from the lane given by a DPP permutation inside each row of 16)
template <int CTRL>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the 16 lanes of a DPP row, result in every lane of the row:
// butterflies over lane^1, lane^2 (quad permutes), then the half-row and
// row mirrors, each pairing a lane with one in the other half it has not
// combined with yet.
__device__ __forceinline__ float row16_allreduce(float v) {
  v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141>(v);  // row_half_mirror
  v = dpp_add<0x140>(v);  // row_mirror
  return v;
}

constexpr int kBwdNB = 16;          // Gaussians per batch (one per DPP row in the contraction)
constexpr int kBwdStride = 272;     // LDS row stride of the per-pixel products (bank spread)

// The per-pixel adjoint of a tile, as a contraction.
//
// Phase A (one thread per pixel, back to front over a batch of kBwdNB
// Gaussians): recover T, and store the blending weight w_ip and
// dL/dpower_ip (zero where the pixel does not use Gaussian i or alpha is
// clamped) in LDS.
// Phase B (thread = (Gaussian i, pixel column)): every per-Gaussian gradient is
// a sum over the tile's pixels of one of these two values times a per-pixel
// constant:
//   colour / depth / feature : sum_p w_ip g_k(p)
//   image-space mean, conic  : sums of dL/dpower_ip times 1, x, y, x^2, xy, y^2
//                              (tile-local pixel coordinates), from which
//                              du, dv, dA, dB, dC follow in closed form
//   opacity                  : sum_p dL/dpower_ip / o_i  (d alpha/d o = G,
//                              d alpha/d power = o G)
// so each column accumulates its 16 pixels and one DPP row reduction
// completes the sum.  Geometry terms come only from the colour, depth and
// opacity upstream; the feature upstream only enters the feature sums.
// Upstream gradient formed inside the adjoint for the L1 losses of the
// method (Eqs. 5, 8, 11 are weighted sums of L1 terms):
//   L = sum_k w_k * mean|out_k - target_k|  over the groups rgb, depth, alpha,
// feature; the per-element gradient is (w_k / numel_k) sign(out - target).
// A group with a NULL target does not enter the loss.
struct L1Upstream {
  const float* out_rgb;
  const float* out_depth;
  const float* out_alpha;
  const float* out_feat;
  const float* t_rgb;
  const float* t_depth;
  const float* t_alpha;
  const float* t_feat;
  float s_rgb, s_depth, s_alpha, s_feat;  // w_k / numel_k
  float* loss;                            // += the loss (may be NULL)
};

__device__ __forceinline__ float l1_sign(float o, float t, float scale, float& l) {
  const float d = o - t;
  l += fabsf(d) * scale;
  return d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
}

template <int CP, bool GEO, bool L1>
__global__ __launch_bounds__(kBlock) void k_composite_bwd(
    DevSettings st, int64_t P, int C, int c0, int W, int H, int tiles_x, int ntiles,
    int rank_bits, uint32_t max_pairs, WsView w, const float* __restrict__ g_rgb,
    const float* __restrict__ g_depth, const float* __restrict__ g_alpha,
    const float* __restrict__ g_feat, float* __restrict__ d_feat, L1Upstream l1) {
  constexpr int NL = (GEO ? 4 : 0) + CP;   // linear channels: r, g, b, depth, features
  constexpr int NLs = NL > 0 ? NL : 1;
  constexpr int NM = GEO ? 6 : 0;          // moments of dL/dpower
  constexpr int NO = NL + NM;
  constexpr int NF = (GEO ? 10 : 0) + CP;  // outputs per Gaussian
  constexpr int NOs = NO > 0 ? NO : 1;
  __shared__ float4 s_r0[kBwdNB], s_r1[kBwdNB], s_r2[kBwdNB];
  __shared__ uint32_t s_gid[kBwdNB];
  __shared__ int s_any[kBwdNB];
  __shared__ float s_w[kBwdNB][kBwdStride];
  __shared__ float s_dp[GEO ? kBwdNB : 1][kBwdStride];
  __shared__ float s_gl[NLs][kBlock];
  __shared__ uint32_t s_end;
  __shared__ float s_loss[kBlock / 64];
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int tid = threadIdx.x;
  const int px = tx * kTile + (tid & (kTile - 1));
  const int py = ty * kTile + (tid / kTile);
  const bool inside = px < W && py < H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 range = clamp_range(w.tile_ranges[tile], max_pairs);
  const uint32_t rmask = (rank_bits >= 32) ? 0xFFFFFFFFu : ((1u << rank_bits) - 1u);
  const int cn = CP > 0 ? min(CP, C - c0) : 0;
  const int64_t HW = (int64_t)W * H;
  const int64_t p = (int64_t)py * W + px;

  // per-pixel state and upstream gradients
  float T = 1.f, Tfin = 1.f;
  uint32_t pend = range.x;
  float gr = 0.f, gg = 0.f, gb = 0.f, gd = 0.f, ga = 0.f;
  float loss = 0.f;
  if (inside) {
    Tfin = w.pix_T[p];
    T = Tfin;
    pend = w.pix_end[p];
    if (GEO) {
      if (L1) {
        if (l1.t_rgb) {
          gr = l1_sign(l1.out_rgb[p], l1.t_rgb[p], l1.s_rgb, loss);
          gg = l1_sign(l1.out_rgb[HW + p], l1.t_rgb[HW + p], l1.s_rgb, loss);
          gb = l1_sign(l1.out_rgb[2 * HW + p], l1.t_rgb[2 * HW + p], l1.s_rgb, loss);
        }
        if (l1.t_depth) gd = l1_sign(l1.out_depth[p], l1.t_depth[p], l1.s_depth, loss);
        if (l1.t_alpha) ga = l1_sign(l1.out_alpha[p], l1.t_alpha[p], l1.s_alpha, loss);
      } else {
        gr = g_rgb[p];
        gg = g_rgb[HW + p];
        gb = g_rgb[2 * HW + p];
        gd = g_depth[p];
        ga = g_alpha[p];
      }
    }
  }
  if (GEO) {
    s_gl[0][tid] = gr;
    s_gl[1][tid] = gg;
    s_gl[2][tid] = gb;
    s_gl[3][tid] = gd;
  }
#pragma unroll
  for (int c = 0; c < CP; ++c) {
    float v = 0.f;
    if (inside && c < cn) {
      const int64_t q = (int64_t)(c0 + c) * HW + p;
      v = L1 ? l1_sign(l1.out_feat[q], l1.t_feat[q], l1.s_feat, loss) : g_feat[q];
    }
    s_gl[(GEO ? 4 : 0) + c][tid] = v;
  }
  if (L1 && l1.loss) {  // uniform: one atomic per workgroup
    const float v = wave_sum(loss);
    if ((tid & 63) == 0) s_loss[tid >> 6] = v;
  }
  if (tid == 0) s_end = range.x;
  __syncthreads();
  if (L1 && l1.loss && tid == 0) {
    const float v = (s_loss[0] + s_loss[1]) + (s_loss[2] + s_loss[3]);
    if (v != 0.f) unsafeAtomicAdd(l1.loss, v);
  }
  if (inside && pend > range.x) atomicMax(&s_end, pend);
  __syncthreads();
  const uint32_t blk_end = min(s_end, range.y);
  float S_r = 0.f, S_g = 0.f, S_b = 0.f, S_d = 0.f;  // sums over the contributors behind

  // phase-B role of this thread
  const int bj = tid >> 4;          // Gaussian slot in the batch (one DPP row)
  const int bq = tid & 15;          // pixel column of the tile
  const float xl = (float)bq + 0.5f - 0.5f * kTile;  // tile-local x of the column
  const float tcx = (float)(tx * kTile) + 0.5f * kTile, tcy = (float)(ty * kTile) + 0.5f * kTile;

  for (uint32_t b1 = blk_end; b1 > range.x;) {
    const uint32_t b0 = (b1 - range.x > (uint32_t)kBwdNB) ? b1 - kBwdNB : range.x;
    const int n = (int)(b1 - b0);
    __syncthreads();  // previous batch fully consumed
    if (tid < n) {
      const uint32_t gid = pair_gid(w, b0 + tid, rmask, P);
      s_gid[tid] = gid;
      load_record(w, gid, P, s_r0[tid], s_r1[tid], s_r2[tid]);
    }
    if (tid < kBwdNB) s_any[tid] = 0;
    __syncthreads();
    // ---- phase A: per-pixel products, back to front
    for (int jj = n - 1; jj >= 0; --jj) {
      const uint32_t j = b0 + (uint32_t)jj;
      const float4 r0 = s_r0[jj], r1 = s_r1[jj];
      float wv = 0.f, dp = 0.f;
      if (inside && j < pend) {
        const AlphaEval e = eval_alpha(r0, r1, pxc, pyc, st.alpha_max);
        if (e.alpha >= st.alpha_min) {
          const float inv = __builtin_amdgcn_rcpf(1.f - e.alpha);  // v_rcp_f32, 1 ulp
          const float Tb = T * inv;  // transmittance in front of this Gaussian
          wv = e.alpha * Tb;
          if constexpr (GEO) {
            const float4 r2 = s_r2[jj];
            const float dal = Tb * (gr * r2.x + gg * r2.y + gb * r2.z + gd * r1.z) -
                              (gr * S_r + gg * S_g + gb * S_b + gd * S_d) * inv + ga * Tfin * inv;
            S_r += wv * r2.x;
            S_g += wv * r2.y;
            S_b += wv * r2.z;
            S_d += wv * r1.z;
            dp = (e.oG < st.alpha_max) ? dal * e.oG : 0.f;
          }
          T = Tb;
          s_any[jj] = 1;
        }
      }
      s_w[jj][tid] = wv;
      if (GEO) s_dp[jj][tid] = dp;
    }
    __syncthreads();
    // ---- phase B: contraction over the tile's pixels, one column per lane
    const bool wave_active =
        __ballot(bj < n && s_any[bj] != 0) != 0ull;  // uniform per wave: skip idle waves
    if (!wave_active) {
      b1 = b0;
      continue;
    }
    float acc[NOs];
#pragma unroll
    for (int k = 0; k < NO; ++k) acc[k] = 0.f;
    if (bj < n && s_any[bj]) {
#pragma unroll 4
      for (int i = 0; i < kTile; ++i) {
        const int pp = i * kTile + bq;
        const float wv = s_w[bj][pp];
#pragma unroll
        for (int k = 0; k < NL; ++k) acc[k] += wv * s_gl[k][pp];
        if constexpr (GEO) {
          const float dp = s_dp[bj][pp];
          const float yl = (float)i + 0.5f - 0.5f * kTile;
          const float dx = dp * xl, dy = dp * yl;
          acc[NL + 0] += dp;
          acc[NL + 1] += dx;
          acc[NL + 2] += dy;
          acc[NL + 3] += dx * xl;
          acc[NL + 4] += dx * yl;
          acc[NL + 5] += dy * yl;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NO; ++k) acc[k] = row16_allreduce(acc[k]);
    // ---- phase C: per-Gaussian outputs, spread over the 16 lanes of the row
    if (bj < n && s_any[bj]) {
      const uint32_t gid = s_gid[bj];
      if (gid < (uint32_t)P) {
        float geo[10];
        if constexpr (GEO) {
          const float4 r0 = s_r0[bj], r1 = s_r1[bj];
          const float ud = r0.x - tcx, vd = r0.y - tcy;  // mean relative to the tile centre
          const float M0 = acc[NL], M1 = acc[NL + 1], M2 = acc[NL + 2];
          const float M3 = acc[NL + 3], M4 = acc[NL + 4], M5 = acc[NL + 5];
          // sums of dL/dpower times (u - x_p), (v - y_p) and their products
          const float Sx = ud * M0 - M1, Sy = vd * M0 - M2;
          const float Sxx = ud * ud * M0 - 2.f * ud * M1 + M3;
          const float Sxy = ud * vd * M0 - ud * M2 - vd * M1 + M4;
          const float Syy = vd * vd * M0 - 2.f * vd * M2 + M5;
          geo[0] = -(r0.z * Sx + r0.w * Sy);
          geo[1] = -(r0.w * Sx + r1.x * Sy);
          geo[2] = -0.5f * Sxx;
          geo[3] = -Sxy;
          geo[4] = -0.5f * Syy;
          geo[5] = r1.y > 0.f ? M0 / r1.y : 0.f;
          geo[6] = acc[0];
          geo[7] = acc[1];
          geo[8] = acc[2];
          geo[9] = acc[3];
        }
#pragma unroll
        for (int f0 = 0; f0 < NF; f0 += 16) {
          const int f = f0 + bq;
          if (f >= NF) break;
          if (GEO && f < 10) {  // geometry slots exist only when GEO
            float v = 0.f;
#pragma unroll
            for (int k = 0; k < 10; ++k) v = (k == f) ? geo[k] : v;
            if (v != 0.f) unsafeAtomicAdd(&w.grad2d[(int64_t)gid * 10 + f], v);
          } else {
            const int c = f - (GEO ? 10 : 0);
            float v = 0.f;
#pragma unroll
            for (int k = 0; k < CP; ++k) v = (k == c) ? acc[(GEO ? 4 : 0) + k] : v;
            if (c < cn && v != 0.f) unsafeAtomicAdd(&d_feat[(int64_t)gid * C + c0 + c], v);
          }
        }
      }
    }
    b1 = b0;
  }
}

template <int CP, bool GEO, bool L1>
static void launch_bwd_t(const DevSettings& st, const DevGaussians& g, const Layout& L,
                         const WsView& w, int c0, const float* g_rgb, const float* g_depth,
                         const float* g_alpha, const float* g_feat, float* d_feat,
                         const L1Upstream& l1, hipStream_t s) {
  const int grid = ((L.ntiles + kNumXcd - 1) / kNumXcd) * kNumXcd;
  hipLaunchKernelGGL((k_composite_bwd<CP, GEO, L1>), dim3(grid), dim3(kBlock), 0, s, st, g.P,
                     g.C, c0, L.W, L.H, L.tiles_x, L.ntiles, L.rank_bits, (uint32_t)L.max_pairs,
                     w, g_rgb, g_depth, g_alpha, g_feat, d_feat, l1);
}

template <bool GEO, bool L1>
static void launch_bwd_dispatch(int cn, const DevSettings& st, const DevGaussians& g,
                                const Layout& L, const WsView& w, int c0, const float* g_rgb,
                                const float* g_depth, const float* g_alpha, const float* g_feat,
                                float* d_feat, const L1Upstream& l1, hipStream_t s) {
  if (cn <= 0)
    launch_bwd_t<0, GEO, L1>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, l1, s);
  else if (cn <= 8)
    launch_bwd_t<8, GEO, L1>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, l1, s);
  else if (cn <= 16)
    launch_bwd_t<16, GEO, L1>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, l1, s);
  else if (cn <= 32)
    launch_bwd_t<32, GEO, L1>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, l1, s);
  else
    launch_bwd_t<64, GEO, L1>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, l1, s);
}

// l1 == nullptr: explicit upstream gradients; otherwise the L1 upstream is
// formed inside the kernel (feature group on iff l1->t_feat is set).
hipError_t launch_composite_bwd_impl(const DevGaussians& g, const DevSettings& st,
                                     const Layout& L, const WsView& w, const float* g_rgb,
                                     const float* g_depth, const float* g_alpha,
                                     const float* g_feat, bool geometry, float* d_feat,
                                     int32_t accumulate, const L1Upstream* l1, hipStream_t s) {
  const bool has_gf = l1 ? (l1->t_feat != nullptr && l1->out_feat != nullptr) : g_feat != nullptr;
  const bool feat_on = st.render_features && g.C > 0 && has_gf && d_feat != nullptr;
  if (geometry && L.P > 0) {
    const int64_t n = L.P * 10;
    hipLaunchKernelGGL(k_fill_zero<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       w.grad2d, n);
  }
  if (d_feat && !accumulate && L.P > 0 && g.C > 0) {
    const int64_t n = L.P * g.C;
    hipLaunchKernelGGL(k_fill_zero<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       d_feat, n);
  }
  L1Upstream none{};
  const L1Upstream& u = l1 ? *l1 : none;
  const int nchunks = feat_on ? (g.C + GSFF_MAX_CHANNELS_PER_PASS - 1) / GSFF_MAX_CHANNELS_PER_PASS
                              : 1;
  for (int k = 0; k < nchunks; ++k) {
    const int c0 = k * GSFF_MAX_CHANNELS_PER_PASS;
    const int cn = feat_on ? min(GSFF_MAX_CHANNELS_PER_PASS, g.C - c0) : 0;
    // the geometry chunk also carries the rgb / depth / alpha loss terms
    const bool geo = geometry && k == 0;
    if (!geo && cn == 0) continue;
    if (L.P == 0 && !l1) continue;
    if (l1) {
      if (geo)
        launch_bwd_dispatch<true, true>(cn, st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat,
                                        d_feat, u, s);
      else
        launch_bwd_dispatch<false, true>(cn, st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat,
                                         d_feat, u, s);
    } else {
      if (geo)
        launch_bwd_dispatch<true, false>(cn, st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat,
                                         d_feat, u, s);
      else
        launch_bwd_dispatch<false, false>(cn, st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat,
                                          d_feat, u, s);
    }
  }
  return hipGetLastError();
}

hipError_t launch_composite_bwd(const DevGaussians& g, const DevSettings& st, const Layout& L,
                                const WsView& w, const float* g_rgb, const float* g_depth,
                                const float* g_alpha, const float* g_feat, bool geometry,
                                float* d_feat, int32_t accumulate, hipStream_t s) {
  return launch_composite_bwd_impl(g, st, L, w, g_rgb, g_depth, g_alpha, g_feat, geometry, d_feat,
                                   accumulate, nullptr, s);
}

hipError_t launch_composite_bwd_l1(const DevGaussians& g, const DevSettings& st, const Layout& L,
                                   const WsView& w, const L1Args& a, bool geometry, float* d_feat,
                                   int32_t accumulate, hipStream_t s) {
  const double HW = (double)L.W * L.H;
  L1Upstream u;
  u.out_rgb = a.out_rgb;
  u.out_depth = a.out_depth;
  u.out_alpha = a.out_alpha;
  u.out_feat = a.out_feat;
  u.t_rgb = a.t_rgb;
  u.t_depth = a.t_depth;
  u.t_alpha = a.t_alpha;
  u.t_feat = a.t_feat;
  u.s_rgb = (float)(a.w_rgb / (3.0 * HW));
  u.s_depth = (float)(a.w_depth / HW);
  u.s_alpha = (float)(a.w_alpha / HW);
  u.s_feat = (float)(g.C > 0 ? a.w_feat / ((double)g.C * HW) : 0.0);
  u.loss = a.loss;
  return launch_composite_bwd_impl(g, st, L, w, nullptr, nullptr, nullptr, nullptr, geometry,
                                   d_feat, accumulate, &u, s);
}

// ---------------------------------------------------------------- L1 ------

__device__ __forceinline__ float l1_elem(float x, float y, float scale, float& l) {
  const float d = x - y;
  l += fabsf(d);
  return d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
}

// grad = scale * sign(x - y), loss += scale * sum |x - y|.  VEC: four
// elements per thread per step (16-byte loads and stores) plus a scalar tail;
// grid-stride, one loss atomic per workgroup.
template <bool VEC>
__global__ __launch_bounds__(256) void k_l1_grad(const float* __restrict__ x,
                                                 const float* __restrict__ y, int64_t n,
                                                 float scale, float* __restrict__ grad,
                                                 float* __restrict__ loss) {
  __shared__ float s_part[4];
  float l = 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t done = 0;
  if (VEC) {
    const int64_t n4 = n / 4;
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const float4* y4 = reinterpret_cast<const float4*>(y);
    float4* g4 = reinterpret_cast<float4*>(grad);
    for (int64_t i = t0; i < n4; i += stride) {
      const float4 a = x4[i], b = y4[i];
      float4 g;
      g.x = l1_elem(a.x, b.x, scale, l);
      g.y = l1_elem(a.y, b.y, scale, l);
      g.z = l1_elem(a.z, b.z, scale, l);
      g.w = l1_elem(a.w, b.w, scale, l);
      g4[i] = g;
    }
    done = 4 * n4;
  }
  for (int64_t i = done + t0; i < n; i += stride) grad[i] = l1_elem(x[i], y[i], scale, l);
  if (!loss) return;  // uniform
  l = wave_sum(l);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float t = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
    if (t != 0.f) unsafeAtomicAdd(loss, t * scale);
  }
}

hipError_t launch_l1_grad(const float* x, const float* y, int64_t n, float scale, float* grad,
                          float* loss, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const bool aligned = (((uintptr_t)x | (uintptr_t)y | (uintptr_t)grad) & 15u) == 0;
  int64_t blocks = (n + 1023) / 1024;
  if (blocks > 2048) blocks = 2048;  // grid-stride; bounds the loss atomics
  if (aligned)
    hipLaunchKernelGGL(k_l1_grad<true>, dim3((unsigned)blocks), dim3(256), 0, s, x, y, n, scale,
                       grad, loss);
  else
    hipLaunchKernelGGL(k_l1_grad<false>, dim3((unsigned)blocks), dim3(256), 0, s, x, y, n, scale,
                       grad, loss);
  return hipGetLastError();
}

}  // namespace gsff
