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

// Gaussian id of sorted pair `idx`; returns P (an out-of-range marker) if
// the stored rank or id is not a valid index, so no gather can leave the
// record arrays.
__device__ __forceinline__ uint32_t pair_gid(const WsView& w, uint32_t idx, uint32_t rmask,
                                             int64_t P) {
  const uint32_t rank = w.pkeys_a[idx] & rmask;
  if (rank >= (uint32_t)P) return (uint32_t)P;
  const uint32_t gid = w.dids_a[rank];
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
    int rank_bits, WsView w, const FT* __restrict__ feat, float* __restrict__ out_rgb,
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
  const uint2 range = w.tile_ranges[tile];
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
                     c0, L.W, L.H, L.tiles_x, L.ntiles, L.rank_bits, w,
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

// GEO: compute the geometry adjoint (10 image-space values per Gaussian);
// CP: feature channels whose gradient is accumulated (0 = none).
template <int CP, bool GEO>
__global__ __launch_bounds__(kBlock) void k_composite_bwd(
    DevSettings st, int64_t P, int C, int c0, int W, int H, int tiles_x, int ntiles,
    int rank_bits, WsView w, const float* __restrict__ g_rgb, const float* __restrict__ g_depth,
    const float* __restrict__ g_alpha, const float* __restrict__ g_feat,
    float* __restrict__ d_feat) {
  constexpr int NG = (GEO ? 10 : 0) + CP;
  constexpr int NGs = NG > 0 ? NG : 1;
  constexpr int CPs = CP > 0 ? CP : 1;
  __shared__ float4 s_r0[kBwdBatch], s_r1[kBwdBatch], s_r2[kBwdBatch];
  __shared__ uint32_t s_gid[kBwdBatch];
  __shared__ float s_grad[kBwdBatch][NGs];
  __shared__ uint32_t s_end;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int px = tx * kTile + (threadIdx.x & (kTile - 1));
  const int py = ty * kTile + (threadIdx.x / kTile);
  const bool inside = px < W && py < H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 range = w.tile_ranges[tile];
  const uint32_t rmask = (rank_bits >= 32) ? 0xFFFFFFFFu : ((1u << rank_bits) - 1u);
  const int cn = CP > 0 ? min(CP, C - c0) : 0;
  const int64_t HW = (int64_t)W * H;
  const int64_t p = (int64_t)py * W + px;

  float T = 1.f, Tfin = 1.f;
  uint32_t pend = range.x;
  float gr = 0.f, gg = 0.f, gb = 0.f, gd = 0.f, ga = 0.f;
  float gf[CPs];
#pragma unroll
  for (int c = 0; c < CPs; ++c) gf[c] = 0.f;
  if (inside) {
    Tfin = w.pix_T[p];
    T = Tfin;
    pend = w.pix_end[p];
    if (GEO) {
      gr = g_rgb[p];
      gg = g_rgb[HW + p];
      gb = g_rgb[2 * HW + p];
      gd = g_depth[p];
      ga = g_alpha[p];
    }
#pragma unroll
    for (int c = 0; c < CP; ++c) gf[c] = (c < cn) ? g_feat[(int64_t)(c0 + c) * HW + p] : 0.f;
  }
  if (threadIdx.x == 0) s_end = range.x;
  __syncthreads();
  if (inside && pend > range.x) atomicMax(&s_end, pend);
  __syncthreads();
  const uint32_t blk_end = min(s_end, range.y);
  const int lane = threadIdx.x & 63;
  float S_r = 0.f, S_g = 0.f, S_b = 0.f, S_d = 0.f;  // suffix sums behind the current Gaussian

  for (uint32_t b1 = blk_end; b1 > range.x;) {
    const uint32_t b0 = (b1 - range.x > (uint32_t)kBwdBatch) ? b1 - kBwdBatch : range.x;
    const uint32_t n = b1 - b0;
    __syncthreads();  // previous batch fully consumed
    if (threadIdx.x < n) {
      const uint32_t gid = pair_gid(w, b0 + threadIdx.x, rmask, P);
      s_gid[threadIdx.x] = gid;
      load_record(w, gid, P, s_r0[threadIdx.x], s_r1[threadIdx.x], s_r2[threadIdx.x]);
    }
    for (int e = threadIdx.x; e < kBwdBatch * NGs; e += kBlock) (&s_grad[0][0])[e] = 0.f;
    __syncthreads();
    for (int jj = (int)n - 1; jj >= 0; --jj) {
      const uint32_t j = b0 + (uint32_t)jj;
      const float4 r0 = s_r0[jj], r1 = s_r1[jj];
      bool contrib = inside && j < pend;
      AlphaEval e;
      e.alpha = 0.f;
      if (contrib) {
        e = eval_alpha(r0, r1, pxc, pyc, st.alpha_max);
        contrib = e.alpha >= st.alpha_min;
      }
      if (__ballot(contrib) == 0ull) continue;  // nothing for this wave
      float gv[NGs];
#pragma unroll
      for (int k = 0; k < NGs; ++k) gv[k] = 0.f;
      if (contrib) {
        const float om = 1.f - e.alpha;
        const float inv = 1.f / om;
        const float Tb = T * inv;  // transmittance in front of this Gaussian
        const float wgt = e.alpha * Tb;
        if (GEO) {
          const float4 r2 = s_r2[jj];
          const float dal = Tb * (gr * r2.x + gg * r2.y + gb * r2.z + gd * r1.z) -
                            (gr * S_r + gg * S_g + gb * S_b + gd * S_d) * inv + ga * Tfin * inv;
          S_r += wgt * r2.x;
          S_g += wgt * r2.y;
          S_b += wgt * r2.z;
          S_d += wgt * r1.z;
          if (e.oG < st.alpha_max) {
            const float dpow = dal * e.oG;
            gv[0] = -dpow * (r0.z * e.dx + r0.w * e.dy);
            gv[1] = -dpow * (r0.w * e.dx + r1.x * e.dy);
            gv[2] = -0.5f * dpow * e.dx * e.dx;
            gv[3] = -dpow * e.dx * e.dy;
            gv[4] = -0.5f * dpow * e.dy * e.dy;
            gv[5] = dal * e.G;
          }
          gv[6] = wgt * gr;
          gv[7] = wgt * gg;
          gv[8] = wgt * gb;
          gv[9] = wgt * gd;
        }
#pragma unroll
        for (int c = 0; c < CP; ++c) gv[(GEO ? 10 : 0) + c] = wgt * gf[c];
        T = Tb;
      }
#pragma unroll
      for (int k = 0; k < NG; ++k) {
        const float v = wave_sum(gv[k]);
        if (lane == 0 && v != 0.f) atomicAdd(&s_grad[jj][k], v);
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < (int)n * NG; e += kBlock) {
      const int jj = e / NGs, k = e % NGs;
      const float v = s_grad[jj][k];
      if (v == 0.f) continue;
      const uint32_t gid = s_gid[jj];
      if (gid >= (uint32_t)P) continue;
      if (GEO && k < 10)
        unsafeAtomicAdd(&w.grad2d[(int64_t)gid * 10 + k], v);
      else {
        const int c = k - (GEO ? 10 : 0);
        if (c < cn) unsafeAtomicAdd(&d_feat[(int64_t)gid * C + c0 + c], v);
      }
    }
    b1 = b0;
  }
}

template <int CP, bool GEO>
static void launch_bwd_t(const DevSettings& st, const DevGaussians& g, const Layout& L,
                         const WsView& w, int c0, const float* g_rgb, const float* g_depth,
                         const float* g_alpha, const float* g_feat, float* d_feat,
                         hipStream_t s) {
  const int grid = ((L.ntiles + kNumXcd - 1) / kNumXcd) * kNumXcd;
  hipLaunchKernelGGL((k_composite_bwd<CP, GEO>), dim3(grid), dim3(kBlock), 0, s, st, g.P, g.C, c0,
                     L.W, L.H, L.tiles_x, L.ntiles, L.rank_bits, w, g_rgb, g_depth, g_alpha,
                     g_feat, d_feat);
}

template <bool GEO>
static void launch_bwd_dispatch(int cn, const DevSettings& st, const DevGaussians& g,
                                const Layout& L, const WsView& w, int c0, const float* g_rgb,
                                const float* g_depth, const float* g_alpha, const float* g_feat,
                                float* d_feat, hipStream_t s) {
  if (cn <= 0)
    launch_bwd_t<0, GEO>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, s);
  else if (cn <= 8)
    launch_bwd_t<8, GEO>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, s);
  else if (cn <= 16)
    launch_bwd_t<16, GEO>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, s);
  else if (cn <= 32)
    launch_bwd_t<32, GEO>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, s);
  else
    launch_bwd_t<64, GEO>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, s);
}

hipError_t launch_composite_bwd(const DevGaussians& g, const DevSettings& st, const Layout& L,
                                const WsView& w, const float* g_rgb, const float* g_depth,
                                const float* g_alpha, const float* g_feat, bool geometry,
                                float* d_feat, int32_t accumulate, hipStream_t s) {
  const bool feat_on = st.render_features && g.C > 0 && g_feat != nullptr && d_feat != nullptr;
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
  if (L.P == 0) return hipGetLastError();
  const int nchunks = feat_on ? (g.C + GSFF_MAX_CHANNELS_PER_PASS - 1) / GSFF_MAX_CHANNELS_PER_PASS
                              : 1;
  for (int k = 0; k < nchunks; ++k) {
    const int c0 = k * GSFF_MAX_CHANNELS_PER_PASS;
    const int cn = feat_on ? min(GSFF_MAX_CHANNELS_PER_PASS, g.C - c0) : 0;
    const bool geo = geometry && k == 0;
    if (!geo && cn == 0) continue;
    if (geo)
      launch_bwd_dispatch<true>(cn, st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, s);
    else
      launch_bwd_dispatch<false>(cn, st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, s);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- L1 ------

__global__ __launch_bounds__(256) void k_l1_grad(const float* __restrict__ x,
                                                 const float* __restrict__ y, int64_t n,
                                                 float scale, float* __restrict__ grad,
                                                 float* __restrict__ loss) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < n) {
    const float d = x[i] - y[i];
    grad[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
    l = fabsf(d) * scale;
  }
  if (loss) {
    l = wave_sum(l);
    if ((threadIdx.x & 63) == 0 && l != 0.f) unsafeAtomicAdd(loss, l);
  }
}

hipError_t launch_l1_grad(const float* x, const float* y, int64_t n, float scale, float* grad,
                          float* loss, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_l1_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n, scale,
                     grad, loss);
  return hipGetLastError();
}

}  // namespace gsff
