// Preprocess (projection, culling, support rectangle, depth key) and its
// adjoint with the Lie-algebra pose gradient (Sec. 3.1 Eq. 1; Sec. 3.2 Eq. 4).
//
// One thread per Gaussian, planar [k, P] loads so every wave reads whole
// cache lines; the adjoint recomputes the forward quantities instead of
// storing them.
#include <hip/hip_runtime.h>

#include "gsff_internal.h"
#include "project.h"

namespace gsff {

// Support rectangle margin in pixels: the FP32 bound is widened by this much
// so that no pixel whose alpha reaches alpha_min in exact arithmetic is left
// outside a Gaussian's tiles by rounding.
constexpr float kRectMargin = 0.05f;

__global__ __launch_bounds__(256) void k_preprocess(DevGaussians g, DevCamera cam,
                                                    DevSettings st, WsView w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {  // the whole status word: later stages read the pair count from it
#pragma unroll
    for (int k = 0; k < 8; ++k) w.status[k] = 0u;
  }
  const int64_t P = g.P;
  uint32_t ntile = 0;  // tiles of the support rectangle
  if (i < P) {
  float V[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) V[k] = cam.viewmat[k];
  const Proj p = project_gaussian(g, cam, st, V, i);
  ushort4 rect = make_ushort4(1, 1, 0, 0);  // empty: x0 > x1
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0;
  if (p.valid) {
    // exact half-widths of { alpha >= alpha_min } = { d^T K d <= 2 ln(o/alpha_min) }
    const float k2 = 2.f * logf(p.o / st.alpha_min);
    const float rx = sqrtf(fmaxf(k2, 0.f) * p.a);
    const float ry = sqrtf(fmaxf(k2, 0.f) * p.c);
    // pixel px is covered when |px + 1/2 - u| <= rx
    float fx0 = ceilf(p.u - rx - 0.5f - kRectMargin);
    float fx1 = floorf(p.u + rx - 0.5f + kRectMargin);
    float fy0 = ceilf(p.v - ry - 0.5f - kRectMargin);
    float fy1 = floorf(p.v + ry - 0.5f + kRectMargin);
    fx0 = fmaxf(fx0, 0.f);
    fy0 = fmaxf(fy0, 0.f);
    fx1 = fminf(fx1, (float)(cam.W - 1));
    fy1 = fminf(fy1, (float)(cam.H - 1));
    if (fx0 <= fx1 && fy0 <= fy1) {
      rect = make_ushort4((unsigned short)((int)fx0 / kTile), (unsigned short)((int)fy0 / kTile),
                          (unsigned short)((int)fx1 / kTile), (unsigned short)((int)fy1 / kTile));
    }
    r0 = make_float4(p.u, p.v, p.A, p.B);
    r1 = make_float4(p.Cc, p.o, p.z, 1.f);
  }
  const float4 r2 = make_float4(g.rgb[i], g.rgb[P + i], g.rgb[2 * P + i], 0.f);
  w.rec[i] = r0;
  w.rec[P + i] = r1;
  w.rec[2 * P + i] = r2;
  w.rects[i] = rect;
  // the image-space gradients the compositing adjoint accumulates start at
  // zero, and the Gaussian's list of adjoint rows empty
  float* d2 = w.grad2d + i * 10;
#pragma unroll
  for (int k = 0; k < 10; ++k) d2[k] = 0.f;
  w.nslot[i] = 0u;
  if (i == 0) *w.item_n = 0u;
  // culled Gaussians keep the largest key and an empty rectangle
  w.dkeys_a[i] = (p.valid && rect.x <= rect.z) ? p.key : 0xFFFFFFFFu;
  w.dids_a[i] = (uint32_t)i;
  if (rect.x <= rect.z && rect.y <= rect.w)
    ntile = (uint32_t)(rect.z - rect.x + 1) * (uint32_t)(rect.w - rect.y + 1);
  }
  // slots for the adjoint: a Gaussian gets one per tile of its rectangle;
  // block-local exclusive offsets and the block's count here, the block bases
  // in the adjoint's set-up (a scan of the counts, repeated by every adjoint)
  __shared__ uint32_t s_ws[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = ntile;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  if (lane == 63) s_ws[wv] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k < wv) pre += s_ws[k];
    tot += s_ws[k];
  }
  if (i < P) w.slot_local[i] = pre + inc - ntile;
  if (threadIdx.x == 0) w.slot_cnt[blockIdx.x] = tot;
}

// Sum of the adjoint rows, one wave per work item (a Gaussian and 64 of its
// slots).  The lanes form 64/CW groups of CW columns; each group takes every
// (64/CW)-th row of the item, so every row load of the item is in flight at
// once, and a butterfly adds the groups.  Image terms go to grad2d (+=, which
// the preprocess adjoint then consumes), features to d_feat (+=) when given; a
// Gaussian with more than 64 slots has several items, which add atomically.
template <int CW>
__global__ __launch_bounds__(256) void k_adjoint_reduce(WsView w, int64_t P, int C,
                                                        float* __restrict__ d_feat,
                                                        uint32_t max_pairs) {
  constexpr int RPI = 64 / CW;  // rows side by side in one load
  const int lane = threadIdx.x & 63;
  const int cl = lane & (CW - 1), rsub = lane / CW;
  uint32_t cnt = *w.item_n;
  if (cnt > w.item_cap) cnt = w.item_cap;
  const int RW = w.row_width;
  const int ncol = 10 + (d_feat ? C : 0);
  const uint32_t nw = gridDim.x * 4u;
  for (uint32_t e = blockIdx.x * 4u + (threadIdx.x >> 6); e < cnt; e += nw) {
    const uint2 it = w.items[e];
    const uint32_t gg = it.x, k0 = it.y;
    if (!guard(w.status, GSFF_CHECK_REDUCE, gg, (uint64_t)P)) continue;
    const uint32_t n = w.nslot[gg];
    if (!guard(w.status, GSFF_CHECK_REDUCE, k0, n)) continue;
    const uint32_t m = n - k0 < 64u ? n - k0 : 64u;
    const uint32_t sl = w.slot_blk[gg >> 8] + w.slot_local[gg] + k0 + (uint32_t)lane;
    const uint32_t myrow =
        ((uint32_t)lane < m && guard(w.status, GSFF_CHECK_SLOT, sl, w.slot_cap)) ? w.slots[sl]
                                                                               : 0xFFFFFFFFu;
    // every filed slot holds a row
    if (GSFF_CHECKED && (uint32_t)lane < m) GSFF_CHECK(w.status, GSFF_CHECK_REDUCE, myrow, w.row_cap);
    const bool single = n <= 64u;
    for (int c0 = 0; c0 < ncol; c0 += CW) {
      const int col = c0 + cl;
      float acc = 0.f;
#pragma unroll
      for (int u = 0; u < 64 / RPI; ++u) {
        const int j = u * RPI + rsub;
        const uint32_t r = (uint32_t)__shfl((int)myrow, j, 64);
        const bool ok = r < w.row_cap && col < ncol;
        const float v = w.rows[ok ? (int64_t)r * RW + col : 0];
        acc += ok ? v : 0.f;
      }
#pragma unroll
      for (int off = CW; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
      if (rsub == 0 && col < ncol && acc != 0.f) {
        float* dst = col < 10 ? w.grad2d + (int64_t)gg * 10 + col
                              : d_feat + (int64_t)gg * C + (col - 10);
        if (single) *dst += acc;
        else unsafeAtomicAdd(dst, acc);
      }
    }
  }
}

// Adjoint of project_gaussian followed by the pose terms of Eq. 4.
__global__ __launch_bounds__(kPoseBlock) void k_preprocess_bwd(DevGaussians g, DevCamera cam,
                                                               DevSettings st, WsView w,
                                                               gsff_grads out, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t P = g.P;
  float V[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) V[k] = cam.viewmat[k];
  float pose[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (i < P) {
    // consume the image-space gradients (the adjoint reduction has added
    // the per-tile rows) and re-arm them at zero, so another adjoint of the
    // same forward starts from nothing
    float* d2 = w.grad2d + i * 10;
    float d[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) d[k] = d2[k];
    bool any = false;
#pragma unroll
    for (int k = 0; k < 10; ++k) any |= d[k] != 0.f;
    w.nslot[i] = 0u;
    if (i == 0) *w.item_n = 0u;
    float dmean[3] = {0.f, 0.f, 0.f}, dls[3] = {0.f, 0.f, 0.f}, dq[4] = {0.f, 0.f, 0.f, 0.f};
    float dlogit = 0.f;
    const float drgb[3] = {d[6], d[7], d[8]};
    // every term is linear in the image-space gradients: a Gaussian no tile
    // walked (most of a frame's) has zero gradients without the projection
    if (any) {
#pragma unroll
      for (int k = 0; k < 10; ++k) d2[k] = 0.f;
      const Proj p = project_gaussian(g, cam, st, V, i);
      if (p.valid) project_adjoint<float>(p, V, cam.fx, cam.fy, d, dmean, dls, dq, dlogit, pose);
    }
    if (accumulate) {
      if (out.means)
        for (int k = 0; k < 3; ++k) out.means[k * P + i] += dmean[k];
      if (out.log_scales)
        for (int k = 0; k < 3; ++k) out.log_scales[k * P + i] += dls[k];
      if (out.quats)
        for (int k = 0; k < 4; ++k) out.quats[k * P + i] += dq[k];
      if (out.logit_opacity) out.logit_opacity[i] += dlogit;
      if (out.rgb)
        for (int k = 0; k < 3; ++k) out.rgb[k * P + i] += drgb[k];
    } else {
      if (out.means)
        for (int k = 0; k < 3; ++k) out.means[k * P + i] = dmean[k];
      if (out.log_scales)
        for (int k = 0; k < 3; ++k) out.log_scales[k * P + i] = dls[k];
      if (out.quats)
        for (int k = 0; k < 4; ++k) out.quats[k * P + i] = dq[k];
      if (out.logit_opacity) out.logit_opacity[i] = dlogit;
      if (out.rgb)
        for (int k = 0; k < 3; ++k) out.rgb[k * P + i] = drgb[k];
    }
  }
  if (!out.pose) return;
  // block reduction of the six pose terms in FP64 (fixed order)
  __shared__ double s_red[kPoseBlock / 64][6];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = 0; k < 6; ++k) {
    double v = (double)pose[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) s_red[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double acc = 0.0;
    for (int j = 0; j < kPoseBlock / 64; ++j) acc += s_red[j][threadIdx.x];
    w.pose_part[blockIdx.x * 6 + threadIdx.x] = acc;
  }
}

// Sum the per-block pose partials (a separate launch: a last-workgroup
// reduction would need a device-scope fence in every workgroup, which writes
// back the L2 of each XCD).  Each thread accumulates whole 6-double records;
// the block reduction runs in a fixed order, so the result is deterministic.
__global__ __launch_bounds__(256) void k_pose_final(const double* __restrict__ part, int nblocks,
                                                    float* pose, int accumulate) {
  __shared__ double s_red[4][6];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += 256)
    for (int k = 0; k < 6; ++k) acc[k] += part[b * 6 + k];
  for (int k = 0; k < 6; ++k) {
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) s_red[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const double v = (s_red[0][threadIdx.x] + s_red[1][threadIdx.x]) +
                     (s_red[2][threadIdx.x] + s_red[3][threadIdx.x]);
    pose[threadIdx.x] = accumulate ? pose[threadIdx.x] + (float)v : (float)v;
  }
}

// Deterministic mode: one wave per Gaussian sums the rows in the slots of
// its rectangle in slot order (a tile's row sits in the slot of the tile's
// place in the rectangle; empty slots hold 0xFFFFFFFF), 64 slots at a time
// with the lane groups of k_adjoint_reduce, adding the chunks in order: the
// same inputs give the same bits, whatever order the rows were written in.
template <int CW>
__global__ __launch_bounds__(256) void k_adjoint_reduce_det(WsView w, int64_t P, int C,
                                                            float* __restrict__ d_feat) {
  constexpr int RPI = 64 / CW;
  const int lane = threadIdx.x & 63;
  const int cl = lane & (CW - 1), rsub = lane / CW;
  const int64_t gg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gg >= P) return;  // whole wave
  const ushort4 rc = w.rects[gg];
  const uint32_t ntile = (rc.x <= rc.z && rc.y <= rc.w)
                             ? (uint32_t)(rc.z - rc.x + 1) * (uint32_t)(rc.w - rc.y + 1)
                             : 0u;
  if (ntile == 0u) return;  // whole wave
  const uint32_t base = w.slot_blk[gg >> 8] + w.slot_local[gg];
  const int RW = w.row_width;
  const int ncol = 10 + (d_feat ? C : 0);
  for (int c0 = 0; c0 < ncol; c0 += CW) {
    const int col = c0 + cl;
    float tot = 0.f;
    for (uint32_t k0 = 0; k0 < ntile; k0 += 64) {
      const uint32_t sl = base + k0 + (uint32_t)lane;
      const uint32_t myrow =
          (k0 + (uint32_t)lane < ntile && guard(w.status, GSFF_CHECK_SLOT, sl, w.slot_cap))
              ? w.slots[sl]
              : 0xFFFFFFFFu;
      // a slot holds a row, or nothing (a tile whose walk ended in front of the Gaussian)
      if (GSFF_CHECKED && myrow != 0xFFFFFFFFu) GSFF_CHECK(w.status, GSFF_CHECK_REDUCE, myrow, w.row_cap);
      float acc = 0.f;
#pragma unroll
      for (int u = 0; u < 64 / RPI; ++u) {
        const int j = u * RPI + rsub;
        const uint32_t r = (uint32_t)__shfl((int)myrow, j, 64);
        const bool ok = r < w.row_cap && col < ncol;
        const float v = w.rows[ok ? (int64_t)r * RW + col : 0];
        acc += ok ? v : 0.f;
      }
#pragma unroll
      for (int off = CW; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
      tot += acc;
    }
    if (rsub == 0 && col < ncol && tot != 0.f) {
      float* dst = col < 10 ? w.grad2d + gg * 10 + col : d_feat + gg * C + (col - 10);
      *dst += tot;
    }
  }
}

hipError_t launch_preprocess(const DevGaussians& g, const DevCamera& cam, const DevSettings& st,
                             const Layout& L, const WsView& w, hipStream_t s) {
  const int64_t blocks = g.P > 0 ? (g.P + 255) / 256 : 1;
  hipLaunchKernelGGL(k_preprocess, dim3((unsigned)blocks), dim3(256), 0, s, g, cam, st, w);
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const DevGaussians& g, const DevCamera& cam,
                                 const DevSettings& st, const Layout& L, const WsView& w,
                                 const gsff_grads& out, int32_t accumulate, hipStream_t s) {
  if (g.P > 0) {
    float* df = g.C > 0 ? out.feat : nullptr;
    const int ncol = 10 + (df ? g.C : 0);
    // one wave per possible item, up to 8192 waves: each item's loads are a
    // dependent chain, so the reduction is bound by how many are in flight
    const unsigned nblk =
        (unsigned)std::min<int64_t>(std::max<int64_t>((L.item_cap + 3) / 4, 1), 2048);
    const unsigned ndet = (unsigned)((g.P + 3) / 4);  // one wave per Gaussian
    if (st.deterministic) {
      if (ncol <= 16)
        hipLaunchKernelGGL(k_adjoint_reduce_det<16>, dim3(ndet), dim3(256), 0, s, w, g.P, g.C, df);
      else if (ncol <= 32)
        hipLaunchKernelGGL(k_adjoint_reduce_det<32>, dim3(ndet), dim3(256), 0, s, w, g.P, g.C, df);
      else
        hipLaunchKernelGGL(k_adjoint_reduce_det<64>, dim3(ndet), dim3(256), 0, s, w, g.P, g.C, df);
    } else if (ncol <= 16)
      hipLaunchKernelGGL(k_adjoint_reduce<16>, dim3(nblk), dim3(256), 0, s, w, g.P, g.C, df,
                         (uint32_t)L.max_pairs);
    else if (ncol <= 32)
      hipLaunchKernelGGL(k_adjoint_reduce<32>, dim3(nblk), dim3(256), 0, s, w, g.P, g.C, df,
                         (uint32_t)L.max_pairs);
    else
      hipLaunchKernelGGL(k_adjoint_reduce<64>, dim3(nblk), dim3(256), 0, s, w, g.P, g.C, df,
                         (uint32_t)L.max_pairs);
    hipLaunchKernelGGL(k_preprocess_bwd, dim3((unsigned)L.pose_blocks), dim3(kPoseBlock), 0, s,
                       g, cam, st, w, out, (int)accumulate);
  }
  if (out.pose)
    hipLaunchKernelGGL(k_pose_final, dim3(1), dim3(256), 0, s, w.pose_part,
                       (int)(g.P > 0 ? L.pose_blocks : 0), out.pose, (int)accumulate);
  return hipGetLastError();
}

}  // namespace gsff
