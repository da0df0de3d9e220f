// FP64 instantiation of the rendering path and its adjoint, for derivative
// checks by central finite differences on small scenes.
//
// The projection (Sec. 3.1, Eq. 1 and its perspective splat) and its adjoint
// with the pose terms (Sec. 3.2, Eq. 4) are project_core / project_adjoint,
// the templated device code the FP32 preprocess kernels run.  The adjoint of
// the blending (Eqs. 2-3) runs back_step per pair and geo_from_moments per
// (tile, Gaussian), as the FP32 compositing adjoint does; the sums the FP32
// kernels take over a tile's pixels on the matrix cores are plain FP64 block
// reductions here.  Every Gaussian is tested against every pixel (no
// binning: the FP32 path's tile lists only leave out pairs with alpha below
// alpha_min), in the FP32 path's depth order.  Slow by design.
#include <hip/hip_runtime.h>

#include "blend.h"
#include "gsff_internal.h"
#include "project.h"

namespace gsff {

namespace {

constexpr int kF64MaxP = 4096;
constexpr int kF64MaxC = 32;
constexpr int kF64MaxSide = 256;
constexpr int kF64Vals = 10 + kF64MaxC;  // moments, colour, depth, features

struct F64Layout {
  uint64_t rec = 0, order = 0, nvalid = 0, pix_T = 0, pix_end = 0, grad2d = 0, pose_part = 0,
           total = 0;
};

F64Layout f64_layout(int64_t P, int32_t W, int32_t H) {
  const uint64_t A = 256, HW = (uint64_t)W * H;
  F64Layout l;
  uint64_t o = 0;
  l.rec = o;       o = align_up(o + (uint64_t)P * 8 * sizeof(double), A);
  l.order = o;     o = align_up(o + (uint64_t)P * sizeof(uint32_t), A);
  l.nvalid = o;    o = align_up(o + sizeof(uint32_t), A);
  l.pix_T = o;     o = align_up(o + HW * sizeof(double), A);
  l.pix_end = o;   o = align_up(o + HW * sizeof(uint32_t), A);
  l.grad2d = o;    o = align_up(o + (uint64_t)P * 10 * sizeof(double), A);
  l.pose_part = o; o = align_up(o + (uint64_t)P * 6 * sizeof(double), A);
  l.total = o;
  return l;
}

struct F64Scene {
  int64_t P;
  int32_t C;
  const double *means, *log_scales, *quats, *logit, *rgb, *feat;
};

struct F64Cam {
  int32_t W, H;
  double fx, fy, cx, cy;
  const double* viewmat;
};

struct F64Ws {
  double* rec;  // [P][8]: u, v, A, B, C, opacity, z, valid
  uint32_t* order;
  uint32_t* nvalid;
  double* pix_T;
  uint32_t* pix_end;  // list positions up to the pixel's last blended Gaussian
  double* grad2d;     // [P][10]: du dv dA dB dC do dr dg db dz
  double* pose_part;  // [P][6]
};

F64Ws f64_view(void* ws, const F64Layout& l) {
  char* b = (char*)ws;
  return F64Ws{(double*)(b + l.rec),      (uint32_t*)(b + l.order), (uint32_t*)(b + l.nvalid),
               (double*)(b + l.pix_T),    (uint32_t*)(b + l.pix_end),
               (double*)(b + l.grad2d),   (double*)(b + l.pose_part)};
}

__device__ ProjT<double> project_f64(const F64Scene& g, const F64Cam& cam, const DevSettings& st,
                                     const double* V, int64_t i) {
  const int64_t P = g.P;
  return project_core<double>(g.means[i], g.means[P + i], g.means[2 * P + i], g.log_scales[i],
                              g.log_scales[P + i], g.log_scales[2 * P + i], g.quats[i],
                              g.quats[P + i], g.quats[2 * P + i], g.quats[3 * P + i], g.logit[i],
                              V, cam.W, cam.H, cam.fx, cam.fy, cam.cx, cam.cy, st);
}

// Eq. 2 at a pixel centre: alpha = min(o exp(power), alpha_max) with
// power = -(A dx^2 + 2 B dx dy + C dy^2) / 2, dx = u - x, dy = v - y.
struct Pair64 {
  double oG, alpha;
};
__device__ __forceinline__ Pair64 pair_alpha(const double* r, double x, double y,
                                             double alpha_max) {
  const double dx = r[0] - x, dy = r[1] - y;
  const double power = -0.5 * (r[2] * dx * dx + 2.0 * r[3] * dx * dy + r[4] * dy * dy);
  Pair64 p;
  p.oG = r[5] * exp(power);
  p.alpha = p.oG < alpha_max ? p.oG : alpha_max;
  return p;
}

__global__ __launch_bounds__(256) void k_f64_project(F64Scene g, F64Cam cam, DevSettings st,
                                                     F64Ws w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *w.nvalid = 0u;
  if (i >= g.P) return;
  double V[12];
  for (int k = 0; k < 12; ++k) V[k] = cam.viewmat[k];
  const ProjT<double> p = project_f64(g, cam, st, V, i);
  double* r = w.rec + i * 8;
  r[0] = p.valid ? p.u : 0.0;
  r[1] = p.valid ? p.v : 0.0;
  r[2] = p.valid ? p.A : 0.0;
  r[3] = p.valid ? p.B : 0.0;
  r[4] = p.valid ? p.Cc : 0.0;
  r[5] = p.valid ? p.o : 0.0;
  r[6] = p.z;
  r[7] = p.valid ? 1.0 : 0.0;
  w.order[i] = (uint32_t)g.P;
}

// Depth order of the valid Gaussians by counting, on the FP32 path's key
// (z rounded to float): rank = valid Gaussians in front (smaller key, or
// equal key and smaller index).
__global__ __launch_bounds__(256) void k_f64_rank(int64_t P, F64Ws w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P || w.rec[i * 8 + 7] == 0.0) return;
  const float zi = (float)w.rec[i * 8 + 6];
  uint32_t r = 0;
  for (int64_t j = 0; j < P; ++j) {
    if (w.rec[j * 8 + 7] == 0.0) continue;
    const float zj = (float)w.rec[j * 8 + 6];
    r += (zj < zi || (zj == zi && j < i)) ? 1u : 0u;
  }
  w.order[r] = (uint32_t)i;
  atomicAdd(w.nvalid, 1u);
}

// Front-to-back blending, one thread per pixel.
__global__ __launch_bounds__(256) void k_f64_render(F64Scene g, int W, int H, DevSettings st,
                                                    F64Ws w, double* out_rgb, double* out_depth,
                                                    double* out_alpha, double* out_feat,
                                                    int32_t* out_n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t HW = (int64_t)W * H;
  if (p >= HW) return;
  const double x = (double)(p % W) + 0.5, y = (double)(p / W) + 0.5;
  const bool feats = st.render_features && g.C > 0 && out_feat;
  const int64_t P = g.P;
  double T = 1.0, c[3] = {0.0, 0.0, 0.0}, d = 0.0, f[kF64MaxC];
  for (int k = 0; k < g.C; ++k) f[k] = 0.0;
  bool done = false;
  uint32_t end = 0;
  int32_t n = 0;
  const uint32_t nv = *w.nvalid;
  for (uint32_t k = 0; k < nv && !done; ++k) {
    const uint32_t gid = w.order[k];
    const double* r = w.rec + (int64_t)gid * 8;
    const Pair64 e = pair_alpha(r, x, y, (double)st.alpha_max);
    bool use;
    const double wt = blend_step(e.alpha, T, done, use, (double)st.alpha_min, (double)st.t_min);
    if (!use) continue;
    end = k + 1;
    ++n;
    for (int q = 0; q < 3; ++q) c[q] += wt * g.rgb[q * P + gid];
    d += wt * r[6];
    if (feats)
      for (int q = 0; q < g.C; ++q) f[q] += wt * g.feat[(int64_t)gid * g.C + q];
  }
  for (int q = 0; q < 3; ++q) out_rgb[q * HW + p] = c[q];
  out_depth[p] = d;
  out_alpha[p] = 1.0 - T;
  if (out_feat)
    for (int q = 0; q < g.C; ++q) out_feat[q * HW + p] = feats ? f[q] : 0.0;
  if (out_n) out_n[p] = n;
  w.pix_T[p] = T;
  w.pix_end[p] = end;
}

__device__ __forceinline__ double wave_sum64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Adjoint of the blending, one 256-thread workgroup per 16x16 tile.  The
// tile's pixels walk the depth order back to front from their last blended
// Gaussian; per Gaussian the workgroup sums the moments of dL/dpower and the
// upstream-weighted blending weights over its pixels (fixed order: wave sums,
// then the four waves), and adds the Gaussian's gradients from this tile.
__global__ __launch_bounds__(256) void k_f64_render_bwd(
    F64Scene g, int W, int H, int tiles_x, DevSettings st, F64Ws w, const double* g_rgb,
    const double* g_depth, const double* g_alpha, const double* g_feat, double* d_feat) {
  __shared__ double s_part[4][kF64Vals];
  __shared__ double s_tot[kF64Vals];
  __shared__ uint32_t s_end;
  const int tile = blockIdx.x;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int px = tx * kTile + (tid % kTile), py = ty * kTile + (tid / kTile);
  const bool inside = px < W && py < H;
  const int64_t HW = (int64_t)W * H;
  const int64_t p = inside ? (int64_t)py * W + px : 0;
  const double x = (double)px + 0.5, y = (double)py + 0.5;
  const double tcx = (double)(tx * kTile) + 0.5 * kTile, tcy = (double)(ty * kTile) + 0.5 * kTile;
  const double xr = x - tcx, yr = y - tcy;  // pixel centre relative to the tile centre
  const int64_t P = g.P;
  const int C = g.C;
  const bool feats = st.render_features && C > 0 && g_feat && d_feat;
  const int nvals = 10 + (feats ? C : 0);
  const double Tfin = inside ? w.pix_T[p] : 1.0;
  const uint32_t pend = inside ? w.pix_end[p] : 0u;
  const double gr = inside ? g_rgb[p] : 0.0, gg = inside ? g_rgb[HW + p] : 0.0;
  const double gb = inside ? g_rgb[2 * HW + p] : 0.0, gd = inside ? g_depth[p] : 0.0;
  const double ga = inside ? g_alpha[p] : 0.0;
  if (tid == 0) s_end = 0u;
  __syncthreads();
  atomicMax(&s_end, pend);
  __syncthreads();
  const uint32_t kmax = s_end;
  const double gaT = ga * Tfin;
  double T = Tfin, D = 0.0;
  for (uint32_t k = kmax; k-- > 0;) {
    const uint32_t gid = w.order[k];
    const double* r = w.rec + (int64_t)gid * 8;
    const Pair64 e = pair_alpha(r, x, y, (double)st.alpha_max);
    const bool act = inside && k < pend && e.alpha >= (double)st.alpha_min;
    const double al = act ? e.alpha : 0.0;
    const double gc = gr * g.rgb[gid] + gg * g.rgb[P + gid] + gb * g.rgb[2 * P + gid] + gd * r[6];
    double wv, dal;
    back_step(al, gc, gaT, T, D, wv, dal);
    const double og = (act && e.oG < (double)st.alpha_max) ? e.oG : 0.0;
    const double dp = dal * og;  // dL/dpower
    double v[kF64Vals];
    v[0] = dp;
    v[1] = dp * xr;
    v[2] = dp * yr;
    v[3] = dp * xr * xr;
    v[4] = dp * xr * yr;
    v[5] = dp * yr * yr;
    v[6] = wv * gr;
    v[7] = wv * gg;
    v[8] = wv * gb;
    v[9] = wv * gd;
    for (int q = 0; q < kF64MaxC; ++q)
      v[10 + q] = (feats && q < C) ? wv * (inside ? g_feat[(int64_t)q * HW + p] : 0.0) : 0.0;
    for (int q = 0; q < nvals; ++q) {
      const double s = wave_sum64(v[q]);
      if (lane == 0) s_part[wave][q] = s;
    }
    __syncthreads();
    if (tid < nvals)
      s_tot[tid] = (s_part[0][tid] + s_part[1][tid]) + (s_part[2][tid] + s_part[3][tid]);
    __syncthreads();
    if (tid == 0) {
      double geo[6];
      geo_from_moments(r[2], r[3], r[4], r[5], r[0] - tcx, r[1] - tcy, s_tot, geo);
      for (int q = 0; q < 6; ++q)
        if (geo[q] != 0.0) atomicAdd(&w.grad2d[(int64_t)gid * 10 + q], geo[q]);
    } else if (tid >= 6 && tid < 10) {
      if (s_tot[tid] != 0.0) atomicAdd(&w.grad2d[(int64_t)gid * 10 + tid], s_tot[tid]);
    } else if (tid >= 10 && tid < nvals) {
      if (s_tot[tid] != 0.0) atomicAdd(&d_feat[(int64_t)gid * C + (tid - 10)], s_tot[tid]);
    }
    __syncthreads();
  }
}

// Adjoint of the projection and the pose terms, one thread per Gaussian.
__global__ __launch_bounds__(256) void k_f64_project_bwd(F64Scene g, F64Cam cam, DevSettings st,
                                                         F64Ws w, gsff_grads_f64 out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.P) return;
  const int64_t P = g.P;
  double V[12];
  for (int k = 0; k < 12; ++k) V[k] = cam.viewmat[k];
  const ProjT<double> p = project_f64(g, cam, st, V, i);
  const double* d = w.grad2d + i * 10;
  double dmean[3] = {0.0, 0.0, 0.0}, dls[3] = {0.0, 0.0, 0.0}, dq[4] = {0.0, 0.0, 0.0, 0.0};
  double dlogit = 0.0, pose[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (p.valid) project_adjoint<double>(p, V, cam.fx, cam.fy, d, dmean, dls, dq, dlogit, pose);
  for (int k = 0; k < 3; ++k) out.means[k * P + i] = dmean[k];
  for (int k = 0; k < 3; ++k) out.log_scales[k * P + i] = dls[k];
  for (int k = 0; k < 4; ++k) out.quats[k * P + i] = dq[k];
  out.logit_opacity[i] = dlogit;
  for (int k = 0; k < 3; ++k) out.rgb[k * P + i] = d[6 + k];
  for (int k = 0; k < 6; ++k) w.pose_part[i * 6 + k] = pose[k];
}

// Pose gradient: the per-Gaussian terms summed in index order.
__global__ void k_f64_pose_sum(int64_t P, const double* part, double* pose) {
  const int k = threadIdx.x;
  if (k >= 6) return;
  double acc = 0.0;
  for (int64_t i = 0; i < P; ++i) acc += part[i * 6 + k];
  pose[k] = acc;
}

__global__ __launch_bounds__(256) void k_f64_zero(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

gsff_status f64_fail(const char* msg) { return record_error(GSFF_ERR_INVALID_ARGUMENT, msg); }

gsff_status f64_hip(hipError_t e) {
  if (e == hipSuccess) return GSFF_OK;
  return record_error(GSFF_ERR_HIP, hipGetErrorString(e));
}

bool sizes_ok(int64_t P, int32_t C, int32_t W, int32_t H) {
  return P >= 0 && P <= kF64MaxP && C >= 0 && C <= kF64MaxC && W > 0 && H > 0 &&
         W <= kF64MaxSide && H <= kF64MaxSide;
}

struct F64Ctx {
  F64Scene g;
  F64Cam cam;
  DevSettings st;
  F64Layout L;
  F64Ws w;
  hipStream_t s;
};

gsff_status f64_common(const gsff_gaussians_f64* g, const gsff_camera_f64* cam,
                       const gsff_settings* st, void* ws, size_t ws_bytes, void* stream,
                       F64Ctx* c) {
  if (!g || !cam || !st) return f64_fail("NULL gaussians/camera/settings");
  if (!sizes_ok(g->P, g->C, cam->width, cam->height))
    return f64_fail("sizes outside P <= 4096, C <= 32, 1 <= width, height <= 256");
  if (g->P > 0 && (!g->means || !g->log_scales || !g->quats || !g->logit_opacity || !g->rgb))
    return f64_fail("NULL Gaussian parameter pointer");
  if (g->P > 0 && g->C > 0 && !g->feat) return f64_fail("C > 0 but feat is NULL");
  if (!(cam->fx > 0.0) || !(cam->fy > 0.0) || !__builtin_isfinite(cam->cx) ||
      !__builtin_isfinite(cam->cy) || !cam->viewmat)
    return f64_fail("camera");
  if (!(st->alpha_min > 0.f) || !(st->alpha_max <= 1.f) || !(st->alpha_min < st->alpha_max) ||
      !(st->t_min > 0.f) || !(st->t_min < 1.f) || !(st->dilation >= 0.f) || !(st->guard > 0.f) ||
      !__builtin_isfinite(st->near_plane))
    return f64_fail("settings out of range");
  if (!ws || ((uintptr_t)ws & 255u) != 0) return f64_fail("NULL or misaligned workspace");
  c->L = f64_layout(g->P, cam->width, cam->height);
  if (ws_bytes < c->L.total) return f64_fail("workspace too small");
  c->w = f64_view(ws, c->L);
  c->g = F64Scene{g->P, g->C, g->means, g->log_scales, g->quats, g->logit_opacity, g->rgb, g->feat};
  c->cam = F64Cam{cam->width, cam->height, cam->fx, cam->fy, cam->cx, cam->cy, cam->viewmat};
  c->st = DevSettings{st->near_plane, st->guard, st->dilation, st->alpha_min,
                      st->alpha_max, st->t_min, st->render_features ? 1 : 0, 0};
  c->s = (hipStream_t)stream;
  return GSFF_OK;
}

int blocks_for(int64_t n) { return (int)((n + 255) / 256); }

}  // namespace

}  // namespace gsff

using namespace gsff;

extern "C" {

gsff_status gsff_f64_workspace_size(int64_t P, int32_t C, int32_t width, int32_t height,
                                    size_t* bytes) {
  if (!bytes) return f64_fail("NULL bytes");
  if (!sizes_ok(P, C, width, height))
    return f64_fail("sizes outside P <= 4096, C <= 32, 1 <= width, height <= 256");
  *bytes = (size_t)f64_layout(P, width, height).total;
  return GSFF_OK;
}

gsff_status gsff_forward_f64(const gsff_gaussians_f64* g, const gsff_camera_f64* cam,
                             const gsff_settings* st, void* ws, size_t ws_bytes, double* out_rgb,
                             double* out_depth, double* out_alpha, double* out_feat,
                             int32_t* out_n, void* stream) {
  F64Ctx c;
  gsff_status rc = f64_common(g, cam, st, ws, ws_bytes, stream, &c);
  if (rc != GSFF_OK) return rc;
  if (!out_rgb || !out_depth || !out_alpha) return f64_fail("NULL output image");
  if (g->C > 0 && st->render_features && !out_feat) return f64_fail("NULL feature output");
  const int64_t HW = (int64_t)cam->width * cam->height;
  k_f64_project<<<blocks_for(g->P > 0 ? g->P : 1), 256, 0, c.s>>>(c.g, c.cam, c.st, c.w);
  if (g->P > 0) k_f64_rank<<<blocks_for(g->P), 256, 0, c.s>>>(g->P, c.w);
  k_f64_render<<<blocks_for(HW), 256, 0, c.s>>>(c.g, cam->width, cam->height, c.st, c.w, out_rgb,
                                                out_depth, out_alpha, out_feat, out_n);
  return f64_hip(hipGetLastError());
}

gsff_status gsff_backward_f64(const gsff_gaussians_f64* g, const gsff_camera_f64* cam,
                              const gsff_settings* st, void* ws, size_t ws_bytes,
                              const double* g_rgb, const double* g_depth, const double* g_alpha,
                              const double* g_feat, const gsff_grads_f64* out, void* stream) {
  F64Ctx c;
  gsff_status rc = f64_common(g, cam, st, ws, ws_bytes, stream, &c);
  if (rc != GSFF_OK) return rc;
  if (!g_rgb || !g_depth || !g_alpha) return f64_fail("NULL upstream gradient");
  if (!out || !out->means || !out->log_scales || !out->quats || !out->logit_opacity ||
      !out->rgb || !out->pose)
    return f64_fail("NULL gradient output");
  if (g->C > 0 && (!out->feat || !g_feat)) return f64_fail("NULL feature gradient or upstream");
  const int W = cam->width, H = cam->height;
  const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
  if (g->P > 0) {
    k_f64_zero<<<blocks_for(g->P * 10), 256, 0, c.s>>>(c.w.grad2d, g->P * 10);
    if (g->C > 0)
      k_f64_zero<<<blocks_for(g->P * g->C), 256, 0, c.s>>>(out->feat, g->P * g->C);
    k_f64_render_bwd<<<tiles_x * tiles_y, 256, 0, c.s>>>(c.g, W, H, tiles_x, c.st, c.w, g_rgb,
                                                         g_depth, g_alpha, g_feat, out->feat);
    k_f64_project_bwd<<<blocks_for(g->P), 256, 0, c.s>>>(c.g, c.cam, c.st, c.w, *out);
  }
  k_f64_pose_sum<<<1, 64, 0, c.s>>>(g->P, c.w.pose_part, out->pose);
  return f64_hip(hipGetLastError());
}

}  // extern "C"
