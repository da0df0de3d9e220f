// CPU FP64 oracle for the feature-field Gaussian rasterizer.
//
// TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
// benchmark's CPU-baseline leg; never by the product path.  No code is shared
// with the HIP kernels.  Built with -ffp-contract=off so every expression is
// evaluated exactly in the order written.
//
// Readings of points the paper leaves open (each applied identically by the
// HIP path, which has its own implementation):
//  * opacity input is a logit, activated by the sigmoid; scales are given as
//    logarithms and activated by exp;
//  * colour is a view-independent RGB triple blended directly;
//  * the depth value blended for a Gaussian is the camera-space z of its mean,
//    and the depth image is not normalised by the accumulated opacity (Eq. 2
//    as written);
//  * the per-pixel alpha is min(alpha_max, o * exp(-1/2 d^T Sigma'^-1 d)),
//    pixels whose alpha is below alpha_min are skipped, and blending stops
//    before the Gaussian that would push transmittance below t_min;
//  * Sigma' receives a dilation on its diagonal; Gaussians at or in front of
//    the near plane, outside a guard band of the field of view, with a zero or
//    non-finite quaternion or with opacity below alpha_min are culled;
//  * pixel (px, py) is sampled at its centre (px + 1/2, py + 1/2);
//  * the depth sort key is float32(z) with z formed in FP64 as
//    ((r20 x + r21 y) + r22 z) + t2, ties broken by the lower index;
//  * the feature map's upstream gradient reaches only the feature embeddings
//    (Sec. 3.1): blending weights are constants on that path;
//  * at the alpha clamp the derivative of alpha w.r.t. o*G is zero;
//  * the pose derivative is the left perturbation T <- Exp(delta) T with
//    delta = (rho, theta), Eq. 4 read column by column for the rotation.
#include "gsff_oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace {

// Pairs just outside a Gaussian's exact support box, with alpha up to this
// fraction below alpha_min, are evaluated for the decision margins and the
// flag sets (visibility bracket, ambiguity) only: a lower-precision alpha can
// reach alpha_min there.  They never change a result.
constexpr double kWide = 1e-2;

struct Proj {
  bool valid = false;
  double mc[3] = {0, 0, 0};  // camera-space mean
  double u = 0, v = 0;
  double a = 0, b = 0, c = 0;      // Sigma' entries (dilated)
  double A = 0, B = 0, Cc = 0;     // conic = Sigma'^-1
  double o = 0;                    // activated opacity
  double rx = 0, ry = 0;           // exact half-widths of the support box
  double rxw = 0, ryw = 0;         // the same for alpha_min (1 - kWide)
  float key = 0;                   // depth sort key
  // kept for the backward pass
  double s[3] = {0, 0, 0};
  double qn[4] = {1, 0, 0, 0};     // normalised quaternion
  double qnorm = 1;
  double Rq[9] = {0};              // rotation from the quaternion
  double Sig[9] = {0};             // world covariance
  double Sc[9] = {0};              // camera covariance
  double J[6] = {0};               // 2x3 projection Jacobian
};

// ---- tiny row-major matrix helpers (3x3 unless stated) --------------------
void mat3_mul(const double* X, const double* Y, double* Z) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += X[3 * i + k] * Y[3 * k + j];
      Z[3 * i + j] = acc;
    }
}
void mat3_T(const double* X, double* Z) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Z[3 * j + i] = X[3 * i + j];
}
void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Rotation matrix of a unit quaternion (w, x, y, z), Hamilton convention.
void quat_to_rot(const double* q, double* R) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

bool finite_all(const double* p, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// ---- projection (Eq. 1 and the EWA splat of Sec. 3.1) ---------------------
Proj project_one(const orc_scene* s, const orc_camera* cam, const orc_settings* st,
                 int64_t i) {
  Proj g;
  const int64_t P = s->P;
  const double m[3] = {s->means[i], s->means[P + i], s->means[2 * P + i]};
  const double ls[3] = {s->log_scales[i], s->log_scales[P + i], s->log_scales[2 * P + i]};
  const double q[4] = {s->quats[i], s->quats[P + i], s->quats[2 * P + i], s->quats[3 * P + i]};
  const double lo = s->logit_opacity[i];
  if (!finite_all(m, 3) || !finite_all(q, 4) || !std::isfinite(lo)) return g;
  for (int k = 0; k < 3; ++k)
    if (std::isnan(ls[k]) || ls[k] == INFINITY) return g;

  const double* V = cam->viewmat;
  // camera-space mean; the order of the sums is fixed (the sort key uses z)
  g.mc[0] = ((V[0] * m[0] + V[1] * m[1]) + V[2] * m[2]) + V[3];
  g.mc[1] = ((V[4] * m[0] + V[5] * m[1]) + V[6] * m[2]) + V[7];
  g.mc[2] = ((V[8] * m[0] + V[9] * m[1]) + V[10] * m[2]) + V[11];
  const double x = g.mc[0], y = g.mc[1], z = g.mc[2];
  g.key = (float)z;
  if (!(z > st->near_plane)) return g;
  const double limx = st->guard * cam->width / (2.0 * cam->fx);
  const double limy = st->guard * cam->height / (2.0 * cam->fy);
  if (std::fabs(x / z) > limx || std::fabs(y / z) > limy) return g;

  const double qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  if (!(qn2 > 0)) return g;
  g.qnorm = std::sqrt(qn2);
  for (int k = 0; k < 4; ++k) g.qn[k] = q[k] / g.qnorm;
  for (int k = 0; k < 3; ++k) g.s[k] = std::exp(ls[k]);
  g.o = 1.0 / (1.0 + std::exp(-lo));
  if (g.o < st->alpha_min) return g;

  // Sigma = (Rq S)(Rq S)^T  (Eq. 1)
  quat_to_rot(g.qn, g.Rq);
  double M[9], Mt[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) M[3 * r + k] = g.Rq[3 * r + k] * g.s[k];
  mat3_T(M, Mt);
  mat3_mul(M, Mt, g.Sig);
  // camera covariance R Sigma R^T
  const double R[9] = {V[0], V[1], V[2], V[4], V[5], V[6], V[8], V[9], V[10]};
  double Rt[9], tmp[9];
  mat3_T(R, Rt);
  mat3_mul(R, g.Sig, tmp);
  mat3_mul(tmp, Rt, g.Sc);
  // Jacobian of the pinhole projection at the mean
  const double fx = cam->fx, fy = cam->fy;
  g.J[0] = fx / z; g.J[1] = 0; g.J[2] = -fx * x / (z * z);
  g.J[3] = 0; g.J[4] = fy / z; g.J[5] = -fy * y / (z * z);
  // Sigma' = J Sc J^T + dilation I
  double JS[6];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) {
      double acc = 0;
      for (int l = 0; l < 3; ++l) acc += g.J[3 * r + l] * g.Sc[3 * l + k];
      JS[3 * r + k] = acc;
    }
  double S2[4];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 2; ++k) {
      double acc = 0;
      for (int l = 0; l < 3; ++l) acc += JS[3 * r + l] * g.J[3 * k + l];
      S2[2 * r + k] = acc;
    }
  g.a = S2[0] + st->dilation;
  g.b = 0.5 * (S2[1] + S2[2]);
  g.c = S2[3] + st->dilation;
  const double det = g.a * g.c - g.b * g.b;
  if (!(det > 0)) return g;
  g.A = g.c / det;
  g.B = -g.b / det;
  g.Cc = g.a / det;
  g.u = fx * x / z + cam->cx;
  g.v = fy * y / z + cam->cy;
  // exact box of { alpha >= alpha_min } = { d^T K d <= 2 ln(o / alpha_min) }
  const double k2 = 2.0 * std::log(g.o / st->alpha_min);
  g.rx = std::sqrt(k2 * g.a);
  g.ry = std::sqrt(k2 * g.c);
  const double k2w = 2.0 * std::log(g.o / (st->alpha_min * (1.0 - kWide)));
  g.rxw = std::sqrt(k2w * g.a);
  g.ryw = std::sqrt(k2w * g.c);
  g.valid = true;
  return g;
}

struct Prepared {
  std::vector<Proj> proj;
  std::vector<int64_t> order;                 // valid Gaussians, (key, index) order
  std::vector<std::vector<int64_t>> rows;     // per image row, in sort order
};

bool check_args(const orc_scene* s, const orc_camera* cam, const orc_settings* st) {
  if (!s || !cam || !st) return false;
  if (s->P < 0 || s->C < 0) return false;
  if (cam->width <= 0 || cam->height <= 0) return false;
  if (s->P > 0 && (!s->means || !s->log_scales || !s->quats || !s->logit_opacity || !s->rgb))
    return false;
  if (s->P > 0 && s->C > 0 && !s->feat) return false;
  return true;
}

void prepare(const orc_scene* s, const orc_camera* cam, const orc_settings* st,
             Prepared& pr) {
  const int64_t P = s->P;
  pr.proj.resize(P);
  for (int64_t i = 0; i < P; ++i) pr.proj[i] = project_one(s, cam, st, i);
  pr.order.clear();
  for (int64_t i = 0; i < P; ++i)
    if (pr.proj[i].valid) pr.order.push_back(i);
  std::stable_sort(pr.order.begin(), pr.order.end(), [&](int64_t a, int64_t b) {
    return pr.proj[a].key < pr.proj[b].key;  // stable: ties keep index order
  });
  pr.rows.assign(cam->height, {});
  for (int64_t i : pr.order) {
    const Proj& g = pr.proj[i];
    long y0 = (long)std::floor(g.v - g.ryw - 0.5) - 1;
    long y1 = (long)std::ceil(g.v + g.ryw - 0.5) + 1;
    y0 = std::max(0L, y0);
    y1 = std::min((long)cam->height - 1, y1);
    for (long py = y0; py <= y1; ++py)
      if (std::fabs(py + 0.5 - g.v) <= g.ryw) pr.rows[py].push_back(i);
  }
}

inline bool covers(const Proj& g, long px, long py) {
  return std::fabs(px + 0.5 - g.u) <= g.rx && std::fabs(py + 0.5 - g.v) <= g.ry;
}

inline bool covers_wide(const Proj& g, long px, long py) {
  return std::fabs(px + 0.5 - g.u) <= g.rxw && std::fabs(py + 0.5 - g.v) <= g.ryw;
}

// One evaluated (pixel, Gaussian) pair.
struct Eval {
  int64_t i;
  double dx, dy;     // mean minus pixel centre
  double G, oG, alpha;
  bool clamped;
};

struct NoEval {
  void operator()(const Eval&, double) const {}
};

// Front-to-back blending at one pixel (Eqs. 2-3).  Calls on_contrib(e, T)
// for every contributor with the transmittance in front of it (and, when
// given, on_eval(e, T) for every evaluated pair before its decision, the
// pairs just outside the exact support box included); returns the final
// transmittance.  Tracks decision margins and a decision signature.
template <class F, class G = NoEval>
double composite_pixel(const Prepared& pr, const orc_settings* st, long px, long py,
                       F&& on_contrib, double* margin, uint64_t* hash,
                       int64_t* n_eval, G on_eval = G{}) {
  double T = 1.0;
  double mg = INFINITY;
  for (int64_t i : pr.rows[py]) {
    const Proj& g = pr.proj[i];
    if (!covers_wide(g, px, py)) continue;
    Eval e;
    e.i = i;
    e.dx = g.u - (px + 0.5);
    e.dy = g.v - (py + 0.5);
    const double power = -0.5 * (g.A * e.dx * e.dx + 2.0 * g.B * e.dx * e.dy + g.Cc * e.dy * e.dy);
    e.G = std::exp(power);
    e.oG = g.o * e.G;
    e.clamped = !(e.oG < st->alpha_max);
    e.alpha = e.clamped ? st->alpha_max : e.oG;
    if (!covers(g, px, py)) {
      // outside the exact box alpha < alpha_min: skipped, margin only
      mg = std::min(mg, std::fabs(e.alpha - st->alpha_min) / st->alpha_min);
      on_eval(e, T);
      continue;
    }
    if (n_eval) ++*n_eval;
    on_eval(e, T);
    mg = std::min(mg, std::fabs(e.alpha - st->alpha_min) / st->alpha_min);
    mg = std::min(mg, std::fabs(e.oG - st->alpha_max) / st->alpha_max);
    int code;
    if (e.alpha < st->alpha_min) {
      code = 0;
    } else {
      const double Tn = T * (1.0 - e.alpha);
      mg = std::min(mg, std::fabs(Tn - st->t_min) / st->t_min);
      if (Tn < st->t_min) {
        code = 2;
      } else {
        code = e.clamped ? 3 : 1;
        on_contrib(e, T);
        T = Tn;
      }
    }
    if (hash) {
      uint64_t h = *hash;
      const uint64_t words[4] = {(uint64_t)px, (uint64_t)py, (uint64_t)i, (uint64_t)code};
      for (uint64_t w : words) {
        h ^= w;
        h *= 1099511628211ULL;
      }
      *hash = h;
    }
    if (code == 2) break;
  }
  if (margin) *margin = mg;
  return T;
}

}  // namespace

extern "C" int orc_project(const orc_scene* s, const orc_camera* cam,
                           const orc_settings* st, double* proj) {
  if (!check_args(s, cam, st) || (s->P > 0 && !proj)) return -1;
  for (int64_t i = 0; i < s->P; ++i) {
    const Proj g = project_one(s, cam, st, i);
    double* r = proj + i * ORC_PROJ_FIELDS;
    r[ORC_VALID] = g.valid ? 1.0 : 0.0;
    r[ORC_U] = g.u;
    r[ORC_V] = g.v;
    r[ORC_CONIC_A] = g.A;
    r[ORC_CONIC_B] = g.B;
    r[ORC_CONIC_C] = g.Cc;
    r[ORC_DEPTH] = g.mc[2];
    r[ORC_KEY] = (double)g.key;
    r[ORC_OPACITY] = g.o;
    r[ORC_RX] = g.rx;
    r[ORC_RY] = g.ry;
    r[ORC_SIG_A] = g.a;
    r[ORC_SIG_B] = g.b;
    r[ORC_SIG_C] = g.c;
  }
  return 0;
}

extern "C" int orc_render(const orc_scene* s, const orc_camera* cam,
                          const orc_settings* st, double* out_rgb, double* out_depth,
                          double* out_alpha, double* out_feat, double* out_T,
                          int32_t* out_n, double* out_margin, uint64_t* hash) {
  if (!check_args(s, cam, st) || !out_rgb || !out_depth || !out_alpha) return -1;
  if (s->C > 0 && !out_feat) return -1;
  Prepared pr;
  prepare(s, cam, st, pr);
  const long W = cam->width, H = cam->height;
  const int64_t HW = (int64_t)W * H;
  const int C = s->C;
  const int64_t P = s->P;
  if (hash) *hash = 1469598103934665603ULL;
  std::vector<double> F(C);
  for (long py = 0; py < H; ++py)
    for (long px = 0; px < W; ++px) {
      double col[3] = {0, 0, 0}, dep = 0;
      std::fill(F.begin(), F.end(), 0.0);
      int32_t n = 0;
      double mg;
      const double T = composite_pixel(
          pr, st, px, py,
          [&](const Eval& e, double Tin) {
            const double w = e.alpha * Tin;
            for (int k = 0; k < 3; ++k) col[k] += w * s->rgb[k * P + e.i];
            dep += w * pr.proj[e.i].mc[2];
            if (st->render_features)
              for (int c = 0; c < C; ++c) F[c] += w * s->feat[e.i * C + c];
            ++n;
          },
          &mg, hash, nullptr);
      const int64_t p = py * W + px;
      for (int k = 0; k < 3; ++k) out_rgb[k * HW + p] = col[k];
      out_depth[p] = dep;
      out_alpha[p] = 1.0 - T;
      for (int c = 0; c < C; ++c) out_feat[c * HW + p] = st->render_features ? F[c] : 0.0;
      if (out_T) out_T[p] = T;
      if (out_n) out_n[p] = n;
      if (out_margin) out_margin[p] = mg;
    }
  return 0;
}

// Visibility record (Sec. 3.2, Eq. 5): Gaussian i is visible when it is
// blended at some pixel while the transmittance in front of it exceeds
// t_vis.  sure[i] = 1 when that holds with the transmittance above
// t_vis (1 + rel) and alpha at least alpha_min (1 + rel) at some pixel;
// possible[i] = 1 when at some evaluated pair alpha reaches
// alpha_min (1 - rel) with the transmittance above t_vis (1 - rel).  A
// computation in lower precision decides every Gaussian in sure as visible
// and none outside possible.
extern "C" int orc_visibility(const orc_scene* s, const orc_camera* cam,
                              const orc_settings* st, double t_vis, double rel, uint8_t* sure,
                              uint8_t* possible) {
  if (!check_args(s, cam, st) || (s->P > 0 && (!sure || !possible))) return -1;
  Prepared pr;
  prepare(s, cam, st, pr);
  for (int64_t i = 0; i < s->P; ++i) sure[i] = possible[i] = 0;
  for (long py = 0; py < cam->height; ++py)
    for (long px = 0; px < cam->width; ++px)
      composite_pixel(
          pr, st, px, py,
          [&](const Eval& e, double Tin) {
            if (Tin > t_vis * (1.0 + rel) && e.alpha >= st->alpha_min * (1.0 + rel))
              sure[e.i] = 1;
          },
          nullptr, nullptr, nullptr,
          [&](const Eval& e, double Tin) {
            if (Tin > t_vis * (1.0 - rel) && e.alpha >= st->alpha_min * (1.0 - rel))
              possible[e.i] = 1;
          });
  return 0;
}

// Gaussians whose gradient a lower-precision computation may legitimately
// take differently.  A pixel is ambiguous when some skip, clamp or stop
// decision there lies within relative distance `thr` of its threshold (the
// pixel's margin, as orc_render reports it).  Flagged: every Gaussian
// evaluated at an ambiguous pixel, and after its stop every Gaussian the
// pixel could still reach if decisions went the other way (taken as the
// transmittance in front of the stopping Gaussian raised by 1%, more than two
// skipped Gaussians at alpha_min restore, and alpha thresholds lowered by
// thr).  Everywhere else both computations take every decision alike, so the
// gradients agree to rounding.  flags[i] = 1 for a flagged Gaussian.
extern "C" int orc_ambiguous(const orc_scene* s, const orc_camera* cam,
                             const orc_settings* st, double thr, int64_t n,
                             const int32_t* pxs, const int32_t* pys, uint8_t* flags) {
  if (!check_args(s, cam, st) || (s->P > 0 && !flags)) return -1;
  if ((pxs == nullptr) != (pys == nullptr) || (pxs && n < 0) || !(thr < kWide)) return -1;
  Prepared pr;
  prepare(s, cam, st, pr);
  for (int64_t i = 0; i < s->P; ++i) flags[i] = 0;
  std::vector<int64_t> walked;
  const int64_t npx = pxs ? n : (int64_t)cam->width * cam->height;
  for (int64_t k = 0; k < npx; ++k) {
    const long px = pxs ? pxs[k] : (long)(k % cam->width);
    const long py = pxs ? pys[k] : (long)(k / cam->width);
    if (px < 0 || px >= cam->width || py < 0 || py >= cam->height) return -1;
    walked.clear();
    double mg, T_last = 1.0;
    composite_pixel(
        pr, st, px, py, [](const Eval&, double) {}, &mg, nullptr, nullptr,
        [&](const Eval& e, double Tin) {
          walked.push_back(e.i);
          T_last = Tin;
        });
    if (!(mg < thr)) continue;
    for (int64_t i : walked) flags[i] = 1;
    if (walked.empty()) continue;
    // past the last evaluated Gaussian: those the pixel could still reach
    double Tw = T_last * 1.01;
    bool past = false;
    for (int64_t i : pr.rows[py]) {
      const Proj& g = pr.proj[i];
      if (!covers_wide(g, px, py)) continue;
      const double dx = g.u - (px + 0.5), dy = g.v - (py + 0.5);
      const double power = -0.5 * (g.A * dx * dx + 2.0 * g.B * dx * dy + g.Cc * dy * dy);
      const double oG = g.o * std::exp(power);
      const double alpha = oG < st->alpha_max ? oG : st->alpha_max;
      if (!past) {
        if (i == walked.back()) {
          past = true;
          if (alpha >= st->alpha_min * (1.0 - thr)) Tw *= 1.0 - alpha;
        }
        continue;
      }
      if (alpha < st->alpha_min * (1.0 - thr)) continue;
      if (Tw < st->t_min * (1.0 - thr)) break;
      flags[i] = 1;
      Tw *= 1.0 - alpha;
    }
  }
  return 0;
}

extern "C" int orc_render_pixels(const orc_scene* s, const orc_camera* cam,
                                 const orc_settings* st, int64_t n, const int32_t* px,
                                 const int32_t* py, double* out) {
  if (!check_args(s, cam, st) || n < 0 || (n > 0 && (!px || !py || !out))) return -1;
  Prepared pr;
  prepare(s, cam, st, pr);
  const int C = s->C;
  const int64_t P = s->P;
  std::vector<double> F(C);
  for (int64_t k = 0; k < n; ++k) {
    if (px[k] < 0 || px[k] >= cam->width || py[k] < 0 || py[k] >= cam->height) return -1;
    double col[3] = {0, 0, 0}, dep = 0;
    std::fill(F.begin(), F.end(), 0.0);
    const double T = composite_pixel(
        pr, st, px[k], py[k],
        [&](const Eval& e, double Tin) {
          const double w = e.alpha * Tin;
          for (int q = 0; q < 3; ++q) col[q] += w * s->rgb[q * P + e.i];
          dep += w * pr.proj[e.i].mc[2];
          if (st->render_features)
            for (int c = 0; c < C; ++c) F[c] += w * s->feat[e.i * C + c];
        },
        nullptr, nullptr, nullptr);
    double* o = out + k * (5 + C);
    o[0] = col[0];
    o[1] = col[1];
    o[2] = col[2];
    o[3] = dep;
    o[4] = 1.0 - T;
    for (int c = 0; c < C; ++c) o[5 + c] = st->render_features ? F[c] : 0.0;
  }
  return 0;
}

extern "C" int orc_backward(const orc_scene* s, const orc_camera* cam,
                            const orc_settings* st, const double* g_rgb,
                            const double* g_depth, const double* g_alpha,
                            const double* g_feat, double* d_means, double* d_log_scales,
                            double* d_quats, double* d_logit, double* d_rgb,
                            double* d_feat, double* d_pose, double* d2d_out) {
  if (!check_args(s, cam, st) || !g_rgb || !g_depth || !g_alpha) return -1;
  if (!d_means || !d_log_scales || !d_quats || !d_logit || !d_rgb || !d_pose) return -1;
  if (s->C > 0 && !d_feat) return -1;
  Prepared pr;
  prepare(s, cam, st, pr);
  const long W = cam->width, H = cam->height;
  const int64_t HW = (int64_t)W * H;
  const int C = s->C;
  const int64_t P = s->P;
  const bool feat_on = st->render_features && C > 0 && g_feat != nullptr;

  // image-space gradients per Gaussian: du dv dA dB dC do dr dg db dz
  std::vector<double> d2d(P * 10, 0.0);
  std::vector<double> df((size_t)P * C, 0.0);

  struct Contrib {
    Eval e;
    double Tin;
  };
  std::vector<Contrib> list;
  for (long py = 0; py < H; ++py)
    for (long px = 0; px < W; ++px) {
      const int64_t p = py * W + px;
      // a pixel whose upstream is exactly zero contributes exactly zero
      bool any = g_rgb[p] != 0.0 || g_rgb[HW + p] != 0.0 || g_rgb[2 * HW + p] != 0.0 ||
                 g_depth[p] != 0.0 || g_alpha[p] != 0.0;
      if (feat_on)
        for (int c = 0; c < C && !any; ++c) any = g_feat[c * HW + p] != 0.0;
      if (!any) continue;
      // pass 1: contributors and the final outputs O_k (k = r, g, b, depth)
      list.clear();
      double O[4] = {0, 0, 0, 0};
      const double Tfin = composite_pixel(
          pr, st, px, py,
          [&](const Eval& e, double Tin) {
            list.push_back({e, Tin});
            const double w = e.alpha * Tin;
            for (int k = 0; k < 3; ++k) O[k] += w * s->rgb[k * P + e.i];
            O[3] += w * pr.proj[e.i].mc[2];
          },
          nullptr, nullptr, nullptr);
      const double gk[4] = {g_rgb[p], g_rgb[HW + p], g_rgb[2 * HW + p], g_depth[p]};
      const double gA = g_alpha[p];
      // pass 2: front to back with running prefix sums
      double pre[4] = {0, 0, 0, 0};
      for (const Contrib& ct : list) {
        const Eval& e = ct.e;
        const Proj& g = pr.proj[e.i];
        const double T = ct.Tin;
        const double w = e.alpha * T;
        const double vk[4] = {s->rgb[e.i], s->rgb[P + e.i], s->rgb[2 * P + e.i], g.mc[2]};
        double dalpha = 0;
        for (int k = 0; k < 4; ++k) {
          pre[k] += w * vk[k];
          const double suffix = O[k] - pre[k];  // sum over later contributors
          dalpha += gk[k] * (T * vk[k] - suffix / (1.0 - e.alpha));
        }
        dalpha += gA * Tfin / (1.0 - e.alpha);
        double* d = &d2d[e.i * 10];
        d[6] += w * gk[0];
        d[7] += w * gk[1];
        d[8] += w * gk[2];
        d[9] += w * gk[3];
        if (feat_on)
          for (int c = 0; c < C; ++c) df[e.i * C + c] += w * g_feat[c * HW + p];
        if (!e.clamped) {
          const double dpow = dalpha * e.oG;  // d alpha / d power = o G
          d[5] += dalpha * e.G;               // d alpha / d o = G
          d[0] += dpow * -(g.A * e.dx + g.B * e.dy);
          d[1] += dpow * -(g.B * e.dx + g.Cc * e.dy);
          d[2] += dpow * (-0.5 * e.dx * e.dx);
          d[3] += dpow * (-e.dx * e.dy);
          d[4] += dpow * (-0.5 * e.dy * e.dy);
        }
      }
    }

  // chain rule from image space to the Gaussian parameters and the pose
  const double* V = cam->viewmat;
  const double R[9] = {V[0], V[1], V[2], V[4], V[5], V[6], V[8], V[9], V[10]};
  const double fx = cam->fx, fy = cam->fy;
  double pose[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = 0; i < P; ++i) {
    const Proj& g = pr.proj[i];
    const double* d = &d2d[i * 10];
    for (int k = 0; k < 3; ++k) d_rgb[k * P + i] = d[6 + k];
    for (int c = 0; c < C; ++c) d_feat[i * C + c] = feat_on ? df[i * C + c] : 0.0;
    if (d2d_out)
      for (int k = 0; k < 10; ++k) d2d_out[i * 10 + k] = d[k];
    for (int k = 0; k < 3; ++k) {
      d_means[k * P + i] = 0;
      d_log_scales[k * P + i] = 0;
    }
    for (int k = 0; k < 4; ++k) d_quats[k * P + i] = 0;
    d_logit[i] = 0;
    if (!g.valid) continue;

    // conic -> Sigma': G_S = -K G_K K with G_K = [[dA, dB/2], [dB/2, dC]]
    const double K[4] = {g.A, g.B, g.B, g.Cc};
    const double GK[4] = {d[2], 0.5 * d[3], 0.5 * d[3], d[4]};
    double KG[4], GS[4];
    for (int r = 0; r < 2; ++r)
      for (int c2 = 0; c2 < 2; ++c2) KG[2 * r + c2] = K[2 * r] * GK[c2] + K[2 * r + 1] * GK[2 + c2];
    for (int r = 0; r < 2; ++r)
      for (int c2 = 0; c2 < 2; ++c2) GS[2 * r + c2] = -(KG[2 * r] * K[c2] + KG[2 * r + 1] * K[2 + c2]);
    // Sigma' = J Sc J^T:  dSc = J^T GS J,  dJ = 2 GS J Sc
    double GJ[6] = {0}, GSc[9] = {0};
    for (int r = 0; r < 3; ++r)
      for (int c2 = 0; c2 < 3; ++c2) {
        double acc = 0;
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) acc += g.J[3 * a + r] * GS[2 * a + b] * g.J[3 * b + c2];
        GSc[3 * r + c2] = acc;
      }
    for (int r = 0; r < 2; ++r)
      for (int c2 = 0; c2 < 3; ++c2) {
        double acc = 0;
        for (int b = 0; b < 2; ++b)
          for (int l = 0; l < 3; ++l) acc += GS[2 * r + b] * g.J[3 * b + l] * g.Sc[3 * l + c2];
        GJ[3 * r + c2] = 2.0 * acc;
      }
    // Sc = R Sig R^T:  dSig = R^T GSc R,  dR = 2 GSc R Sig
    double Rt[9], t1[9], GSig[9], GR[9];
    mat3_T(R, Rt);
    mat3_mul(Rt, GSc, t1);
    mat3_mul(t1, R, GSig);
    mat3_mul(GSc, R, t1);
    mat3_mul(t1, g.Sig, GR);
    for (int k = 0; k < 9; ++k) GR[k] *= 2.0;
    // Sig = M M^T with M = Rq S:  dM = 2 GSig M
    double M[9], GM[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) M[3 * r + k] = g.Rq[3 * r + k] * g.s[k];
    mat3_mul(GSig, M, GM);
    for (int k = 0; k < 9; ++k) GM[k] *= 2.0;
    double GRq[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) GRq[3 * r + k] = GM[3 * r + k] * g.s[k];
    for (int k = 0; k < 3; ++k) {
      double ds = 0;
      for (int r = 0; r < 3; ++r) ds += GM[3 * r + k] * g.Rq[3 * r + k];
      d_log_scales[k * P + i] = ds * g.s[k];
    }
    // rotation entries -> unit quaternion
    const double w = g.qn[0], x = g.qn[1], y = g.qn[2], z = g.qn[3];
    const double* Gq = GRq;
    double dq[4];
    dq[0] = 2 * (-z * Gq[1] + y * Gq[2] + z * Gq[3] - x * Gq[5] - y * Gq[6] + x * Gq[7]);
    dq[1] = 2 * (y * Gq[1] + z * Gq[2] + y * Gq[3] - 2 * x * Gq[4] - w * Gq[5] + z * Gq[6] +
                 w * Gq[7] - 2 * x * Gq[8]);
    dq[2] = 2 * (-2 * y * Gq[0] + x * Gq[1] + w * Gq[2] + x * Gq[3] + z * Gq[5] - w * Gq[6] +
                 z * Gq[7] - 2 * y * Gq[8]);
    dq[3] = 2 * (-2 * z * Gq[0] - w * Gq[1] + x * Gq[2] + w * Gq[3] - 2 * z * Gq[4] + y * Gq[5] +
                 x * Gq[6] + y * Gq[7]);
    // through q / |q|
    const double qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
    for (int k = 0; k < 4; ++k) d_quats[k * P + i] = (dq[k] - g.qn[k] * qd) / g.qnorm;
    // opacity logit
    d_logit[i] = d[5] * g.o * (1.0 - g.o);
    // camera-space mean: through (u, v), J and the blended depth
    const double xc = g.mc[0], yc = g.mc[1], zc = g.mc[2];
    double gm[3] = {0, 0, 0};
    gm[0] += d[0] * fx / zc;
    gm[2] += d[0] * (-fx * xc / (zc * zc));
    gm[1] += d[1] * fy / zc;
    gm[2] += d[1] * (-fy * yc / (zc * zc));
    gm[0] += GJ[2] * (-fx / (zc * zc));
    gm[1] += GJ[5] * (-fy / (zc * zc));
    gm[2] += GJ[0] * (-fx / (zc * zc)) + GJ[2] * (2.0 * fx * xc / (zc * zc * zc)) +
             GJ[4] * (-fy / (zc * zc)) + GJ[5] * (2.0 * fy * yc / (zc * zc * zc));
    gm[2] += d[9];
    // world mean: R^T gm
    for (int k = 0; k < 3; ++k) d_means[k * P + i] = R[k] * gm[0] + R[3 + k] * gm[1] + R[6 + k] * gm[2];
    // pose (Eq. 4): rho += gm; theta += mc x gm + sum_k w_k x GR[:, k]
    double cr[3];
    cross3(g.mc, gm, cr);
    for (int k = 0; k < 3; ++k) {
      pose[k] += gm[k];
      pose[3 + k] += cr[k];
    }
    for (int k = 0; k < 3; ++k) {
      const double wk[3] = {R[k], R[3 + k], R[6 + k]};
      const double gk[3] = {GR[k], GR[3 + k], GR[6 + k]};
      cross3(wk, gk, cr);
      for (int l = 0; l < 3; ++l) pose[3 + l] += cr[l];
    }
  }
  for (int k = 0; k < 6; ++k) d_pose[k] = pose[k];
  return 0;
}

extern "C" int64_t orc_tile_lists(const orc_scene* s, const orc_camera* cam,
                                  const orc_settings* st, int32_t tile, int64_t* counts,
                                  int32_t* ids) {
  if (!check_args(s, cam, st) || tile <= 0 || !counts) return -1;
  Prepared pr;
  prepare(s, cam, st, pr);
  const long W = cam->width, H = cam->height;
  const long tx = (W + tile - 1) / tile, ty = (H + tile - 1) / tile;
  std::vector<std::vector<int32_t>> lists(tx * ty);
  for (int64_t i : pr.order) {
    const Proj& g = pr.proj[i];
    const long x0 = std::max(0L, (long)std::floor(g.u - g.rx - 0.5) - 1);
    const long x1 = std::min(W - 1, (long)std::ceil(g.u + g.rx - 0.5) + 1);
    const long y0 = std::max(0L, (long)std::floor(g.v - g.ry - 0.5) - 1);
    const long y1 = std::min(H - 1, (long)std::ceil(g.v + g.ry - 0.5) + 1);
    for (long by = y0 / tile; by <= y1 / tile; ++by)
      for (long bx = x0 / tile; bx <= x1 / tile; ++bx) {
        bool hit = false;
        for (long py = by * tile; py < std::min(H, (by + 1) * tile) && !hit; ++py)
          for (long px = bx * tile; px < std::min(W, (bx + 1) * tile) && !hit; ++px) {
            if (!covers(g, px, py)) continue;
            const double dx = g.u - (px + 0.5), dy = g.v - (py + 0.5);
            const double power = -0.5 * (g.A * dx * dx + 2.0 * g.B * dx * dy + g.Cc * dy * dy);
            const double oG = g.o * std::exp(power);
            const double alpha = oG < st->alpha_max ? oG : st->alpha_max;
            if (alpha >= st->alpha_min) hit = true;
          }
        if (hit) lists[by * tx + bx].push_back((int32_t)i);
      }
  }
  int64_t total = 0;
  for (long t = 0; t < tx * ty; ++t) {
    counts[t] = (int64_t)lists[t].size();
    if (ids && !lists[t].empty())  // (an empty list's data() may be null)
      std::memcpy(ids + total, lists[t].data(), lists[t].size() * sizeof(int32_t));
    total += counts[t];
  }
  return total;
}

extern "C" int orc_work_counts(const orc_scene* s, const orc_camera* cam,
                               const orc_settings* st, int32_t tile, int64_t* out) {
  if (!check_args(s, cam, st) || tile <= 0 || !out) return -1;
  const long W = cam->width, H = cam->height;
  const long tx = (W + tile - 1) / tile, ty = (H + tile - 1) / tile;
  std::vector<int64_t> counts(tx * ty);
  const int64_t M = orc_tile_lists(s, cam, st, tile, counts.data(), nullptr);
  if (M < 0) return -1;
  std::vector<int32_t> ids(M);
  orc_tile_lists(s, cam, st, tile, counts.data(), ids.data());
  std::vector<int64_t> start(tx * ty + 1, 0);
  for (long t = 0; t < tx * ty; ++t) start[t + 1] = start[t] + counts[t];
  Prepared pr;
  prepare(s, cam, st, pr);
  int64_t w_alg = 0, w_tile = 0, contrib = 0;
  for (long by = 0; by < ty; ++by)
    for (long bx = 0; bx < tx; ++bx) {
      const long t = by * tx + bx;
      int64_t prefix = 0;
      for (long py = by * tile; py < std::min(H, (by + 1) * tile); ++py)
        for (long px = bx * tile; px < std::min(W, (bx + 1) * tile); ++px) {
          int64_t ne = 0;
          // walk the block's list to find this pixel's stop position
          double T = 1.0;
          int64_t pos = counts[t];
          for (int64_t j = 0; j < counts[t]; ++j) {
            const Proj& g = pr.proj[ids[start[t] + j]];
            if (!covers(g, px, py)) continue;
            ++ne;
            const double dx = g.u - (px + 0.5), dy = g.v - (py + 0.5);
            const double power = -0.5 * (g.A * dx * dx + 2.0 * g.B * dx * dy + g.Cc * dy * dy);
            const double oG = g.o * std::exp(power);
            const double alpha = oG < st->alpha_max ? oG : st->alpha_max;
            if (alpha < st->alpha_min) continue;
            const double Tn = T * (1.0 - alpha);
            if (Tn < st->t_min) {
              pos = j + 1;
              break;
            }
            ++contrib;
            T = Tn;
          }
          w_alg += ne;
          prefix = std::max(prefix, pos);
        }
      w_tile += prefix * (int64_t)tile * tile;
    }
  out[0] = M;
  out[1] = w_alg;
  out[2] = w_tile;
  out[3] = contrib;
  return 0;
}
