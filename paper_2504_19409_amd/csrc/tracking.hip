// Tracking support (Sec. 3.2, camera pose optimisation and tracking loss):
// the two per-pixel masks of the tracking loss (Eq. 6) and the pose step that
// turns the pose gradient of Eq. 4 into the next camera pose.
//
// Masks.  m_e keeps the pixels where the target colour image has a strong
// gradient: the Sobel gradient of the grey image (mean of r, g, b), scaled
// by 1/8 so that a ramp of slope a has magnitude a, with the image edge
// replicated beyond the border; kept where the magnitude exceeds the
// threshold.  m_v keeps the pixels the render at the frozen Gaussians covers:
// accumulated opacity above the threshold.
//
// Pose step.  The pose gradient is taken for the left perturbation
// T <- Exp(delta) T, delta = (rho, theta).  One Adam step (first and second
// moments, bias-corrected; separate rates for rho and theta) gives delta;
// the pose becomes Exp(delta) T with the closed-form SE(3) exponential
// R = I + a W + b W^2, t = (I + b W + c W^2) rho, W = theta^, phi = |theta|,
// a = sin(phi)/phi, b = (1 - cos(phi))/phi^2, c = (phi - sin(phi))/phi^3.
// The step runs in FP64 on one lane; the pose is stored in FP32.
//
// Convergence (the test on the change of the camera-frame means and of the
// rotation, Sec. 3.2).  Adam at a fixed rate keeps taking steps of about
// the rate near the optimum, so single increments never vanish; what does
// vanish is the net motion over several steps once the pose oscillates
// about the optimum.  Every `window` steps the step measures the rotation
// angle and the translation of T_now T_start^-1 (T_start: the pose at the
// window's start; the translation is the shift of the camera-frame position
// of the world origin, and every camera-frame mean moves by at most that
// plus the angle times its distance) and sets the converged flag when both
// are below their tolerances.  From then on the step leaves the pose alone
// until a call with step 1 starts the next frame, so a captured loop of a
// fixed number of iterations ends where an early exit would.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gsff_internal.h"

namespace gsff {
namespace {

__global__ __launch_bounds__(256) void k_tracking_masks(const float* __restrict__ rgb,
                                                        const float* __restrict__ alpha, int W,
                                                        int H, float edge2, float vis_threshold,
                                                        uint8_t* __restrict__ mask_v,
                                                        uint8_t* __restrict__ mask_e) {
  const int64_t HW = (int64_t)W * H;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= HW) return;
  const int x = (int)(p % W), y = (int)(p / W);
  if (mask_v) mask_v[p] = alpha[p] > vis_threshold ? 1 : 0;
  if (!mask_e) return;
  // r + g + b at the 3x3 neighbourhood, the border replicated
  const int xs[3] = {x > 0 ? x - 1 : 0, x, x + 1 < W ? x + 1 : W - 1};
  const int ys[3] = {y > 0 ? y - 1 : 0, y, y + 1 < H ? y + 1 : H - 1};
  float s[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int64_t q = (int64_t)ys[j] * W + xs[i];
      s[j][i] = rgb[q] + rgb[HW + q] + rgb[2 * HW + q];
    }
  const float gx = (s[0][2] + 2.f * s[1][2] + s[2][2]) - (s[0][0] + 2.f * s[1][0] + s[2][0]);
  const float gy = (s[2][0] + 2.f * s[2][1] + s[2][2]) - (s[0][0] + 2.f * s[0][1] + s[0][2]);
  // |grad of the grey image| = sqrt(gx^2 + gy^2) / (8 * 3) against the
  // threshold, compared squared: edge2 = (24 threshold)^2
  mask_e[p] = gx * gx + gy * gy > edge2 ? 1 : 0;
}

// Rotation angle and translation length of the relative motion
// Tn T0^-1 = [Rn R0^T | tn - Rn R0^T t0] between two poses [R | t] (row-major
// 3x4): the change of the world-to-camera rotation W and of the
// camera-frame position of the world origin.
__device__ void relative_motion(const double* Tn, const double* T0, double& angle,
                                double& shift) {
  double D[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int l = 0; l < 3; ++l) acc += Tn[4 * r + l] * T0[4 * k + l];
      D[3 * r + k] = acc;
    }
  const double sx = D[7] - D[5], sy = D[2] - D[6], sz = D[3] - D[1];
  const double sn = 0.5 * sqrt(sx * sx + sy * sy + sz * sz);
  const double cs = 0.5 * (D[0] + D[4] + D[8] - 1.0);
  angle = atan2(sn, cs);
  double ss = 0.0;
  for (int r = 0; r < 3; ++r) {
    const double t = Tn[4 * r + 3] - (D[3 * r] * T0[3] + D[3 * r + 1] * T0[7] + D[3 * r + 2] * T0[11]);
    ss += t * t;
  }
  shift = sqrt(ss);
}

// state: [0, 6) first moments, [6, 12) second moments, [12, 24) the pose at
// the start of the current test window, [24] converged (0 / 1).
__global__ void k_pose_adam_step(float* __restrict__ viewmat, const float* __restrict__ grad,
                                 float* __restrict__ state, int step, float lr_trans,
                                 float lr_rot, float beta1, float beta2, float eps, int window,
                                 float tol_trans, float tol_rot, float* __restrict__ delta_out,
                                 uint32_t* __restrict__ converged_out) {
  if (threadIdx.x != 0) return;
  if (step == 1) {  // a new frame: fresh moments and test window
    for (int k = 0; k < 12; ++k) state[k] = 0.f;
    for (int k = 0; k < 12; ++k) state[12 + k] = viewmat[k];
    state[24] = 0.f;
  }
  if (state[24] != 0.f) {  // converged earlier: the pose stays
    if (delta_out)
      for (int k = 0; k < 6; ++k) delta_out[k] = 0.f;
    if (converged_out) converged_out[0] = 1u;
    return;
  }
  const double b1 = beta1, b2 = beta2;
  const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
  double d[6];
  for (int k = 0; k < 6; ++k) {
    const double g = grad[k];
    const double m = b1 * state[k] + (1.0 - b1) * g;
    const double v = b2 * state[6 + k] + (1.0 - b2) * g * g;
    state[k] = (float)m;
    state[6 + k] = (float)v;
    const double lr = k < 3 ? lr_trans : lr_rot;
    d[k] = -lr * (m / c1) / (sqrt(v / c2) + (double)eps);
  }
  if (delta_out)
    for (int k = 0; k < 6; ++k) delta_out[k] = (float)d[k];
  // Exp(delta): rotation Rd and translation td
  const double th[3] = {d[3], d[4], d[5]};
  const double phi2 = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
  const double phi = sqrt(phi2);
  double a, b, c;
  if (phi < 1e-4) {  // Taylor series, exact to rounding at this size
    a = 1.0 - phi2 / 6.0;
    b = 0.5 - phi2 / 24.0;
    c = 1.0 / 6.0 - phi2 / 120.0;
  } else {
    a = sin(phi) / phi;
    b = (1.0 - cos(phi)) / phi2;
    c = (phi - sin(phi)) / (phi2 * phi);
  }
  const double Wm[9] = {0.0, -th[2], th[1], th[2], 0.0, -th[0], -th[1], th[0], 0.0};
  double W2[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int l = 0; l < 3; ++l) acc += Wm[3 * r + l] * Wm[3 * l + k];
      W2[3 * r + k] = acc;
    }
  double Rd[9], V[9];
  for (int e = 0; e < 9; ++e) {
    const double I = (e % 4 == 0) ? 1.0 : 0.0;
    Rd[e] = I + a * Wm[e] + b * W2[e];
    V[e] = I + b * Wm[e] + c * W2[e];
  }
  double td[3];
  for (int r = 0; r < 3; ++r) td[r] = V[3 * r] * d[0] + V[3 * r + 1] * d[1] + V[3 * r + 2] * d[2];
  // [R | t] <- [Rd R | Rd t + td]
  double T[12], Tn[12];
  for (int e = 0; e < 12; ++e) T[e] = viewmat[e];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 4; ++k) {
      double acc = k == 3 ? td[r] : 0.0;
      for (int l = 0; l < 3; ++l) acc += Rd[3 * r + l] * T[4 * l + k];
      viewmat[4 * r + k] = (float)acc;
      Tn[4 * r + k] = (double)(float)acc;
    }
  // convergence test at the end of every window of `window` steps: the net
  // motion over the window against the tolerances
  uint32_t conv = 0u;
  if (window > 0 && step % window == 0) {
    double T0[12];
    for (int e = 0; e < 12; ++e) T0[e] = state[12 + e];
    double angle, shift;
    relative_motion(Tn, T0, angle, shift);
    conv = (shift < (double)tol_trans && angle < (double)tol_rot) ? 1u : 0u;
    for (int e = 0; e < 12; ++e) state[12 + e] = (float)Tn[e];
    state[24] = conv ? 1.f : 0.f;
  }
  if (converged_out) converged_out[0] = conv;
}

}  // namespace
}  // namespace gsff

using namespace gsff;

extern "C" {

gsff_status gsff_tracking_masks(const float* t_rgb, const float* alpha, int32_t width,
                                int32_t height, float edge_threshold, float vis_threshold,
                                uint8_t* mask_v, uint8_t* mask_e, void* stream) {
  if (width <= 0 || height <= 0) return GSFF_ERR_INVALID_ARGUMENT;
  if ((mask_e && !t_rgb) || (mask_v && !alpha)) return GSFF_ERR_INVALID_ARGUMENT;
  if (!std::isfinite(edge_threshold) || !std::isfinite(vis_threshold) || edge_threshold < 0.f)
    return GSFF_ERR_INVALID_ARGUMENT;
  if (!mask_v && !mask_e) return GSFF_OK;
  const int64_t HW = (int64_t)width * height;
  const float e24 = 24.f * edge_threshold;
  hipLaunchKernelGGL(k_tracking_masks, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, t_rgb, alpha, (int)width, (int)height, e24 * e24,
                     vis_threshold, mask_v, mask_e);
  return hipGetLastError() == hipSuccess ? GSFF_OK : GSFF_ERR_HIP;
}

gsff_status gsff_pose_adam_step(float* viewmat, const float* d_pose, float* state, int32_t step,
                                float lr_trans, float lr_rot, float beta1, float beta2,
                                float eps, const gsff_pose_convergence* conv, float* delta,
                                uint32_t* converged, void* stream) {
  if (!viewmat || !d_pose || !state || step < 1) return GSFF_ERR_INVALID_ARGUMENT;
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) ||
      !std::isfinite(lr_trans) || !std::isfinite(lr_rot))
    return GSFF_ERR_INVALID_ARGUMENT;
  int window = 0;
  float tol_t = 0.f, tol_r = 0.f;
  if (conv) {
    if (conv->window < 1 || !(conv->tol_trans >= 0.f) || !(conv->tol_rot >= 0.f) ||
        !std::isfinite(conv->tol_trans) || !std::isfinite(conv->tol_rot))
      return GSFF_ERR_INVALID_ARGUMENT;
    window = conv->window;
    tol_t = conv->tol_trans;
    tol_r = conv->tol_rot;
  }
  hipLaunchKernelGGL(k_pose_adam_step, dim3(1), dim3(64), 0, (hipStream_t)stream, viewmat,
                     d_pose, state, (int)step, lr_trans, lr_rot, beta1, beta2, eps, window,
                     tol_t, tol_r, delta, converged);
  return hipGetLastError() == hipSuccess ? GSFF_OK : GSFF_ERR_HIP;
}

}  // extern "C"
