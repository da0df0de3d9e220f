// Per-Gaussian projection (Sec. 3.1: Eq. 1 covariance and its perspective
// splat) and its adjoint with the pose terms (Sec. 3.2, Eq. 4), device code
// shared by the preprocess kernel and the preprocess-adjoint kernel so both
// see bit-identical intermediates.  Templated on the scalar type: the
// rendering path instantiates FP32, and an FP64 instantiation of the same
// code lets finite differences check the adjoint's derivatives.
//
// The 2D covariance is formed as Sigma' = (T M)(T M)^T + dilation I with
// T = J R (2x3: projection Jacobian times the view rotation) and M = R_q S,
// which equals J R (R_q S S^T R_q^T) R^T J^T (Eq. 1 pushed through the
// linearised projection) and stays positive semi-definite in rounding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsff_internal.h"

namespace gsff {

template <typename R>
struct ProjT {
  bool valid;
  R x, y, z;            // camera-space mean
  R q[4];               // normalised quaternion (w, x, y, z)
  R qinv;               // 1 / |q|
  R s[3];               // activated scales
  R o;                  // activated opacity
  R Rq[9];              // rotation of the quaternion, row-major
  R TM[6];              // (J R)(R_q S), 2x3 row-major
  R J00, J02, J11, J12; // non-zero entries of the 2x3 Jacobian
  R a, b, c;            // dilated 2D covariance
  R A, B, Cc;           // its inverse (conic)
  R u, v;               // image-plane mean
  uint32_t key;         // depth sort key: float32 bits of z formed in FP64
};
using Proj = ProjT<float>;

__device__ __forceinline__ bool finite_f(float v) { return __builtin_isfinite(v); }
__device__ __forceinline__ bool finite_f(double v) { return __builtin_isfinite(v); }
__device__ __forceinline__ float r_exp(float v) { return expf(v); }
__device__ __forceinline__ double r_exp(double v) { return exp(v); }
__device__ __forceinline__ float r_sqrt(float v) { return sqrtf(v); }
__device__ __forceinline__ double r_sqrt(double v) { return sqrt(v); }

// Camera-space depth in FP64 with a fixed association and no contraction:
// ((r20 x + r21 y) + r22 z) + t2.  Products of two FP32 values are exact in
// FP64, so only the three additions round.
template <typename R>
__device__ __forceinline__ double depth_fp64(const R* V, R mx, R my, R mz) {
  double p0 = __dmul_rn((double)V[8], (double)mx);
  double p1 = __dmul_rn((double)V[9], (double)my);
  double p2 = __dmul_rn((double)V[10], (double)mz);
  return __dadd_rn(__dadd_rn(__dadd_rn(p0, p1), p2), (double)V[11]);
}

template <typename R>
__device__ __forceinline__ void quat_rot(const R* q, R* Rm) {
  const R w = q[0], x = q[1], y = q[2], z = q[3];
  Rm[0] = R(1) - R(2) * (y * y + z * z);
  Rm[1] = R(2) * (x * y - w * z);
  Rm[2] = R(2) * (x * z + w * y);
  Rm[3] = R(2) * (x * y + w * z);
  Rm[4] = R(1) - R(2) * (x * x + z * z);
  Rm[5] = R(2) * (y * z - w * x);
  Rm[6] = R(2) * (x * z - w * y);
  Rm[7] = R(2) * (y * z + w * x);
  Rm[8] = R(1) - R(2) * (x * x + y * y);
}

// Projection of one Gaussian from its raw parameters (mean, log-scales,
// quaternion, opacity logit); V is the 3x4 row-major view matrix.  The FP32
// path and the FP64 instantiation (finite-difference checks) share it.
template <typename R>
__device__ __forceinline__ ProjT<R> project_core(R mx, R my, R mz, R ls0, R ls1, R ls2, R qw,
                                                 R qx, R qy, R qz, R lo, const R* V, int W,
                                                 int H, R fx, R fy, R cx, R cy,
                                                 const DevSettings& st) {
  ProjT<R> p;
  p.valid = false;
  p.key = 0xFFFFFFFFu;
  if (!(finite_f(mx) && finite_f(my) && finite_f(mz) && finite_f(qw) && finite_f(qx) &&
        finite_f(qy) && finite_f(qz) && finite_f(lo)))
    return p;
  if (ls0 != ls0 || ls1 != ls1 || ls2 != ls2 || ls0 == INFINITY || ls1 == INFINITY ||
      ls2 == INFINITY)
    return p;
  const double z64 = depth_fp64(V, mx, my, mz);
  p.x = V[0] * mx + V[1] * my + V[2] * mz + V[3];
  p.y = V[4] * mx + V[5] * my + V[6] * mz + V[7];
  p.z = (R)z64;
  if (!(z64 > (double)st.near_plane)) return p;
  const R rz = R(1) / p.z;
  const R limx = (R)st.guard * (R)W / (R(2) * fx);
  const R limy = (R)st.guard * (R)H / (R(2) * fy);
  if (fabs(p.x * rz) > limx || fabs(p.y * rz) > limy) return p;
  const R qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
  if (!(qn2 > R(0))) return p;
  const R qn = r_sqrt(qn2);
  p.qinv = R(1) / qn;
  p.q[0] = qw * p.qinv;
  p.q[1] = qx * p.qinv;
  p.q[2] = qy * p.qinv;
  p.q[3] = qz * p.qinv;
  p.s[0] = r_exp(ls0);
  p.s[1] = r_exp(ls1);
  p.s[2] = r_exp(ls2);
  p.o = R(1) / (R(1) + r_exp(-lo));
  if (p.o < (R)st.alpha_min) return p;
  quat_rot(p.q, p.Rq);
  // Jacobian of the pinhole projection at the camera-space mean
  p.J00 = fx * rz;
  p.J02 = -fx * p.x * rz * rz;
  p.J11 = fy * rz;
  p.J12 = -fy * p.y * rz * rz;
  // T = J R (rows of the view rotation R are V[0..2], V[4..6], V[8..10])
  R T[6];
  for (int k = 0; k < 3; ++k) {
    T[k] = p.J00 * V[k] + p.J02 * V[8 + k];
    T[3 + k] = p.J11 * V[4 + k] + p.J12 * V[8 + k];
  }
  // TM = T (R_q S)
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) {
      R acc = R(0);
      for (int l = 0; l < 3; ++l) acc += T[3 * r + l] * p.Rq[3 * l + k];
      p.TM[3 * r + k] = acc * p.s[k];
    }
  p.a = p.TM[0] * p.TM[0] + p.TM[1] * p.TM[1] + p.TM[2] * p.TM[2] + (R)st.dilation;
  p.b = p.TM[0] * p.TM[3] + p.TM[1] * p.TM[4] + p.TM[2] * p.TM[5];
  p.c = p.TM[3] * p.TM[3] + p.TM[4] * p.TM[4] + p.TM[5] * p.TM[5] + (R)st.dilation;
  const R det = p.a * p.c - p.b * p.b;
  if (!(det > R(0)) || !finite_f(det)) return p;
  const R idet = R(1) / det;
  p.A = p.c * idet;
  p.B = -p.b * idet;
  p.Cc = p.a * idet;
  p.u = fx * p.x * rz + cx;
  p.v = fy * p.y * rz + cy;
  union {
    float f;
    uint32_t u;
  } kb;
  kb.f = (float)p.z;
  p.key = kb.u;
  p.valid = true;
  return p;
}

// Full projection of Gaussian i (FP32 parameters).
__device__ __forceinline__ Proj project_gaussian(const DevGaussians& g, const DevCamera& cam,
                                                 const DevSettings& st, const float* V,
                                                 int64_t i) {
  const int64_t P = g.P;
  return project_core<float>(g.means[i], g.means[P + i], g.means[2 * P + i], g.log_scales[i],
                             g.log_scales[P + i], g.log_scales[2 * P + i], g.quats[i],
                             g.quats[P + i], g.quats[2 * P + i], g.quats[3 * P + i], g.logit[i],
                             V, cam.W, cam.H, cam.fx, cam.fy, cam.cx, cam.cy, st);
}


// Adjoint of project_core: from the image-space gradients d = (du, dv, dA,
// dB, dC, dopacity, -, -, -, dz) to the world mean, the log-scales, the raw
// quaternion and the opacity logit, and the Gaussian's pose terms of Eq. 4
// (left perturbation, rho then theta).  p must be valid.
template <typename R>
__device__ __forceinline__ void project_adjoint(const ProjT<R>& p, const R* V, R fx, R fy,
                                              const R* d, R* dmean, R* dls, R* dq, R& dlogit,
                                              R* pose) {
  const R du = d[0], dv = d[1], dA = d[2], dB = d[3], dC = d[4], dop = d[5], dz = d[9];
  dlogit = dop * p.o * (R(1) - p.o);
  // conic -> 2D covariance: G = -K Gk K with Gk = [[dA, dB/2], [dB/2, dC]]
  const R hB = R(0.5) * dB;
  const R k00 = p.A * dA + p.B * hB, k01 = p.A * hB + p.B * dC;
  const R k10 = p.B * dA + p.Cc * hB, k11 = p.B * hB + p.Cc * dC;
  const R G00 = -(k00 * p.A + k01 * p.B);
  const R G01 = -(k00 * p.B + k01 * p.Cc);
  const R G11 = -(k10 * p.B + k11 * p.Cc);
  // Sigma' = TM TM^T:  dTM = 2 G TM
  R dTM[6];
  for (int k = 0; k < 3; ++k) {
    dTM[k] = R(2) * (G00 * p.TM[k] + G01 * p.TM[3 + k]);
    dTM[3 + k] = R(2) * (G01 * p.TM[k] + G11 * p.TM[3 + k]);
  }
  // TM[r][k] = sum_l T[r][l] Rq[l][k] s_k
  R T[6];
  for (int k = 0; k < 3; ++k) {
    T[k] = p.J00 * V[k] + p.J02 * V[8 + k];
    T[3 + k] = p.J11 * V[4 + k] + p.J12 * V[8 + k];
  }
  R dM[9];  // d/d(Rq S)
  for (int l = 0; l < 3; ++l)
    for (int k = 0; k < 3; ++k) dM[3 * l + k] = T[l] * dTM[k] + T[3 + l] * dTM[3 + k];
  R dT[6];  // d/dT = dTM (Rq S)^T
  for (int r = 0; r < 2; ++r)
    for (int l = 0; l < 3; ++l) {
      R acc = R(0);
      for (int k = 0; k < 3; ++k) acc += dTM[3 * r + k] * p.Rq[3 * l + k] * p.s[k];
      dT[3 * r + l] = acc;
    }
  R dRq[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) dRq[3 * r + k] = dM[3 * r + k] * p.s[k];
  for (int k = 0; k < 3; ++k) {
    const R ds = dM[k] * p.Rq[k] + dM[3 + k] * p.Rq[3 + k] + dM[6 + k] * p.Rq[6 + k];
    dls[k] = ds * p.s[k];
  }
  const R qw = p.q[0], qx = p.q[1], qy = p.q[2], qz = p.q[3];
  const R* Gq = dRq;
  R dqn[4];
  dqn[0] = R(2) * (-qz * Gq[1] + qy * Gq[2] + qz * Gq[3] - qx * Gq[5] - qy * Gq[6] + qx * Gq[7]);
  dqn[1] = R(2) * (qy * Gq[1] + qz * Gq[2] + qy * Gq[3] - R(2) * qx * Gq[4] - qw * Gq[5] +
                  qz * Gq[6] + qw * Gq[7] - R(2) * qx * Gq[8]);
  dqn[2] = R(2) * (-R(2) * qy * Gq[0] + qx * Gq[1] + qw * Gq[2] + qx * Gq[3] + qz * Gq[5] -
                  qw * Gq[6] + qz * Gq[7] - R(2) * qy * Gq[8]);
  dqn[3] = R(2) * (-R(2) * qz * Gq[0] - qw * Gq[1] + qx * Gq[2] + qw * Gq[3] - R(2) * qz * Gq[4] +
                  qy * Gq[5] + qx * Gq[6] + qy * Gq[7]);
  const R qd = qw * dqn[0] + qx * dqn[1] + qy * dqn[2] + qz * dqn[3];
  for (int k = 0; k < 4; ++k) dq[k] = (dqn[k] - p.q[k] * qd) * p.qinv;
  // T = J R:  dJ = dT R^T (only J00, J02, J11, J12 vary),  dR = J^T dT
  const R dJ00 = dT[0] * V[0] + dT[1] * V[1] + dT[2] * V[2];
  const R dJ02 = dT[0] * V[8] + dT[1] * V[9] + dT[2] * V[10];
  const R dJ11 = dT[3] * V[4] + dT[4] * V[5] + dT[5] * V[6];
  const R dJ12 = dT[3] * V[8] + dT[4] * V[9] + dT[5] * V[10];
  R dR[9];
  for (int l = 0; l < 3; ++l) {
    dR[l] = p.J00 * dT[l];
    dR[3 + l] = p.J11 * dT[3 + l];
    dR[6 + l] = p.J02 * dT[l] + p.J12 * dT[3 + l];
  }
  // camera-space mean: image position, Jacobian, blended depth
  const R rz = R(1) / p.z, rz2 = rz * rz, rz3 = rz2 * rz;
  R gm0 = du * fx * rz + dJ02 * (-fx * rz2);
  R gm1 = dv * fy * rz + dJ12 * (-fy * rz2);
  R gm2 = du * (-fx * p.x * rz2) + dv * (-fy * p.y * rz2) +
              dJ00 * (-fx * rz2) + dJ02 * (R(2) * fx * p.x * rz3) +
              dJ11 * (-fy * rz2) + dJ12 * (R(2) * fy * p.y * rz3) + dz;
  // world mean: R^T gm
  for (int k = 0; k < 3; ++k) dmean[k] = V[k] * gm0 + V[4 + k] * gm1 + V[8 + k] * gm2;
  // pose, left perturbation (Eq. 4): rho += gm, theta += mc x gm + sum_k R[:,k] x dR[:,k]
  pose[0] = gm0;
  pose[1] = gm1;
  pose[2] = gm2;
  pose[3] = p.y * gm2 - p.z * gm1;
  pose[4] = p.z * gm0 - p.x * gm2;
  pose[5] = p.x * gm1 - p.y * gm0;
  for (int k = 0; k < 3; ++k) {
    const R c0 = V[k], c1 = V[4 + k], c2 = V[8 + k];
    const R e0 = dR[k], e1 = dR[3 + k], e2 = dR[6 + k];
    pose[3] += c1 * e2 - c2 * e1;
    pose[4] += c2 * e0 - c0 * e2;
    pose[5] += c0 * e1 - c1 * e0;
  }
}

}  // namespace gsff
