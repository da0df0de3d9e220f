// Per-Gaussian projection (Sec. 3.1: Eq. 1 covariance and its perspective
// splat) and its adjoint, FP32 device code shared by the preprocess kernel and
// the preprocess-adjoint kernel so both see bit-identical intermediates.
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

struct Proj {
  bool valid;
  float x, y, z;            // camera-space mean
  float q[4];               // normalised quaternion (w, x, y, z)
  float qinv;               // 1 / |q|
  float s[3];               // activated scales
  float o;                  // activated opacity
  float Rq[9];              // rotation of the quaternion, row-major
  float TM[6];              // (J R)(R_q S), 2x3 row-major
  float J00, J02, J11, J12; // non-zero entries of the 2x3 Jacobian
  float a, b, c;            // dilated 2D covariance
  float A, B, Cc;           // its inverse (conic)
  float u, v;               // image-plane mean
  uint32_t key;             // depth sort key: float32 bits of z formed in FP64
};

__device__ __forceinline__ bool finite_f(float v) { return __builtin_isfinite(v); }

// Camera-space depth in FP64 with a fixed association and no contraction:
// ((r20 x + r21 y) + r22 z) + t2.  Products of two FP32 values are exact in
// FP64, so only the three additions round.
__device__ __forceinline__ double depth_fp64(const float* V, float mx, float my, float mz) {
  double p0 = __dmul_rn((double)V[8], (double)mx);
  double p1 = __dmul_rn((double)V[9], (double)my);
  double p2 = __dmul_rn((double)V[10], (double)mz);
  return __dadd_rn(__dadd_rn(__dadd_rn(p0, p1), p2), (double)V[11]);
}

__device__ __forceinline__ void quat_rot(const float* q, float* R) {
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.f - 2.f * (y * y + z * z);
  R[1] = 2.f * (x * y - w * z);
  R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z);
  R[4] = 1.f - 2.f * (x * x + z * z);
  R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y);
  R[7] = 2.f * (y * z + w * x);
  R[8] = 1.f - 2.f * (x * x + y * y);
}

// Full projection of Gaussian i.  V is the 3x4 row-major view matrix.
__device__ __forceinline__ Proj project_gaussian(const DevGaussians& g, const DevCamera& cam,
                                                 const DevSettings& st, const float* V,
                                                 int64_t i) {
  Proj p;
  p.valid = false;
  p.key = 0xFFFFFFFFu;
  const int64_t P = g.P;
  const float mx = g.means[i], my = g.means[P + i], mz = g.means[2 * P + i];
  const float ls0 = g.log_scales[i], ls1 = g.log_scales[P + i], ls2 = g.log_scales[2 * P + i];
  const float qw = g.quats[i], qx = g.quats[P + i], qy = g.quats[2 * P + i],
              qz = g.quats[3 * P + i];
  const float lo = g.logit[i];
  if (!(finite_f(mx) && finite_f(my) && finite_f(mz) && finite_f(qw) && finite_f(qx) &&
        finite_f(qy) && finite_f(qz) && finite_f(lo)))
    return p;
  if (ls0 != ls0 || ls1 != ls1 || ls2 != ls2 || ls0 == INFINITY || ls1 == INFINITY ||
      ls2 == INFINITY)
    return p;
  const double z64 = depth_fp64(V, mx, my, mz);
  p.x = V[0] * mx + V[1] * my + V[2] * mz + V[3];
  p.y = V[4] * mx + V[5] * my + V[6] * mz + V[7];
  p.z = (float)z64;
  if (!(z64 > (double)st.near_plane)) return p;
  const float rz = 1.f / p.z;
  const float limx = st.guard * (float)cam.W / (2.f * cam.fx);
  const float limy = st.guard * (float)cam.H / (2.f * cam.fy);
  if (fabsf(p.x * rz) > limx || fabsf(p.y * rz) > limy) return p;
  const float qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
  if (!(qn2 > 0.f)) return p;
  const float qn = sqrtf(qn2);
  p.qinv = 1.f / qn;
  p.q[0] = qw * p.qinv;
  p.q[1] = qx * p.qinv;
  p.q[2] = qy * p.qinv;
  p.q[3] = qz * p.qinv;
  p.s[0] = expf(ls0);
  p.s[1] = expf(ls1);
  p.s[2] = expf(ls2);
  p.o = 1.f / (1.f + expf(-lo));
  if (p.o < st.alpha_min) return p;
  quat_rot(p.q, p.Rq);
  // Jacobian of the pinhole projection at the camera-space mean
  p.J00 = cam.fx * rz;
  p.J02 = -cam.fx * p.x * rz * rz;
  p.J11 = cam.fy * rz;
  p.J12 = -cam.fy * p.y * rz * rz;
  // T = J R (rows of the view rotation R are V[0..2], V[4..6], V[8..10])
  float T[6];
  for (int k = 0; k < 3; ++k) {
    T[k] = p.J00 * V[k] + p.J02 * V[8 + k];
    T[3 + k] = p.J11 * V[4 + k] + p.J12 * V[8 + k];
  }
  // TM = T (R_q S)
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) {
      float acc = 0.f;
      for (int l = 0; l < 3; ++l) acc += T[3 * r + l] * p.Rq[3 * l + k];
      p.TM[3 * r + k] = acc * p.s[k];
    }
  p.a = p.TM[0] * p.TM[0] + p.TM[1] * p.TM[1] + p.TM[2] * p.TM[2] + st.dilation;
  p.b = p.TM[0] * p.TM[3] + p.TM[1] * p.TM[4] + p.TM[2] * p.TM[5];
  p.c = p.TM[3] * p.TM[3] + p.TM[4] * p.TM[4] + p.TM[5] * p.TM[5] + st.dilation;
  const float det = p.a * p.c - p.b * p.b;
  if (!(det > 0.f) || !finite_f(det)) return p;
  const float idet = 1.f / det;
  p.A = p.c * idet;
  p.B = -p.b * idet;
  p.Cc = p.a * idet;
  p.u = cam.fx * p.x * rz + cam.cx;
  p.v = cam.fy * p.y * rz + cam.cy;
  union {
    float f;
    uint32_t u;
  } kb;
  kb.f = p.z;
  p.key = kb.u;
  p.valid = true;
  return p;
}

}  // namespace gsff
