// Per-pair steps of the compositing (Sec. 3.1, Eqs. 2-3) and of its adjoint,
// templated on the scalar type: the FP32 compositing adjoint calls the
// back-to-front step and the moments-to-gradient step, and the FP64
// instantiation that finite differences check calls all three.
#pragma once

#include <hip/hip_runtime.h>

namespace gsff {

__device__ __forceinline__ float r_rcp(float v) { return __builtin_amdgcn_rcpf(v); }  // 1 ulp
__device__ __forceinline__ double r_rcp(double v) { return 1.0 / v; }
__device__ __forceinline__ float r_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double r_fma(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

// One front-to-back step at a pixel (Eq. 3).  A pair is used when the pixel
// has not stopped and alpha >= alpha_min; the pixel stops before a Gaussian
// that would take its transmittance below t_min (that Gaussian is not
// blended).  Gives the blending weight alpha T (0 if unused) and whether the
// pair was used, and updates T and the stop flag.  (The FP32 forward kernel
// spells this step out inline in the same operations: routed through this
// function its boolean logic compiled differently and spilled.)
template <typename R>
__device__ __forceinline__ R blend_step(R alpha, R& T, bool& done, bool& use, R alpha_min,
                                        R t_min) {
  const bool valid = !done && alpha >= alpha_min;
  const R aT = alpha * T;
  const R Tn = r_fma(-alpha, T, T);  // T (1 - alpha), one rounding
  const bool stop = valid && Tn < t_min;
  use = valid && !stop;
  done = done || stop;
  const R wgt = use ? aT : R(0);
  T = use ? Tn : T;
  return wgt;
}

// One back-to-front step of the adjoint at a pixel.  al is the pair's alpha,
// or 0 for a pair the pixel did not use (then 1 / (1 - al) = 1, T passes
// through and the weight is 0).  On entry T is the transmittance behind the
// Gaussian and D the upstream-weighted sum of what is blended behind it; gc
// is the upstream-weighted value of the Gaussian (colour and depth) and gaT
// the alpha upstream times the final transmittance.  Gives the weight and
// dL/dalpha = T_front gc + (gaT - D) / (1 - alpha), and moves T and D in
// front of the Gaussian.
template <typename R>
__device__ __forceinline__ void back_step(R al, R gc, R gaT, R& T, R& D, R& wv, R& dal) {
  const R inv = r_rcp(R(1) - al);
  const R Tb = T * inv;
  wv = al * Tb;
  dal = Tb * gc + (gaT - D) * inv;
  D = r_fma(wv, gc, D);
  T = Tb;
}

// Image-space gradients of one Gaussian from one tile, through the moments
// of g_p = dL/dpower over the tile's pixels: M = sum_p g_p (1, x, y, x^2, xy,
// y^2) with (x, y) the pixel centre relative to the tile centre.  (udx, vdy)
// is the mean relative to the tile centre, (cA, cB, cC) the conic of Eq. 2
// (power = -(A dx^2 + 2 B dx dy + C dy^2) / 2 with dx = u - x), o the
// opacity (dalpha/do = G = oG / o).  Out: du, dv, dA, dB, dC, do.
template <typename R>
__device__ __forceinline__ void geo_from_moments(R cA, R cB, R cC, R o, R udx, R vdy, const R* M,
                                                 R* geo) {
  const R Sx = udx * M[0] - M[1], Sy = vdy * M[0] - M[2];
  const R Sxx = udx * udx * M[0] - R(2) * udx * M[1] + M[3];
  const R Sxy = udx * vdy * M[0] - udx * M[2] - vdy * M[1] + M[4];
  const R Syy = vdy * vdy * M[0] - R(2) * vdy * M[2] + M[5];
  geo[0] = -(cA * Sx + cB * Sy);
  geo[1] = -(cB * Sx + cC * Sy);
  geo[2] = R(-0.5) * Sxx;
  geo[3] = -Sxy;
  geo[4] = R(-0.5) * Syy;
  geo[5] = o > R(0) ? M[0] * r_rcp(o) : R(0);
}

}  // namespace gsff
