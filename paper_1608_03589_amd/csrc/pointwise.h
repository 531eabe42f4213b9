// Per-pixel arithmetic that every kernel of the library shares, so that two
// kernels computing the same quantity agree bit for bit.
//
// Projection onto the ball {|p| <= lam} (the prox of the regulariser's
// conjugate): P(q) = c q with c = min(1, lam / |q|).  1 / |q| is the
// hardware reciprocal square root of |q|^2 (about 1 ulp), which replaces a
// correctly rounded square root and an IEEE division; the two roundings
// differ by ~1e-7 relative, far inside the tolerance against the float64
// oracle.  The projection acts where c < 1 (the forward sweeps and the
// adjoints take that same decision from the same c).  At q = 0 the
// reciprocal is +inf and lam / |q| is +inf, or NaN when lam = 0; the
// minimum (IEEE minNum, which returns the other operand of a NaN) is 1
// either way, and P(0) = 0.
//
// Data prox: f^{k+1} = (f^k + tau (g + div p)) * (1 / (1 + tau)), the
// reciprocal formed once per launch with an IEEE division; g + div p is the
// sum the extrapolation from the prox also uses.
//
// The update formulas are written with explicit fused multiply-adds (one
// rounding instead of two): fbar = fma(theta, f - f_prev, f) or
// fma(theta tau, (g + d) - f, f), q = fma(sigma,
// grad, p), |q|^2 = fma(qx, qx, qy^2) (3D: fma(qz, qz, that)), and
// f^{k+1} = fma(tau, g + d, f) * (1 / (1 + tau)).  They cut the
// instruction count of the blocked sweeps by about a fifth; no implicit
// contraction happens anywhere else (-ffp-contract=off).
#pragma once

#include <hip/hip_runtime.h>

namespace tvpd {
namespace dev {

// 1 / |q| from |q|^2 (+inf at q = 0).
__device__ __forceinline__ float inv_norm(float n2) {
  return __builtin_amdgcn_rsqf(n2);
}

// Scale c with P_lam(q) = c q, for n2 = |q|^2 and the reciprocal r of |q|.
__device__ __forceinline__ float ball_scale_r(float r, float lam) {
  return fminf(1.0f, lam * r);
}
__device__ __forceinline__ float ball_scale(float n2, float lam) {
  return ball_scale_r(inv_norm(n2), lam);
}

// fbar = f + theta (f - f_prev).
__device__ __forceinline__ float extrap(float f, float f_prev, float theta) {
  return fmaf(theta, f - f_prev, f);
}

// fbar^k from the data prox that produced f^k: with tau that step and
// d^k = div p^k, f^{k-1} = (1 + tau) f^k - tau (g + d^k), so
// f^k + theta (f^k - f^{k-1}) = f^k + theta tau (g + d^k - f^k).
// thtau = theta * tau.
__device__ __forceinline__ float extrap_prox(float f, float g, float d,
                                             float thtau) {
  return fmaf(thtau, (g + d) - f, f);
}

// Data prox f^{k+1} = (f + tau (g + d)) * iopt, iopt = 1 / (1 + tau).
__device__ __forceinline__ float data_prox(float f, float g, float d,
                                           float tau, float iopt) {
  return fmaf(tau, g + d, f) * iopt;
}

// One component of the dual argument q = p + sigma grad fbar.
__device__ __forceinline__ float dual_arg(float p, float sigma, float grad) {
  return fmaf(sigma, grad, p);
}

// |q|^2 in 2D and 3D.
__device__ __forceinline__ float sq2(float a, float b) {
  return fmaf(a, a, b * b);
}
__device__ __forceinline__ float sq3(float a, float b, float c) {
  return fmaf(c, c, fmaf(a, a, b * b));
}

// 1 / (1 + tau), the factor of the data prox.
__device__ __forceinline__ float prox_factor(float tau) {
  return 1.0f / (1.0f + tau);
}

}  // namespace dev
}  // namespace tvpd
