// Per-pixel arithmetic that every kernel of the library shares, so that two
// kernels computing the same quantity agree bit for bit.
//
// Projection onto the ball {|p| <= lam} (the prox of the regulariser's
// conjugate): P(q) = c q with c = lam / |q| outside the ball and c = 1
// inside.  c is formed from the hardware reciprocal square root of |q|^2
// (about 1 ulp), which replaces a correctly rounded square root and an IEEE
// division; the two roundings differ by ~1e-7 relative, far inside the
// tolerance against the float64 oracle.  The test |q|^2 > lam^2 decides the
// branch (the forward sweep and the adjoint make the same decision).
//
// Data prox: f^{k+1} = (f^k + tau div p + tau g) * (1 / (1 + tau)), the
// reciprocal formed once per launch with an IEEE division.
//
// The update formulas are written with explicit fused multiply-adds (one
// rounding instead of two): fbar = fma(theta, f - f_prev, f) or
// fma(theta tau, (g + d) - f, f), q = fma(sigma,
// grad, p), |q|^2 = fma(qx, qx, qy^2) (3D: fma(qz, qz, that)), and
// f^{k+1} = fma(tau, g, fma(tau, d, f)) * (1 / (1 + tau)).  They cut the
// instruction count of the blocked sweeps by about a fifth; no implicit
// contraction happens anywhere else (-ffp-contract=off).
#pragma once

#include <hip/hip_runtime.h>

namespace tvpd {
namespace dev {

// Smallest normal float: clamping |q|^2 to it keeps v_rsq_f32 finite (a
// zero or subnormal |q|^2 only occurs inside the ball, where c = 1, unless
// lam^2 is itself below it).
constexpr float kMinNormal = 1.17549435e-38f;

// 1 / |q| from |q|^2.
__device__ __forceinline__ float inv_norm(float n2) {
  return __builtin_amdgcn_rsqf(fmaxf(n2, kMinNormal));
}

// Scale c with P_lam(q) = c q, for n2 = |q|^2 and lam2 = lam * lam.
__device__ __forceinline__ float ball_scale(float n2, float lam, float lam2) {
  const float r = inv_norm(n2);
  return n2 > lam2 ? lam * r : 1.0f;
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
