// Kernels of the unrolled solver and of its hand-written adjoint.
//
// Forward step k (coefficients c_k = (lam_k, tau_k, sigma_k) read from device
// memory, theta fixed):
//     fbar    = f^k + theta (f^k - f^{k-1})
//     p^{k+1} = P_lam(p^k + sigma grad fbar)
//     f^{k+1} = (f^k + tau div p^{k+1} + tau g) / (1 + tau)
// 2D runs as passes of up to five iterations on the plain solver's strip tile
// (tile2d_xs.h, with this extrapolation and every iterate stored), 3D one
// iteration per launch on the plain solver's tile (tile3d.h), with the
// steps' coefficients read from device memory.
//
// Adjoint step k (reverse-mode derivative of the forward step; a = dL/df^{k+1},
// b = the part of dL/df^k collected from step k+1's extrapolation, r =
// dL/dp^{k+1}), in two passes that recompute the forward quantities with the
// forward's exact arithmetic, so the projection takes the same branch:
//   pass A (forward differences):  alpha = a / (1 + tau);  (times the
//       reciprocal of 1 + tau, as in the forward's data prox)
//       s = r - grad(tau alpha);  q = p^k + sigma grad fbar;  p^{k+1} = P(q);
//       t = s where |q| <= lam, else (lam/|q|)(s - n (n.s)) with n = q/|q|;
//       partial sums of  lambar = sum_{|q|>lam} n.s  and  sigmabar = sum t.grad fbar
//   pass B (backward differences):  d = div p^{k+1};  f^{k+1} recomputed;
//       gbar += tau alpha;  taubar = sum alpha (d + g - f^{k+1});
//       w = -sigma div t;  a' = alpha + b + (1 + theta) w;  b' = -theta w;  r' = t.
// After step 0, dL/dg = gbar + a + b (f^0 = f^{-1} = g).
//
// Per-pixel kernels run one pixel per thread, rows of up to 256 pixels per
// block; neighbour values are read directly (they are cache hits).
#include "adj2d.h"
#include "adj3d.h"
#include "tile2d.h"
#include "tile2d_xs.h"
#include "tile3d.h"
#include "unrolled.h"

namespace tvpd {
namespace {

using namespace dev;

constexpr int kRowBlock = 256;

struct Pix {
  int b, z, y, x;
  int64_t o;   // offset within the image plane
  bool ok;
};

__device__ __forceinline__ Pix pixel_at(const PlaneSet& P, int64_t blk) {
  Pix q;
  const int xc = (P.nx + kRowBlock - 1) / kRowBlock;
  const int64_t row = blk / xc;
  const int xchunk = (int)(blk - row * xc);
  q.x = xchunk * kRowBlock + threadIdx.x;
  const int64_t per = (int64_t)P.nz * P.ny;
  q.b = (int)(row / per);
  const int64_t rem = row - (int64_t)q.b * per;
  q.z = (int)(rem / P.ny);
  q.y = (int)(rem - (int64_t)q.z * P.ny);
  q.ok = q.x < P.nx && q.b < P.nb;
  q.o = ((int64_t)q.z * P.ny + q.y) * P.pitch + q.x;
  return q;
}

__device__ __forceinline__ Pix pixel_of(const PlaneSet& P) {
  return pixel_at(P, blockIdx.x);
}

__device__ __forceinline__ int64_t row_blocks(const PlaneSet& P) {
  return (int64_t)((P.nx + kRowBlock - 1) / kRowBlock) * P.nb * P.nz * P.ny;
}

__device__ __forceinline__ const float* cplane(const PlaneSet& P, int b,
                                               int id) {
  return P.base + (int64_t)b * P.istride + (int64_t)id * P.plane;
}
__device__ __forceinline__ float* plane(const PlaneSet& P, int b, int id) {
  return P.base + (int64_t)b * P.istride + (int64_t)id * P.plane;
}

template <int ND>
__device__ __forceinline__ void project(const float* q, float lam, float* p) {
  const float n2 = ND == 3 ? sq3(q[0], q[1], q[2]) : sq2(q[0], q[1]);
  const float c = ball_scale(n2, lam);
#pragma unroll
  for (int i = 0; i < ND; ++i) p[i] = q[i] * c;
}

// Strides along x, y, z of a pixel offset, and whether the pixel has a
// forward neighbour along each axis.
template <int ND>
__device__ __forceinline__ void axes(const PlaneSet& P, const Pix& q,
                                     int64_t* st, bool* fwd, bool* bwd) {
  st[0] = 1;
  st[1] = P.pitch;
  fwd[0] = q.x < P.nx - 1;
  fwd[1] = q.y < P.ny - 1;
  bwd[0] = q.x > 0;
  bwd[1] = q.y > 0;
  if (ND == 3) {
    st[2] = (int64_t)P.ny * P.pitch;
    fwd[2] = q.z < P.nz - 1;
    bwd[2] = q.z > 0;
  }
}

// q = p^k + sigma grad fbar at one pixel (forward differences, Neumann).
template <int ND>
__device__ __forceinline__ void dual_point(const float* fk, const float* fkm,
                                           const float* pk, int64_t PL,
                                           int64_t o, const int64_t* st,
                                           const bool* fwd, float sig,
                                           float th, float* q, float* gfb) {
  const float f0 = fk[o];
  const float fb = extrap(f0, fkm[o], th);
#pragma unroll
  for (int c = 0; c < ND; ++c) {
    float gc = 0.0f;
    if (fwd[c]) {
      const float f1 = fk[o + st[c]];
      const float fb1 = extrap(f1, fkm[o + st[c]], th);
      gc = fb1 - fb;
    }
    gfb[c] = gc;
    q[c] = dual_arg(pk[c * PL + o], sig, gc);
  }
}

// div v at one pixel (backward differences; v_c vanishes at the last index)
template <int ND>
__device__ __forceinline__ float div_point(const float* v, int64_t PL,
                                           int64_t o, const int64_t* st,
                                           const bool* bwd) {
  float d = 0.0f;
#pragma unroll
  for (int c = 0; c < ND; ++c) {
    const float here = v[c * PL + o];
    const float prev = bwd[c] ? v[c * PL + o - st[c]] : 0.0f;
    d = (c == 0) ? (here - prev) : d + (here - prev);
  }
  return d;
}

// ----------------------------- forward ------------------------------------

// Iterations k .. k+S-1 of every image in one launch (tile2d_xs.h with the
// extrapolation as defined, per-stage coefficients read from device memory,
// and every iterate stored to its plane slot).
template <int S>
__global__ __launch_bounds__(kMaxBlock) void u_sweep2d_xs_kernel(
    PlaneSet P, PassIds ids, const float* __restrict__ coeffs, int k,
    float theta, int th_rows, int wpb, int ntx, int nty) {
  const int b = blockIdx.y;
  // (not wave_in_block(): with uniform tile coordinates the compiler's
  // schedule of the depth-5 walk needs more than 256 registers)
  const int wave = threadIdx.x / kWave;
  const int nbx = gridDim.x, bx = blockIdx.x;
  const int q8 = nbx >> 3, r8 = nbx & 7, xcd = bx & 7;
  const int bt = xcd * q8 + min(xcd, r8) + (bx >> 3);
  const int wt = bt * wpb + wave;
  if (wt >= ntx * nty) return;
  const int ty = wt / ntx, tx = wt - ty * ntx;
  TileCtxS c;
  c.F = cplane(P, b, ids.fk);
  c.MF = cplane(P, b, ids.fkm);
  c.PX = cplane(P, b, ids.pk);
  c.PY = cplane(P, b, ids.pk + 1);
  c.G = cplane(P, b, 0);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    c.SF[s] = plane(P, b, ids.fn[s]);
    c.SQX[s] = plane(P, b, ids.pn[s]);
    c.SQY[s] = plane(P, b, ids.pn[s] + 1);
    c.slam[s] = coeffs[3 * (k + s)];
    c.stau[s] = coeffs[3 * (k + s) + 1];
    c.ssig[s] = coeffs[3 * (k + s) + 2];
  }
  c.FN = c.QX = c.QY = nullptr;
  c.ny = P.ny;
  c.nx = P.nx;
  c.pitch = P.pitch;
  c.x0 = tx * xs_owned(S);
  c.y0 = ty * th_rows;
  c.y1 = min(c.y0 + th_rows, P.ny);
  c.lam = c.slam[0];
  c.tau = c.stau[0];
  c.sig = c.ssig[0];
  c.th = theta;
  c.tau_prev = 0.0f;
  double sg = 0.0, sp = 0.0;
  sweep_tile_xs<S, xs_margin(S), false, true, false, true>(c, sg, sp);
}

template <int TH>
__global__ __launch_bounds__(kMaxBlock) void u_sweep3d_kernel(
    PlaneSet P, StepIds ids, const float* __restrict__ coeffs, int k,
    float theta, int tz, int wpb, int ntx, int nty, int ntiles) {
  const int b = blockIdx.y;
  // (not wave_in_block(): measured 2-3 % slower in the 3D kernels)
  const int wave = threadIdx.x / kWave;
  const int nbx = gridDim.x, bx = blockIdx.x;
  const int q8 = nbx >> 3, r8 = nbx & 7, xcd = bx & 7;
  const int bt = xcd * q8 + min(xcd, r8) + (bx >> 3);
  const int wt = bt * wpb + wave;
  if (wt >= ntiles) return;
  const int per_seg = ntx * nty;
  const int tzi = wt / per_seg;
  const int rem = wt - tzi * per_seg;
  const int ty = rem / ntx, tx = rem - ty * ntx;
  Tile3DCtx c;
  c.fk = cplane(P, b, ids.fk);
  c.fkm = cplane(P, b, ids.fkm);
  c.pk = cplane(P, b, ids.pk);
  c.g = cplane(P, b, 0);
  c.fn = plane(P, b, ids.fn);
  c.pn = plane(P, b, ids.pn);
  c.cs = P.plane;
  c.nz = P.nz;
  c.ny = P.ny;
  c.nx = P.nx;
  c.pitch = P.pitch;
  c.x0 = tx * kStripCols;
  c.y0 = ty * TH;
  c.z0 = tzi * tz;
  c.z1 = min(c.z0 + tz, P.nz);
  c.lam = coeffs[3 * k];
  c.tau = coeffs[3 * k + 1];
  c.sig = coeffs[3 * k + 2];
  c.th = theta;
  double sg = 0.0, sp = 0.0;
  sweep_tile3d<TH, false>(c, sg, sp);
}

// ----------------------------- adjoint ------------------------------------

__device__ __forceinline__ void block_sum(double& a, double& b,
                                          double (*red)[kMaxBlock / kWave]) {
  block_sum2(a, b, red);
}

template <int ND>
__global__ __launch_bounds__(kRowBlock) void u_adjA_kernel(
    PlaneSet P, AdjIds ids, const float* __restrict__ coeffs, int k,
    float theta, double* __restrict__ partials) {
  __shared__ double red[2][kMaxBlock / kWave];
  double lb = 0.0, sb = 0.0;
  const int64_t nrow = row_blocks(P);
  for (int64_t rb = blockIdx.x; rb < nrow; rb += gridDim.x) {
    const Pix q = pixel_at(P, rb);
    if (!q.ok) continue;
    int64_t st[3];
    bool fwd[3], bwd[3];
    axes<ND>(P, q, st, fwd, bwd);
    const float lam = coeffs[3 * k], tau = coeffs[3 * k + 1],
                sig = coeffs[3 * k + 2];
    const float iopt = prox_factor(tau);
    const float* a = cplane(P, q.b, ids.a_in);
    const float* r = cplane(P, q.b, ids.r_in);
    const float ta0 = tau * (a[q.o] * iopt);
    float s[ND];
#pragma unroll
    for (int c = 0; c < ND; ++c) {
      const float gc = fwd[c] ? tau * (a[q.o + st[c]] * iopt) - ta0 : 0.0f;
      s[c] = r[c * P.plane + q.o] - gc;
    }
    float qq[ND], gfb[ND], pn[ND];
    dual_point<ND>(cplane(P, q.b, ids.fk), cplane(P, q.b, ids.fkm),
                   cplane(P, q.b, ids.pk), P.plane, q.o, st, fwd, sig, theta,
                   qq, gfb);
    project<ND>(qq, lam, pn);
    const float n2 = ND == 3 ? sq3(qq[0], qq[1], qq[2]) : sq2(qq[0], qq[1]);
    float t[ND];
    const float rn = inv_norm(n2);
    if (ball_scale_r(rn, lam) < 1.0f) {  // the forward's branch (ball_scale)
      float nv[ND];
      float ns = 0.0f;
#pragma unroll
      for (int c = 0; c < ND; ++c) {
        nv[c] = qq[c] * rn;
        ns = (c == 0) ? nv[c] * s[c] : ns + nv[c] * s[c];
      }
      const float sc = lam * rn;
#pragma unroll
      for (int c = 0; c < ND; ++c) t[c] = sc * (s[c] - nv[c] * ns);
      lb += ns;
    } else {
#pragma unroll
      for (int c = 0; c < ND; ++c) t[c] = s[c];
    }
    float* pno = plane(P, q.b, ids.pn);
    float* to = plane(P, q.b, ids.t_out);
#pragma unroll
    for (int c = 0; c < ND; ++c) {
      pno[c * P.plane + q.o] = pn[c];
      to[c * P.plane + q.o] = t[c];
      sb += (double)t[c] * (double)gfb[c];
    }
  }
  block_sum(lb, sb, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = lb;
    partials[2 * blockIdx.x + 1] = sb;
  }
}

template <int ND>
__global__ __launch_bounds__(kRowBlock) void u_adjB_kernel(
    PlaneSet P, AdjIds ids, const float* __restrict__ coeffs, int k,
    float theta, double* __restrict__ partials) {
  __shared__ double red[2][kMaxBlock / kWave];
  double tb = 0.0, unused = 0.0;
  const int64_t nrow = row_blocks(P);
  for (int64_t rb = blockIdx.x; rb < nrow; rb += gridDim.x) {
    const Pix q = pixel_at(P, rb);
    if (!q.ok) continue;
    int64_t st[3];
    bool fwd[3], bwd[3];
    axes<ND>(P, q, st, fwd, bwd);
    const float tau = coeffs[3 * k + 1], sig = coeffs[3 * k + 2];
    const float iopt = prox_factor(tau);
    const float d =
        div_point<ND>(cplane(P, q.b, ids.pn), P.plane, q.o, st, bwd);
    const float f = cplane(P, q.b, ids.fk)[q.o];
    const float g = cplane(P, q.b, ids.g)[q.o];
    const float fn = data_prox(f, g, d, tau, iopt);
    const float alpha = cplane(P, q.b, ids.a_in)[q.o] * iopt;
    float* gbar = plane(P, q.b, ids.gbar);
    gbar[q.o] = gbar[q.o] + tau * alpha;
    tb += (double)alpha * (((double)d + (double)g) - (double)fn);
    const float dt =
        div_point<ND>(cplane(P, q.b, ids.t_out), P.plane, q.o, st, bwd);
    const float w = -sig * dt;
    const float bb = cplane(P, q.b, ids.b_in)[q.o];
    plane(P, q.b, ids.a_out)[q.o] = (alpha + bb) + (1.0f + theta) * w;
    plane(P, q.b, ids.b_out)[q.o] = -theta * w;
  }
  block_sum(tb, unused, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = tb;
}

// Fused 2D adjoint step (adj2d.h): one pass over wave tiles of th rows; block
// (bx, image b) writes its (lambar, sigmabar) partials to pa and its taubar
// partial to pb at index b * gridDim.x + bx.
__global__ __launch_bounds__(kMaxBlock) void u_adj2d_kernel(
    PlaneSet P, AdjIds ids, const float* __restrict__ coeffs, int k,
    float theta, int th_rows, int wpb, int ntx, int nty,
    double* __restrict__ pa, double* __restrict__ pb) {
  __shared__ double red[2][kMaxBlock / kWave];
  const int b = blockIdx.y;
  const int wave = wave_in_block();
  const int nbx = gridDim.x, bx = blockIdx.x;
  const int q8 = nbx >> 3, r8 = nbx & 7, xcd = bx & 7;
  const int bt = xcd * q8 + min(xcd, r8) + (bx >> 3);
  const int wt = bt * wpb + wave;
  double l = 0.0, sg = 0.0, t = 0.0;
  if (wt < ntx * nty) {
    const int ty = wt / ntx, tx = wt - ty * ntx;
    AdjCtx2D c;
    c.fk = cplane(P, b, ids.fk);
    c.fkm = cplane(P, b, ids.fkm);
    c.px = cplane(P, b, ids.pk);
    c.py = cplane(P, b, ids.pk + 1);
    c.g = cplane(P, b, ids.g);
    c.a = cplane(P, b, ids.a_in);
    c.b = cplane(P, b, ids.b_in);
    c.rx = cplane(P, b, ids.r_in);
    c.ry = cplane(P, b, ids.r_in + 1);
    c.ao = plane(P, b, ids.a_out);
    c.bo = plane(P, b, ids.b_out);
    c.tx = plane(P, b, ids.t_out);
    c.ty = plane(P, b, ids.t_out + 1);
    c.gbar = plane(P, b, ids.gbar);
    c.ny = P.ny;
    c.nx = P.nx;
    c.pitch = P.pitch;
    c.x0 = tx * kStripCols;
    c.y0 = ty * th_rows;
    c.y1 = min(c.y0 + th_rows, P.ny);
    c.lam = coeffs[3 * k];
    c.tau = coeffs[3 * k + 1];
    c.sig = coeffs[3 * k + 2];
    c.th = theta;
    adj_tile2d(c, l, sg, t);
  }
  block_sum2(l, sg, red);
  __syncthreads();
  double unused = 0.0;
  block_sum2(t, unused, red);
  if (threadIdx.x == 0) {
    const int64_t i = (int64_t)b * nbx + bx;
    pa[2 * i] = l;
    pa[2 * i + 1] = sg;
    pb[i] = t;
  }
}

// Fused 3D adjoint step (adj3d.h), tiles of 2 rows by tz planes; partials as
// in u_adj2d_kernel.
__global__ __launch_bounds__(kMaxBlock) void u_adj3d_kernel(
    PlaneSet P, AdjIds ids, const float* __restrict__ coeffs, int k,
    float theta, int tz, int wpb, int ntx, int nty, int ntiles,
    double* __restrict__ pa, double* __restrict__ pb) {
  constexpr int TH = 2;
  __shared__ double red[2][kMaxBlock / kWave];
  const int b = blockIdx.y;
  // (not wave_in_block(): measured 2-3 % slower in the 3D kernels)
  const int wave = threadIdx.x / kWave;
  const int nbx = gridDim.x, bx = blockIdx.x;
  const int q8 = nbx >> 3, r8 = nbx & 7, xcd = bx & 7;
  const int bt = xcd * q8 + min(xcd, r8) + (bx >> 3);
  const int wt = bt * wpb + wave;
  double l = 0.0, sg = 0.0, t = 0.0;
  if (wt < ntiles) {
    const int per_seg = ntx * nty;
    const int tzi = wt / per_seg;
    const int rem = wt - tzi * per_seg;
    const int ty = rem / ntx, tx = rem - ty * ntx;
    AdjCtx3D c;
    c.fk = cplane(P, b, ids.fk);
    c.fkm = cplane(P, b, ids.fkm);
    c.pk = cplane(P, b, ids.pk);
    c.g = cplane(P, b, ids.g);
    c.a = cplane(P, b, ids.a_in);
    c.b = cplane(P, b, ids.b_in);
    c.r = cplane(P, b, ids.r_in);
    c.ao = plane(P, b, ids.a_out);
    c.bo = plane(P, b, ids.b_out);
    c.t = plane(P, b, ids.t_out);
    c.gbar = plane(P, b, ids.gbar);
    c.cs = P.plane;
    c.nz = P.nz;
    c.ny = P.ny;
    c.nx = P.nx;
    c.pitch = P.pitch;
    c.x0 = tx * kStripCols;
    c.y0 = ty * TH;
    c.z0 = tzi * tz;
    c.z1 = min(c.z0 + tz, P.nz);
    c.lam = coeffs[3 * k];
    c.tau = coeffs[3 * k + 1];
    c.sig = coeffs[3 * k + 2];
    c.th = theta;
    adj_tile3d<TH>(c, l, sg, t);
  }
  block_sum2(l, sg, red);
  __syncthreads();
  double unused = 0.0;
  block_sum2(t, unused, red);
  if (threadIdx.x == 0) {
    const int64_t i = (int64_t)b * nbx + bx;
    pa[2 * i] = l;
    pa[2 * i + 1] = sg;
    pb[i] = t;
  }
}

// grad_coeffs[k] = (lambar, taubar, sigmabar) from the block partials of the
// two adjoint passes, summed in a fixed order.
__global__ __launch_bounds__(kMaxBlock) void u_coeff_reduce_kernel(
    const double* __restrict__ pa, const double* __restrict__ pb, int nblk,
    float* __restrict__ grad_coeffs, int k) {
  __shared__ double red[2][kMaxBlock / kWave];
  double l = 0.0, s = 0.0, t = 0.0, unused = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
    l += pa[2 * i];
    s += pa[2 * i + 1];
    t += pb[i];
  }
  block_sum2(l, s, red);
  __syncthreads();
  block_sum2(t, unused, red);
  if (threadIdx.x == 0) {
    grad_coeffs[3 * k] = (float)l;
    grad_coeffs[3 * k + 1] = (float)t;
    grad_coeffs[3 * k + 2] = (float)s;
  }
}

// ------------------------------ plumbing ----------------------------------

__global__ void u_init_kernel(PlaneSet P, const float* __restrict__ g,
                              int id_g, int id_zero, int nzero) {
  const Pix q = pixel_of(P);
  if (!q.ok) return;
  const int64_t dense = (((int64_t)q.b * P.nz + q.z) * P.ny + q.y) * P.nx + q.x;
  plane(P, q.b, id_g)[q.o] = g[dense];
  for (int i = 0; i < nzero; ++i) plane(P, q.b, id_zero + i)[q.o] = 0.0f;
}

__global__ void u_zero_pitch_kernel(PlaneSet P, int id, int n) {
  // zero whole planes, padding included
  const int64_t total = (int64_t)P.nb * n * P.plane;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / ((int64_t)n * P.plane);
    const int64_t rem = e - b * n * P.plane;
    P.base[b * P.istride + (int64_t)id * P.plane + rem] = 0.0f;
  }
}

__global__ void u_read_kernel(PlaneSet P, int id, float* __restrict__ out) {
  const Pix q = pixel_of(P);
  if (!q.ok) return;
  const int64_t dense = (((int64_t)q.b * P.nz + q.z) * P.ny + q.y) * P.nx + q.x;
  out[dense] = cplane(P, q.b, id)[q.o];
}

__global__ void u_load_kernel(PlaneSet P, const float* __restrict__ in,
                              int id) {
  const Pix q = pixel_of(P);
  if (!q.ok) return;
  const int64_t dense = (((int64_t)q.b * P.nz + q.z) * P.ny + q.y) * P.nx + q.x;
  plane(P, q.b, id)[q.o] = in[dense];
}

__global__ void u_final_grad_kernel(PlaneSet P, int gbar, int a, int b,
                                    float* __restrict__ out) {
  const Pix q = pixel_of(P);
  if (!q.ok) return;
  const int64_t dense = (((int64_t)q.b * P.nz + q.z) * P.ny + q.y) * P.nx + q.x;
  out[dense] = cplane(P, q.b, gbar)[q.o] +
               (cplane(P, q.b, a)[q.o] + cplane(P, q.b, b)[q.o]);
}

int64_t nrow_blocks(const PlaneSet& P) {
  return (int64_t)((P.nx + kRowBlock - 1) / kRowBlock) * P.nb * P.nz * P.ny;
}

// Blocks of the adjoint passes: grid-stride over row blocks, so that the
// per-step coefficient reduction sums a few thousand partials at most.
constexpr int64_t kAdjBlocks = 4096;
int64_t adj_blocks(const PlaneSet& P) {
  const int64_t n = nrow_blocks(P);
  return n < kAdjBlocks ? n : kAdjBlocks;
}

}  // namespace

int64_t u_partials_needed(const PlaneSet& P) { return 3 * adj_blocks(P) + 1; }

hipError_t launch_u_init(const PlaneSet& P, const float* g, int id_g,
                         int id_zero, int nzero, hipStream_t s) {
  // Only g and p^0 are read before a kernel has written them: zero those
  // planes (padding included; g's padding stays zero), then copy g in.
  // Every other plane is written whole (all rows, all pitch columns) by the
  // sweep that produces it before anything reads it.
  const int first = id_g < id_zero ? id_g : id_zero;
  const int last = id_g > id_zero + nzero - 1 ? id_g : id_zero + nzero - 1;
  hipLaunchKernelGGL(u_zero_pitch_kernel, dim3(4096), dim3(256), 0, s, P,
                     first, last - first + 1);
  hipLaunchKernelGGL(u_init_kernel, dim3((unsigned)nrow_blocks(P)),
                     dim3(kRowBlock), 0, s, P, g, id_g, id_zero, nzero);
  return hipGetLastError();
}

hipError_t launch_u_zero(const PlaneSet& P, int id, int n, hipStream_t s) {
  hipLaunchKernelGGL(u_zero_pitch_kernel, dim3(4096), dim3(256), 0, s, P, id,
                     n);
  return hipGetLastError();
}

hipError_t launch_u_pass2d(const PlaneSet& P, const PassIds& ids,
                           const float* coeffs, int k, int n, float theta,
                           hipStream_t s) {
  if (P.ndim != 2 || n < 1 || n > kMaxPass - 1) return hipErrorInvalidValue;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
          hipSuccess || cus < 1)
    cus = 256;
  // the plain solver's rule for deep passes: the shortest bands whose
  // blocks (4 waves) all fit on the GPU at once, two per CU
  const int strip = xs_owned(n);
  const int64_t ntx = (P.nx + strip - 1) / strip;
  const int wpb = 4;
  int64_t th = 8;
  while (th < 256 &&
         (ntx * ((P.ny + th - 1) / th) + wpb - 1) / wpb * P.nb > 2LL * cus)
    ++th;
  const int nty = (int)((P.ny + th - 1) / th);
  const int nbx = (int)((ntx * nty + wpb - 1) / wpb);
  const dim3 grid(nbx, P.nb), block(wpb * kWave);
  switch (n) {
    case 1: hipLaunchKernelGGL(u_sweep2d_xs_kernel<1>, grid, block, 0, s, P, ids, coeffs, k, theta, (int)th, wpb, (int)ntx, nty); break;
    case 2: hipLaunchKernelGGL(u_sweep2d_xs_kernel<2>, grid, block, 0, s, P, ids, coeffs, k, theta, (int)th, wpb, (int)ntx, nty); break;
    case 3: hipLaunchKernelGGL(u_sweep2d_xs_kernel<3>, grid, block, 0, s, P, ids, coeffs, k, theta, (int)th, wpb, (int)ntx, nty); break;
    case 4: hipLaunchKernelGGL(u_sweep2d_xs_kernel<4>, grid, block, 0, s, P, ids, coeffs, k, theta, (int)th, wpb, (int)ntx, nty); break;
    default: hipLaunchKernelGGL(u_sweep2d_xs_kernel<5>, grid, block, 0, s, P, ids, coeffs, k, theta, (int)th, wpb, (int)ntx, nty); break;
  }
  return hipGetLastError();
}

hipError_t launch_u_step(const PlaneSet& P, const StepIds& ids,
                         const float* coeffs, int k, float theta,
                         hipStream_t s) {
  if (P.ndim != 3) return hipErrorInvalidValue;   // 2D: launch_u_pass2d
  // the plain solver's tile for this volume shape
  Layout L;
  L.ndim = 3;
  L.nz = P.nz;
  L.ny = P.ny;
  L.nx = P.nx;
  const Tile3D t = tile3d_for(L);
  if (!tile3d_ok(t)) return hipErrorInvalidValue;
  const int ntx = (P.nx + kStripCols - 1) / kStripCols;
  const int nty = (P.ny + t.th - 1) / t.th;
  const int ntz = (P.nz + t.tz - 1) / t.tz;
  const int64_t nt = (int64_t)ntx * nty * ntz;
  if (nt > INT32_MAX / 2) return hipErrorInvalidValue;
  const int nbx = (int)((nt + t.wpb - 1) / t.wpb);
  const dim3 grid(nbx, P.nb), block(t.wpb * kWave);
  if (t.th == 2)
    hipLaunchKernelGGL(u_sweep3d_kernel<2>, grid, block, 0, s, P, ids,
                       coeffs, k, theta, t.tz, t.wpb, ntx, nty, (int)nt);
  else
    hipLaunchKernelGGL(u_sweep3d_kernel<4>, grid, block, 0, s, P, ids,
                       coeffs, k, theta, t.tz, t.wpb, ntx, nty, (int)nt);
  return hipGetLastError();
}

hipError_t launch_u_read(const PlaneSet& P, int id, float* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(u_read_kernel, dim3((unsigned)nrow_blocks(P)),
                     dim3(kRowBlock), 0, s, P, id, out);
  return hipGetLastError();
}

hipError_t launch_u_load(const PlaneSet& P, const float* in, int id,
                         hipStream_t s) {
  hipLaunchKernelGGL(u_load_kernel, dim3((unsigned)nrow_blocks(P)),
                     dim3(kRowBlock), 0, s, P, in, id);
  return hipGetLastError();
}

hipError_t launch_u_adjoint(const PlaneSet& P, const AdjIds& ids,
                            const float* coeffs, int k, float theta,
                            double* partials, int64_t max_partials,
                            float* grad_coeffs, hipStream_t s) {
  const int64_t nblk = adj_blocks(P);
  if (3 * nblk > max_partials) return hipErrorInvalidValue;
  double* pa = partials;
  double* pb = partials + 2 * nblk;
  const dim3 grid((unsigned)nblk);
  if (P.ndim == 2 && fused_adjoint_enabled()) {
    // bands for about one block of four waves per CU, and at most nblk
    // blocks in all
    const int wpb = 4;
    const int64_t ntx = (P.nx + kStripCols - 1) / kStripCols;
    const int64_t cols = ntx * P.ny * P.nb;
    int64_t th = (cols + 1023) / 1024;
    const int64_t th_min = (cols + nblk * wpb - 1) / (nblk * wpb);
    if (th < th_min) th = th_min;
    if (th < 8) th = 8;
    const int nty = (int)((P.ny + th - 1) / th);
    const int nbx = (int)((ntx * nty + wpb - 1) / wpb);
    const int64_t nb_total = (int64_t)nbx * P.nb;
    if (nb_total > nblk) return hipErrorInvalidValue;
    hipLaunchKernelGGL(u_adj2d_kernel, dim3(nbx, P.nb), dim3(wpb * kWave), 0,
                       s, P, ids, coeffs, k, theta, (int)th, wpb, (int)ntx,
                       nty, pa, pb);
    hipLaunchKernelGGL(u_coeff_reduce_kernel, dim3(1), dim3(kMaxBlock), 0, s,
                       pa, pb, (int)nb_total, grad_coeffs, k);
    return hipGetLastError();
  }
  if (P.ndim == 3 && fused_adjoint_enabled()) {
    // bands of 2 rows; segments deep enough for about 4 waves per CU (at
    // most nblk blocks in all)
    const int wpb = 4, th = 2;
    const int64_t ntx = (P.nx + kStripCols - 1) / kStripCols;
    const int64_t nty = (P.ny + th - 1) / th;
    const int64_t cols = ntx * nty * P.nb;
    int64_t tz = (cols * P.nz + 1023) / 1024;
    const int64_t tz_min = (cols * P.nz + nblk * wpb - 1) / (nblk * wpb);
    if (tz < tz_min) tz = tz_min;
    if (tz < 4) tz = 4;
    if (tz > P.nz) tz = P.nz;
    const int64_t ntz = (P.nz + tz - 1) / tz;
    const int64_t nt = ntx * nty * ntz;
    const int nbx = (int)((nt + wpb - 1) / wpb);
    const int64_t nb_total = (int64_t)nbx * P.nb;
    if (nb_total > nblk || nt > INT32_MAX / 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(u_adj3d_kernel, dim3(nbx, P.nb), dim3(wpb * kWave), 0,
                       s, P, ids, coeffs, k, theta, (int)tz, wpb, (int)ntx,
                       (int)nty, (int)nt, pa, pb);
    hipLaunchKernelGGL(u_coeff_reduce_kernel, dim3(1), dim3(kMaxBlock), 0, s,
                       pa, pb, (int)nb_total, grad_coeffs, k);
    return hipGetLastError();
  }
  if (P.ndim == 2) {
    hipLaunchKernelGGL(u_adjA_kernel<2>, grid, dim3(kRowBlock), 0, s, P, ids,
                       coeffs, k, theta, pa);
    hipLaunchKernelGGL(u_adjB_kernel<2>, grid, dim3(kRowBlock), 0, s, P, ids,
                       coeffs, k, theta, pb);
  } else {
    hipLaunchKernelGGL(u_adjA_kernel<3>, grid, dim3(kRowBlock), 0, s, P, ids,
                       coeffs, k, theta, pa);
    hipLaunchKernelGGL(u_adjB_kernel<3>, grid, dim3(kRowBlock), 0, s, P, ids,
                       coeffs, k, theta, pb);
  }
  hipLaunchKernelGGL(u_coeff_reduce_kernel, dim3(1), dim3(kMaxBlock), 0, s, pa,
                     pb, (int)nblk, grad_coeffs, k);
  return hipGetLastError();
}

hipError_t launch_u_final_grad(const PlaneSet& P, int gbar, int a, int b,
                               float* grad_g, hipStream_t s) {
  hipLaunchKernelGGL(u_final_grad_kernel, dim3((unsigned)nrow_blocks(P)),
                     dim3(kRowBlock), 0, s, P, gbar, a, b, grad_g);
  return hipGetLastError();
}

}  // namespace tvpd
