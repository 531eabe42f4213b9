// Backprojection by the backprojection slice theorem (BST): the paper's fast
// backprojection (Section 3, eq. bst; algorithm of Section 5), on the
// geometry of the tomographic operators (tomo.h).
//
// In the cycles convention the theorem reads F[B g](nu xi_theta) =
// G(nu, theta) / |nu| (B the continuous backprojection; B = dtheta A^T for
// sampled data).  Steps:
//   1. per projection, the DFT of the zero-padded projection, length M (a
//      power of two >= 2 n_det), with the phase of the detector's centring;
//   2. times K(nu) = 1/|nu|, and 1/dnu = M at nu = 0 (the origin rule);
//   3. bilinear interpolation of the polar samples (theta_k, nu_j) at the
//      frequencies (p, q)/Q of a Q x Q grid (Q a power of two >= 2 max(ny,
//      nx)), zero beyond |nu| = 1/2, times the phase that puts the pixel
//      centres on the integer grid;
//   4. 2D inverse DFT, real part at the pixels, divided by Q^2: transforms
//      of the grid rows fused with step 3 (of which only the nx pixel
//      columns are kept), a transpose of those columns, and their
//      transforms (of which only the ny pixel rows are read).
// The regularised filtered backprojection f_lam = B F_lam g (Section 6, eq.
// reg_sol) runs the same steps with K(nu) = 1/(1 + lam |nu|) in step 2: the
// ramp |nu| of the filter F_lam cancels the 1/|nu| of the theorem (eq.
// reg_fst), which leaves a kernel with no singularity at the origin.
// The transforms are radix-16 Stockham FFTs in LDS (lengths up to 4096; a
// radix-2 and/or radix-4 stage for the remaining factor; a padded LDS layout
// against bank conflicts), with twiddles from a float64 table.  Every phase is reduced as an exact integer
// before its sine and cosine.
#include <cfloat>
#include <cmath>

#include "tomo.h"

namespace tvpd {

constexpr int kBstMaxLen = 4096;   // LDS FFT length limit
// phases reduced in 32-bit integers: two products of a signed frequency
// index (at most kBstMaxLen / 2) and a side (at most kTomoMaxSide)
static_assert(2LL * (kBstMaxLen / 2) * kTomoMaxSide < (1LL << 31), "bst phase range");
// LDS index of element i of a transform: one spare slot per 16 elements, so
// that the strided writes of the Stockham stages spread over the banks.
constexpr int kBstLds = kBstMaxLen + kBstMaxLen / 16;
__device__ __forceinline__ int lds_at(int i) { return i + (i >> 4); }

__host__ __device__ inline int bst_pow2_at_least(int v) {
  int L = 1;
  while (L < v) L *= 2;
  return L;
}

struct BstLayout {
  int ny, nx, na, nd, M, Q;
  size_t off_tw, off_spec, off_a, off_b, bytes;
};

BstLayout bst_layout(int ny, int nx, int na, int nd) {
  BstLayout L;
  L.ny = ny;
  L.nx = nx;
  L.na = na;
  L.nd = nd;
  L.M = bst_pow2_at_least(2 * nd);
  L.Q = bst_pow2_at_least(2 * (ny > nx ? ny : nx));
  const int tl = L.M > L.Q ? L.M : L.Q;
  L.off_tw = kHeaderBytes;
  L.off_spec = (size_t)round_up((int64_t)L.off_tw + 8 * (int64_t)tl, (int64_t)kAlign);
  L.off_a = (size_t)round_up((int64_t)L.off_spec + 8 * (int64_t)na * L.M, (int64_t)kAlign);
  L.off_b = (size_t)round_up((int64_t)L.off_a + 8 * (int64_t)L.Q * L.Q, (int64_t)kAlign);
  L.bytes = L.off_b + 8 * (size_t)L.Q * (size_t)L.Q;
  return L;
}

namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// tw[m] = exp(-2 pi i m / L), m < L, from float64.
__global__ void bst_twiddle_kernel(float2* tw, int L) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= L) return;
  const double a = -2.0 * (double)m / (double)L;
  tw[m] = make_float2((float)cospi(a), (float)sinpi(a));
}

// Stockham transform of length n (a power of two, <= 4096) in one LDS buffer
// (Govindaraju et al. 2008): radix-16 stages, each thread holding one
// 16-point butterfly in registers (a 4 x 4 decomposition with constant inner
// twiddles), after one radix-2 and/or one radix-4 stage for the remaining
// factor of n; each stage reads its inputs into registers, waits for the
// block, then writes its outputs.  SIGN -1: forward (exp(-2 pi i ...)), +1:
// inverse without the 1/n.  tw: the full table of length tl (a multiple of
// n).  Every thread of the block takes part.
constexpr int kFftPerThread = kBstMaxLen / 4 / kMaxBlock;   // radix-4 butterflies

__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}
// SIGN i a
template <int SIGN>
__device__ __forceinline__ float2 cmul_i(float2 a) {
  return SIGN > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// 4-point DFT with root SIGN i, in place.
template <int SIGN>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const float2 t2 = cadd(a1, a3), t3 = cmul_i<SIGN>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a1 = cadd(t1, t3);
  a2 = csub(t0, t2);
  a3 = csub(t1, t3);
}

// 16-point DFT with root exp(SIGN 2 pi i / 16), in place and in natural
// order: inputs n = 4 n1 + n2, outputs k = k1 + 4 k2.
template <int SIGN>
__device__ __forceinline__ void dft16(float2 v[16]) {
  // cos and sin of m pi / 8
  constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508977f;
  constexpr float h = 0.70710678118654752f;
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<SIGN>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  // v[4 k1 + n2] now holds the k1 output of column n2; times W^(n2 k1)
  auto w16 = [](int m) {
    float c, sn;
    switch (m) {
      case 1: c = c1; sn = s1; break;
      case 2: c = h; sn = h; break;
      case 3: c = s1; sn = c1; break;
      case 4: c = 0.0f; sn = 1.0f; break;
      case 6: c = -h; sn = h; break;
      default: c = -c1; sn = -s1; break;   // m = 9
    }
    return make_float2(c, SIGN > 0 ? sn : -sn);
  };
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) v[4 * k1 + n2] = cmul(v[4 * k1 + n2], w16(n2 * k1));
  float2 y[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a0 = v[4 * k1], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
    dft4<SIGN>(a0, a1, a2, a3);
    y[k1] = a0;
    y[k1 + 4] = a1;
    y[k1 + 8] = a2;
    y[k1 + 12] = a3;
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = y[r];
}

template <int SIGN>
__device__ __forceinline__ float2 twiddle(const float2* tw, int m) {
  float2 w = tw[m];
  if (SIGN > 0) w.y = -w.y;
  return w;
}

template <int SIGN>
__device__ void fft_lds(float2* x, int n, const float2* tw, int tl) {
  int Ns = 1;
  const int lg = __builtin_ctz(n);
  if (lg & 1) {                                    // radix-2 stage
    float2 v[2 * kFftPerThread][2];
#pragma unroll
    for (int u = 0; u < 2 * kFftPerThread; ++u) {
      const int j = threadIdx.x + u * kMaxBlock;
      if (j < n / 2) {
        v[u][0] = x[lds_at(j)];
        v[u][1] = x[lds_at(j + n / 2)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2 * kFftPerThread; ++u) {
      const int j = threadIdx.x + u * kMaxBlock;
      if (j < n / 2) {
        x[lds_at(2 * j)] = cadd(v[u][0], v[u][1]);
        x[lds_at(2 * j + 1)] = csub(v[u][0], v[u][1]);
      }
    }
    __syncthreads();
    Ns = 2;
  }
  if (lg & 2) {                                    // radix-4 stage
    const int stride = tl / (4 * Ns);
    float2 v[kFftPerThread][4];
#pragma unroll
    for (int u = 0; u < kFftPerThread; ++u) {
      const int j = threadIdx.x + u * kMaxBlock;
      if (j < n / 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[u][r] = x[lds_at(j + r * (n / 4))];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kFftPerThread; ++u) {
      const int j = threadIdx.x + u * kMaxBlock;
      if (j < n / 4) {
        const int k = j & (Ns - 1);
#pragma unroll
        for (int r = 1; r < 4; ++r) v[u][r] = cmul(v[u][r], twiddle<SIGN>(tw, r * k * stride));
        dft4<SIGN>(v[u][0], v[u][1], v[u][2], v[u][3]);
        const int d = ((j - k) << 2) + k;
#pragma unroll
        for (int r = 0; r < 4; ++r) x[lds_at(d + r * Ns)] = v[u][r];
      }
    }
    __syncthreads();
    Ns *= 4;
  }
  for (; Ns < n; Ns <<= 4) {                       // radix-16 stages
    const int stride = tl / (16 * Ns);
    const int j = threadIdx.x;                     // n / 16 <= blockDim.x
    float2 v[16];
    if (j < n / 16) {
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = x[lds_at(j + r * (n / 16))];
    }
    __syncthreads();
    if (j < n / 16) {
      const int k = j & (Ns - 1);
#pragma unroll
      for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twiddle<SIGN>(tw, r * k * stride));
      dft16<SIGN>(v);
      const int d = ((j - k) << 4) + k;
#pragma unroll
      for (int r = 0; r < 16; ++r) x[lds_at(d + r * Ns)] = v[r];
    }
    __syncthreads();
  }
}

// Steps 1-2 for projection k: spec[k][m + M/2] = K(nu) exp(-2 pi i nu t_0) DFT(g_k)
// at nu = m / M, m = -M/2 .. M/2-1.  lam < 0: the backprojection kernel
// K = 1/|nu| (M at nu = 0); lam >= 0: K = 1/(1 + lam |nu|), the ramp of the
// regularised filter cancelled against 1/|nu| (Section 6, eq. reg_fst).
__global__ __launch_bounds__(kMaxBlock) void bst_spectra_kernel(const float* g, float2* spec,
                                                                const float2* tw, int nd,
                                                                int M, int tl, float lam) {
  __shared__ float2 x[kBstLds];
  const int k = blockIdx.x;
  const float* gr = g + (int64_t)k * nd;
  constexpr int kPer = kBstMaxLen / kMaxBlock;
  float v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = threadIdx.x + u * kMaxBlock;
    v[u] = i < nd ? gr[i] : 0.0f;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = threadIdx.x + u * kMaxBlock;
    if (i < M) x[lds_at(i)] = make_float2(v[u], 0.0f);
  }
  __syncthreads();
  fft_lds<-1>(x, M, tw, tl);
  float2* out = spec + (int64_t)k * M;
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    const int ms = m < M / 2 ? m : m - M;          // signed frequency index
    // t_0 = (1 - nd) / 2: phase -2 pi ms t_0 / M = pi ms (nd - 1) / M,
    // reduced modulo 2M exactly (a mask: 2M is a power of two, and
    // |ms (nd - 1)| <= 2048 x 32767 fits in 32 bits)
    const int ph = (ms * (nd - 1)) & (2 * M - 1);
    float sn, cs;
    sincospif((float)ph * (1.0f / (float)M), &sn, &cs);   // (exact: M a power of two)
    const int am = ms < 0 ? -ms : ms;
    const float kk = lam < 0.0f ? (am == 0 ? (float)M : (float)M / (float)am)
                                : 1.0f / fmaf(lam, (float)am / (float)M, 1.0f);
    const float2 v = cmul(x[lds_at(m)], make_float2(cs, sn));
    out[ms + M / 2] = make_float2(v.x * kk, v.y * kk);
  }
}

// Step 3 at the grid frequency (ps, qs)/Q (signed indices) with polar
// angle phi = atan2(qs, ps) in (-pi, pi] and radius rho: phase * bilinear(spec).
// per_dphi = na / pi (angle steps per radian), inv_q = 1 / Q (exact: Q is a
// power of two).
__device__ float2 cartesian_value(const float2* spec, int na, int M, int Q, int nx, int ny,
                                  int ps, int qs, double phi, double rho, double per_dphi,
                                  float inv_q) {
  if (rho > 0.5) return make_float2(0.0f, 0.0f);
  double nu = rho;
  if (phi < 0.0) {
    phi += M_PI;
    nu = -rho;
  }
  if (phi >= M_PI) {
    phi -= M_PI;
    nu = -nu;
  }
  const double aidx = phi * per_dphi;
  int k0 = (int)floor(aidx);
  if (k0 > na - 1) k0 = na - 1;                   // rounding at phi -> pi
  if (k0 < 0) k0 = 0;
  const float wa = (float)(aidx - k0);
  int k1 = k0 + 1;
  double nu1 = nu;
  if (k1 >= na) {                                 // theta = pi: angle 0, -nu
    k1 = 0;
    nu1 = -nu;
  }
  auto radial = [&](int k, double nv) {
    const double xr = nv * M + M / 2;
    const int j0 = (int)floor(xr);
    const float wr = (float)(xr - j0);
    const float2* row = spec + (int64_t)k * M;
    const float2 p0 = (j0 >= 0 && j0 < M) ? row[j0] : make_float2(0.0f, 0.0f);
    const float2 p1 = (j0 + 1 >= 0 && j0 + 1 < M) ? row[j0 + 1] : make_float2(0.0f, 0.0f);
    return make_float2(p0.x + wr * (p1.x - p0.x), p0.y + wr * (p1.y - p0.y));
  };
  const float2 r0 = radial(k0, nu), r1 = radial(k1, nu1);
  const float2 val = make_float2(r0.x + wa * (r1.x - r0.x), r0.y + wa * (r1.y - r0.y));
  // pixel centres at n + (1 - n_side)/2: phase 2 pi (ps (1 - nx) + qs (1 - ny)) / (2Q),
  // reduced modulo 2Q exactly (a mask: 2Q is a power of two, and the sum is
  // at most 2 x 2048 x 32767 in magnitude, within 32 bits)
  const int ph = (ps * (1 - nx) + qs * (1 - ny)) & (2 * Q - 1);
  float sn, cs;
  sincospif((float)ph * inv_q, &sn, &cs);
  return cmul(val, make_float2(cs, sn));
}

// Step 3 for grid row q and its inverse transform along p, in LDS; the
// first nx outputs (the pixel columns) go to A[q][0 .. nx).  The points
// (ps, qs) and (-ps, qs) share rho and one float64 arctangent:
// atan2(qs, -ps) = +-pi - atan2(qs, ps) (the sign of qs, +pi for qs = 0).
__global__ __launch_bounds__(kMaxBlock) void bst_cartesian_rows_kernel(
    const float2* spec, float2* A, const float2* tw, int na, int M, int Q, int nx, int ny,
    int tl) {
  __shared__ float2 x[kBstLds];
  const int q = blockIdx.x;
  const int qs = q < Q / 2 ? q : q - Q;
  const double inv_q = 1.0 / Q;                  // exact: Q is a power of two
  const double per_dphi = na / M_PI;
  const double v = (double)qs * inv_q;
  for (int a = threadIdx.x; a <= Q / 2; a += blockDim.x) {
    const double u = (double)a * inv_q;
    const double rho = sqrt(u * u + v * v);
    const double phi = atan2(v, u);                        // point (a, qs)
    if (a < Q / 2)
      x[lds_at(a)] = cartesian_value(spec, na, M, Q, nx, ny, a, qs, phi, rho, per_dphi,
                                     (float)inv_q);
    if (a > 0) {                                           // point (-a, qs)
      const double phm = (qs >= 0 ? M_PI : -M_PI) - phi;
      x[lds_at(Q - a)] = cartesian_value(spec, na, M, Q, nx, ny, -a, qs, phm, rho, per_dphi,
                                         (float)inv_q);
    }
  }
  __syncthreads();
  fft_lds<+1>(x, Q, tw, tl);
  float2* out = A + (int64_t)q * nx;
  for (int i = threadIdx.x; i < nx; i += blockDim.x) out[i] = x[lds_at(i)];
}

// Inverse transforms of n rows of length Q, in place.
__global__ __launch_bounds__(kMaxBlock) void bst_rows_inverse_kernel(float2* A, const float2* tw,
                                                                     int Q, int tl) {
  __shared__ float2 x[kBstLds];
  float2* row = A + (int64_t)blockIdx.x * Q;
  // every load of the row issued before the first use (a fixed count per
  // thread, so the loop unrolls)
  constexpr int kPer = kBstMaxLen / kMaxBlock;
  float2 v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = threadIdx.x + u * kMaxBlock;
    if (i < Q) v[u] = row[i];
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = threadIdx.x + u * kMaxBlock;
    if (i < Q) x[lds_at(i)] = v[u];
  }
  __syncthreads();
  fft_lds<+1>(x, Q, tw, tl);
  for (int i = threadIdx.x; i < Q; i += blockDim.x) row[i] = x[lds_at(i)];
}

// B[c][r] = A[r][c] for A of Q rows and nx columns (B: nx rows of Q), 32 x 32
// tiles (Q is a multiple of 32).
__global__ void bst_transpose_kernel(const float2* A, float2* B, int Q, int nx) {
  __shared__ float2 t[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int c = c0 + threadIdx.x;
  for (int r = threadIdx.y; r < 32; r += 8)
    t[r][threadIdx.x] = c < nx ? A[(int64_t)(r0 + r) * nx + c] : make_float2(0.0f, 0.0f);
  __syncthreads();
  for (int cc = threadIdx.y; cc < 32; cc += 8)
    if (c0 + cc < nx) B[(int64_t)(c0 + cc) * Q + r0 + threadIdx.x] = t[threadIdx.x][cc];
}

// img[a][b] = Re(B[b][a]) / Q^2 (B holds the image transposed).
__global__ void bst_extract_kernel(const float2* B, float* img, int Q, int ny, int nx,
                                   float scale) {
  __shared__ float t[32][33];
  const int a0 = blockIdx.y * 32, b0 = blockIdx.x * 32;   // image rows a, columns b
  for (int bb = threadIdx.y; bb < 32; bb += 8) {
    const int b = b0 + bb, a = a0 + threadIdx.x;
    t[bb][threadIdx.x] = (b < nx && a < ny) ? B[(int64_t)b * Q + a].x : 0.0f;
  }
  __syncthreads();
  for (int aa = threadIdx.y; aa < 32; aa += 8) {
    const int a = a0 + aa, b = b0 + threadIdx.x;
    if (a < ny && b < nx) img[(int64_t)a * nx + b] = t[threadIdx.x][aa] * scale;
  }
}

#define BST_TRY(call)                   \
  do {                                  \
    const int st_ = (call);             \
    if (st_ != TVPD_OK) return st_;     \
  } while (0)

// Regularised FBP filtering through the FFT (Section 6: the filter
// |sigma| / (1 + lam |sigma|) of the regularised FBP): rays 2k and 2k + 1 as
// the real and imaginary parts of one sequence, zero padded to L >= 2 nd (so
// that the circular convolution is the linear one over the nd outputs),
// transformed, multiplied by H_m = |nu_m| / (1 + lam |nu_m|) with nu_m the
// signed frequency m/L (real and even, so the two rays stay apart),
// transformed back; the outputs are scaled by scale / L.
__global__ __launch_bounds__(kMaxBlock) void fbp_fft_filter_kernel(const float* g, float* q,
                                                                   const float2* tw, int na,
                                                                   int nd, int L, float lam,
                                                                   float scale) {
  __shared__ float2 x[kBstLds];
  const int ka = 2 * blockIdx.x, kb = ka + 1;
  const bool hb = kb < na;
  const float* ga = g + (int64_t)ka * nd;
  const float* gb = g + (int64_t)(hb ? kb : ka) * nd;
  constexpr int kPer = kBstMaxLen / kMaxBlock;
  float va[kPer], vb[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = threadIdx.x + u * kMaxBlock;
    va[u] = i < nd ? ga[i] : 0.0f;
    vb[u] = (hb && i < nd) ? gb[i] : 0.0f;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = threadIdx.x + u * kMaxBlock;
    if (i < L) x[lds_at(i)] = make_float2(va[u], vb[u]);
  }
  __syncthreads();
  fft_lds<-1>(x, L, tw, L);
  const float inv_l = 1.0f / (float)L;          // exact: L is a power of two
  for (int m = threadIdx.x; m < L; m += blockDim.x) {
    const int am = m <= L / 2 ? m : L - m;      // |signed index|; m = L/2 gives 1/2
    const float nu = (float)am * inv_l;
    const float h = nu / fmaf(lam, nu, 1.0f);
    const float2 v = x[lds_at(m)];
    x[lds_at(m)] = make_float2(v.x * h, v.y * h);
  }
  __syncthreads();
  fft_lds<+1>(x, L, tw, L);
  const float sc = scale * inv_l;
  float* qa = q + (int64_t)ka * nd;
  float* qb = q + (int64_t)kb * nd;
  for (int i = threadIdx.x; i < nd; i += blockDim.x) {
    const float2 v = x[lds_at(i)];
    qa[i] = v.x * sc;
    if (hb) qb[i] = v.y * sc;
  }
}

int launched() { return hipGetLastError() == hipSuccess ? TVPD_OK : TVPD_ERR_HIP; }

bool geom_ok(const tvpd_tomo_geom* g) {
  if (!g) return false;
  return g->ny >= 1 && g->nx >= 1 && g->n_angles >= 1 && g->n_det >= 1 &&
         g->ny <= kTomoMaxSide && g->nx <= kTomoMaxSide && g->n_det <= kTomoMaxSide &&
         g->n_angles <= kTomoMaxAngles;
}

int supported(const BstLayout& L) {
  return (L.M <= kBstMaxLen && L.Q <= kBstMaxLen && L.Q >= 32) ? TVPD_OK
                                                                : TVPD_ERR_UNSUPPORTED;
}

int ws_check(const BstLayout& L, const void* ws, size_t bytes) {
  if (!ws) return TVPD_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return TVPD_ERR_ALIGNMENT;
  if (bytes < L.bytes) return TVPD_ERR_WORKSPACE;
  return TVPD_OK;
}

// Steps 1-2 into the workspace's spectra (lam as in bst_spectra_kernel).
int spectra(const BstLayout& L, const float* g, char* base, float lam, hipStream_t s) {
  const int tl = L.M > L.Q ? L.M : L.Q;
  float2* tw = reinterpret_cast<float2*>(base + L.off_tw);
  bst_twiddle_kernel<<<(tl + 255) / 256, 256, 0, s>>>(tw, tl);
  BST_TRY(launched());
  bst_spectra_kernel<<<L.na, kMaxBlock, 0, s>>>(
      g, reinterpret_cast<float2*>(base + L.off_spec), tw, L.nd, L.M, tl, lam);
  return launched();
}

// Steps 3-4: the spectra in the workspace to the image.
int grid_inverse(const BstLayout& L, char* base, float* img, hipStream_t s) {
  const int tl = L.M > L.Q ? L.M : L.Q;
  const float2* tw = reinterpret_cast<const float2*>(base + L.off_tw);
  float2* A = reinterpret_cast<float2*>(base + L.off_a);
  float2* B = reinterpret_cast<float2*>(base + L.off_b);
  // rows of the grid: step 3 and the transforms along x, keeping the nx
  // pixel columns (A: Q rows of nx)
  bst_cartesian_rows_kernel<<<L.Q, kMaxBlock, 0, s>>>(
      reinterpret_cast<const float2*>(base + L.off_spec), A, tw, L.na, L.M, L.Q, L.nx, L.ny,
      tl);
  BST_TRY(launched());
  // the pixel columns as rows (B: nx rows of Q), transformed along y
  bst_transpose_kernel<<<dim3((L.nx + 31) / 32, L.Q / 32), dim3(32, 8), 0, s>>>(A, B, L.Q,
                                                                                L.nx);
  BST_TRY(launched());
  bst_rows_inverse_kernel<<<L.nx, kMaxBlock, 0, s>>>(B, tw, L.Q, tl);
  BST_TRY(launched());
  bst_extract_kernel<<<dim3((L.nx + 31) / 32, (L.ny + 31) / 32), dim3(32, 8), 0, s>>>(
      B, img, L.Q, L.ny, L.nx, (float)(1.0 / ((double)L.Q * (double)L.Q)));
  return launched();
}

// The whole pipeline from g to img with the spectra's kernel chosen by lam.
int run_bst(const tvpd_tomo_geom* geom, const float* g, float* img, float lam, void* ws,
            size_t ws_bytes, void* stream) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!g || !img) return TVPD_ERR_INVALID_ARG;
  const BstLayout L = bst_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  BST_TRY(supported(L));
  BST_TRY(ws_check(L, ws, ws_bytes));
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  BST_TRY(spectra(L, g, base, lam, s));
  return grid_inverse(L, base, img, s);
}

}  // namespace

static_assert(kFbpFftMaxLen <= kBstMaxLen, "FBP FFT length");

int launch_fbp_fft_filter(const float* g, float* q, float2* tw, int na, int nd, float lam,
                          float scale, hipStream_t s) {
  const int L = tomo_fbp_length(nd);
  if (L > kFbpFftMaxLen) return TVPD_ERR_UNSUPPORTED;
  bst_twiddle_kernel<<<(L + 255) / 256, 256, 0, s>>>(tw, L);
  if (int rc = launched()) return rc;
  fbp_fft_filter_kernel<<<(na + 1) / 2, kMaxBlock, 0, s>>>(g, q, tw, na, nd, L, lam, scale);
  return launched();
}

}  // namespace tvpd

using namespace tvpd;

extern "C" {

int tvpd_bst_lengths(const tvpd_tomo_geom* geom, int32_t* M, int32_t* Q) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!M || !Q) return TVPD_ERR_INVALID_ARG;
  const BstLayout L = bst_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  *M = L.M;
  *Q = L.Q;
  return supported(L);
}

int tvpd_bst_workspace_size(const tvpd_tomo_geom* geom, size_t* bytes) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!bytes) return TVPD_ERR_INVALID_ARG;
  const BstLayout L = bst_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  BST_TRY(supported(L));
  *bytes = L.bytes;
  return TVPD_OK;
}

int tvpd_bst_spectra(const tvpd_tomo_geom* geom, const float* g, float* spec, void* ws,
                     size_t ws_bytes, void* stream) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!g || !spec) return TVPD_ERR_INVALID_ARG;
  const BstLayout L = bst_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  BST_TRY(supported(L));
  BST_TRY(ws_check(L, ws, ws_bytes));
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  BST_TRY(spectra(L, g, base, -1.0f, s));
  if (hipMemcpyAsync(spec, base + L.off_spec, 8 * (size_t)L.na * L.M, hipMemcpyDeviceToDevice,
                     s) != hipSuccess)
    return TVPD_ERR_HIP;
  return TVPD_OK;
}

int tvpd_bst_backproject(const tvpd_tomo_geom* geom, const float* g, float* img, void* ws,
                         size_t ws_bytes, void* stream) {
  return run_bst(geom, g, img, -1.0f, ws, ws_bytes, stream);
}

int tvpd_fbp_bst(const tvpd_tomo_geom* geom, const float* g, float lam, float* img, void* ws,
                 size_t ws_bytes, void* stream) {
  if (!(lam >= 0.0f) || !(lam <= FLT_MAX)) return TVPD_ERR_INVALID_ARG;
  return run_bst(geom, g, img, lam, ws, ws_bytes, stream);
}

}  // extern "C"
