// Log-polar backprojection: Andersson's formula (Section 2.1, eq.
// and_approach, and_kernel; the change of variables of eq. andersson) by the
// four-step algorithm of Section 5, on the geometry of the tomographic
// operators (tomo.h): pixel units, bins t_i = i + 1/2 - n_det/2, angles
// theta_k = k pi / n_angles, the paper's unit disc the detector's, R = n_det/2.
//
// In log-polar coordinates x = R e^rho xi_theta the backprojection is a 2D
// convolution of the semi-polar sinogram [g]_L(mu, phi) (2 n_angles rays over
// [0, 2 pi), ray phi carrying g(+-s, phi mod pi)) with K(a, b) =
// delta(1 - e^a cos b).  The mesh (table of symbols, eq. N_rho, adaptive rho_0):
// rho_0 = ln(1 / (2R)) (half a pixel), nodes rho_i = rho_0 + (i + 1) drho,
// i < N_rho, the top node at 0 or at ln(r_max / R) when the image's corners lie
// outside the detector's disc, radial steps of at most one bin inside the
// disc.  The kernel is the hat of height 1/drho at the root a = -ln cos b on
// the lag mesh a_l = l drho (two lags per angle, weights summing to one).
//
// GPU layout of the steps (rho is the long axis, N_rho up to 8192):
//   plan  (once per geometry and workspace) the node table (bin index and
//         weight of R e^{rho_i} on both sides of the detector, float64), the
//         twiddle tables, and the kernel's 2D spectrum: its rho transform in
//         closed form (two lags per angle), transformed along the angle and
//         scaled by dphi / (L n_phi) (the weight drho of the quadrature
//         cancels the kernel's height 1/drho; the inverse transforms are
//         unnormalised);
//   rows  per pair of rays: Step 1 (linear interpolation along the sinogram
//         row) into the real and imaginary parts of one complex sequence,
//         zero-padded to L (a power of two >= 2 N_rho - 1: the convolution in
//         rho is linear), one LDS transform of length L, then the two real
//         spectra separated by their Hermitian symmetry; bins 0 .. L/2 - 1
//         stored in tiles of C consecutive bins, all rays of a tile
//         contiguous, the real bin L/2 in the imaginary part of the real bin 0;
//   conv  per tile: C columns of n_phi rays transformed along the angle
//         (mixed-radix Stockham, n_phi = 2^a 3^b 5^c), times the kernel's
//         spectrum, transformed back (Step 3, periodic in the angle); the
//         packed column of bins 0 and L/2 is split, filtered and recombined;
//   back  per pair of rays: the full spectrum rebuilt from the two half
//         spectra, one inverse transform of length L, the first N_rho values
//         of each ray written out ([B g]_L);
//   cart  Step 4, bilinear in (rho, theta) at every pixel centre (float64
//         coordinates, first node for pixels nearer the origin).
// The transforms are Stockham FFTs in LDS with radix-16, 5, 4, 3 and 2
// butterflies (Govindaraju et al. 2008), twiddles from float64 tables, every
// phase reduced exactly as an integer before its sine and cosine.
#include <algorithm>
#include <cmath>
#include <vector>

#include "tomo.h"

namespace tvpd {
namespace {

constexpr int kLpMaxL = 16384;        // rho transform length limit (LDS)
constexpr int kLpMaxRho = kLpMaxL / 2;
constexpr int kLpMaxPhi = 4096;
constexpr int kLpElems = 16384;       // LDS elements of the angle transforms (n_phi C)
constexpr int kLpThreads = 1024;      // 16 waves: 4 per SIMD at <= 128 VGPRs
constexpr int kLpPer = kLpElems / kLpThreads;          // tile elements per thread
constexpr int kLpRowBatch = 8;                         // rho samples per thread and batch
constexpr int kLpHalfPer = kLpMaxL / 2 / kLpThreads;   // half-spectrum bins per thread
constexpr int kLpMaxStages = 16;
constexpr uint32_t kLpMagic = 0x4c50424bu;

__device__ __forceinline__ int lds_at(int i) { return i + (i >> 4); }
constexpr int kLpRowLds = kLpMaxL + kLpMaxL / 16;

struct LpMesh {
  double R, rho0, drho, dphi;
  int n_rho, n_phi, L;
};

// The mesh of the readings above, in float64 on the host.
LpMesh lp_mesh(int ny, int nx, int na, int nd) {
  LpMesh m;
  m.R = nd / 2.0;
  const double ds = 2.0 / nd;
  m.rho0 = std::log(0.5 / m.R);
  const double rmax = std::hypot(nx / 2.0 - 0.5, ny / 2.0 - 0.5);
  const double top = rmax > 0.0 ? std::fmax(0.0, std::log(rmax / m.R)) : 0.0;
  m.n_rho = (int)std::ceil((top - m.rho0) / -std::log(1.0 - ds));
  m.drho = (top - m.rho0) / m.n_rho;
  m.n_phi = 2 * na;
  m.dphi = M_PI / na;
  int L = 1;
  while (L < 2 * m.n_rho - 1) L *= 2;
  m.L = L;
  return m;
}

// Workspace header (device), written by the plan.
struct LpHdr {
  uint32_t magic;
  int32_t ny, nx, na, nd;
  int32_t pad[59];
};
static_assert(sizeof(LpHdr) == 256, "lp header");

struct LpNode {     // R e^{rho_i} on the detector: bin index and weight, + and - side
  int32_t ip;
  float wp;
  int32_t im;
  float wm;
};

struct LpLayout {
  LpMesh m;
  int ny, nx, na, nd;
  int C;            // bins per tile
  int ntiles;       // tiles of bins 0 .. L/2
  int nstages;
  int radix[kLpMaxStages];     // angle transform, in stage order
  int rstages;
  int rradix[kLpMaxStages];    // rho transform
  size_t off_nodes, off_twr, off_twa, off_k2, off_s, off_bl, bytes;
};

// Radices of a Stockham transform of length n: 16s, one 4 or 2 for the rest
// of the power of two, then 5s and 3s.  False if n has another prime factor.
bool factor(int n, int* r, int* count) {
  int c = 0;
  int p2 = 0;
  while (n % 2 == 0) {
    n /= 2;
    ++p2;
  }
  if (p2 % 4 >= 2) r[c++] = 4;
  if (p2 % 2 == 1) r[c++] = 2;
  for (int i = 0; i < p2 / 4; ++i) r[c++] = 16;
  while (n % 5 == 0) {
    n /= 5;
    r[c++] = 5;
  }
  while (n % 3 == 0) {
    n /= 3;
    r[c++] = 3;
  }
  *count = c;
  return n == 1 && c <= kLpMaxStages;
}

LpLayout lp_layout(int ny, int nx, int na, int nd) {
  LpLayout Y;
  Y.ny = ny;
  Y.nx = nx;
  Y.na = na;
  Y.nd = nd;
  Y.m = lp_mesh(ny, nx, na, nd);
  Y.C = Y.m.n_phi <= kLpElems / 8 ? 8 : 4;
  // at most L/2 bins a tile, so that the last tile holds bin L/2 alone
  // (column 0), the bin packed into bin 0's imaginary part
  Y.C = std::min(Y.C, Y.m.L / 2);
  Y.ntiles = (Y.m.L / 2 + 1 + Y.C - 1) / Y.C;
  if (!factor(Y.m.n_phi, Y.radix, &Y.nstages)) Y.nstages = -1;
  if (!factor(Y.m.L, Y.rradix, &Y.rstages)) Y.rstages = -1;
  const int64_t tile = (int64_t)Y.m.n_phi * Y.C;
  Y.off_nodes = kHeaderBytes;
  Y.off_twr = (size_t)round_up((int64_t)Y.off_nodes + 16 * (int64_t)Y.m.n_rho, kAlign);
  Y.off_twa = (size_t)round_up((int64_t)Y.off_twr + 8 * (int64_t)Y.m.L, kAlign);
  Y.off_k2 = (size_t)round_up((int64_t)Y.off_twa + 8 * (int64_t)Y.m.n_phi, kAlign);
  Y.off_s = (size_t)round_up((int64_t)Y.off_k2 + 8 * tile * Y.ntiles, kAlign);
  Y.off_bl = (size_t)round_up((int64_t)Y.off_s + 8 * tile * Y.ntiles, kAlign);
  Y.bytes = Y.off_bl + 4 * (size_t)Y.m.n_phi * (size_t)Y.m.n_rho;
  return Y;
}

int lp_supported(const LpLayout& Y) {
  if (Y.nd < 4 || Y.m.n_rho < 2 || Y.m.n_rho > kLpMaxRho || Y.m.L > kLpMaxL) return TVPD_ERR_UNSUPPORTED;
  if (Y.m.n_phi > kLpMaxPhi || Y.nstages < 0 || Y.rstages < 0) return TVPD_ERR_UNSUPPORTED;
  return TVPD_OK;
}

// Kernel arguments (by value).
struct LpArgs {
  const LpHdr* hdr;
  const LpNode* nodes;
  const float2* twr;   // exp(-2 pi i m / L), m < L
  const float2* twa;   // exp(-2 pi i m / n_phi), m < n_phi
  float2* k2;          // kernel spectrum tiles [ntiles][n_phi][C]
  float2* s;           // data spectrum tiles, same layout
  float* bl;           // [n_phi][n_rho]
  int ny, nx, na, nd;
  int n_rho, n_phi, L, C, ntiles;
  double R, rho_first, drho, dphi;
  double lnR, inv_drho, inv_dphi;   // ln R, 1 / drho, 1 / dphi
  int nstages, rstages;
  int radix[kLpMaxStages];
  int rradix[kLpMaxStages];
  // rfused: the rho transform's last radix-16 stage runs fused, first in the
  // forward (with Step 1) and last in the inverse (with the stores of
  // [B g]_L), and rrest lists the other stages; otherwise rrest = rradix.
  int rfused, rrest_n;
  int rrest[kLpMaxStages];
};

// ---------------------------------------------------------------------------
// Complex helpers and butterflies.
// ---------------------------------------------------------------------------

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// SIGN i a
template <int SIGN>
__device__ __forceinline__ float2 mul_i(float2 a) {
  return SIGN > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int SIGN>
__device__ __forceinline__ void dft2(float2* v) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <int SIGN>
__device__ __forceinline__ void dft3(float2* v) {
  constexpr float h = 0.86602540378443865f;   // sin(2 pi / 3)
  const float2 t = cadd(v[1], v[2]);
  const float2 s = cscale(mul_i<SIGN>(csub(v[1], v[2])), h);
  const float2 m = make_float2(v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y);
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, s);
  v[2] = csub(m, s);
}

template <int SIGN>
__device__ __forceinline__ void dft4(float2* v) {
  const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  const float2 t2 = cadd(v[1], v[3]), t3 = mul_i<SIGN>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[1] = cadd(t1, t3);
  v[2] = csub(t0, t2);
  v[3] = csub(t1, t3);
}

template <int SIGN>
__device__ __forceinline__ void dft5(float2* v) {
  // cos and sin of 2 pi / 5 and 4 pi / 5
  constexpr float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
  constexpr float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
  const float2 b1 = cadd(v[1], v[4]), b2 = cadd(v[2], v[3]);
  const float2 d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
  const float2 a0 = v[0];
  const float2 r1 = make_float2(a0.x + c1 * b1.x + c2 * b2.x, a0.y + c1 * b1.y + c2 * b2.y);
  const float2 r2 = make_float2(a0.x + c2 * b1.x + c1 * b2.x, a0.y + c2 * b1.y + c1 * b2.y);
  const float2 q1 = mul_i<SIGN>(make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
  const float2 q2 = mul_i<SIGN>(make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
  v[0] = cadd(a0, cadd(b1, b2));
  v[1] = cadd(r1, q1);
  v[4] = csub(r1, q1);
  v[2] = cadd(r2, q2);
  v[3] = csub(r2, q2);
}

// 16 points as 4 x 4: inputs n = 4 n1 + n2, outputs k = k1 + 4 k2.
template <int SIGN>
__device__ __forceinline__ void dft16(float2* v) {
  constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508977f;
  constexpr float h = 0.70710678118654752f;
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    float2 q[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
    dft4<SIGN>(q);
    v[n2] = q[0];
    v[4 + n2] = q[1];
    v[8 + n2] = q[2];
    v[12 + n2] = q[3];
  }
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
    float2 q[4] = {v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]};
    dft4<SIGN>(q);
    y[k1] = q[0];
    y[k1 + 4] = q[1];
    y[k1 + 8] = q[2];
    y[k1 + 12] = q[3];
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = y[r];
}

template <int R, int SIGN>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 2) dft2<SIGN>(v);
  else if constexpr (R == 3) dft3<SIGN>(v);
  else if constexpr (R == 4) dft4<SIGN>(v);
  else if constexpr (R == 5) dft5<SIGN>(v);
  else dft16<SIGN>(v);
}

// ---------------------------------------------------------------------------
// Stockham stages in LDS.  C interleaved transforms of length n: element i
// of transform c at x[i C + c] (PAD = false), or one transform with one
// spare slot per 16 elements (PAD = true, C = 1).  A stage of radix R after
// stages whose radices multiply to Ns: butterfly j (< n/R) of transform c
// reads x[j + r n/R], r < R, twiddles them by w^{r k} (k = j mod Ns,
// w = exp(SIGN 2 pi i / (Ns R)), from tw of length n), transforms them and
// writes x[(j - k) R + k + r Ns].  All loads of the stage come first, then
// the block waits, then the stores.
// ---------------------------------------------------------------------------

template <bool PAD>
__device__ __forceinline__ int at(int i, int C, int c) {
  return PAD ? lds_at(i) : i * C + c;
}

// Twiddle w^i (i < n) from a table of length n ...
struct TwTable {
  const float2* p;
  __device__ __forceinline__ float2 operator()(int i) const { return p[i]; }
};
// ... or as the product of two short tables, w^(128 h) and w^l for
// i = 128 h + l (both in LDS: the row transforms' full table does not fit).
constexpr int kTwSplit = 128;
struct TwSplit {
  const float2* hi;
  const float2* lo;
  __device__ __forceinline__ float2 operator()(int i) const {
    return cmul(hi[i / kTwSplit], lo[i % kTwSplit]);
  }
};

template <int R, int SIGN, bool PAD, int NT, class TW>
__device__ void stage(float2* x, int n, int C, int Ns, TW tw) {
  constexpr int U = (kLpElems / R + NT - 1) / NT;
  const int nb = (n / R) * C;                 // butterflies
  const int stride = n / (Ns * R);
  float2 v[U][R];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int b = threadIdx.x + u * NT;
    if (b < nb) {
      const int j = b / C, c = b - j * C;
#pragma unroll
      for (int r = 0; r < R; ++r) v[u][r] = x[at<PAD>(j + r * (n / R), C, c)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int b = threadIdx.x + u * NT;
    if (b < nb) {
      const int j = b / C, c = b - j * C;
      const int k = j % Ns;
      if (Ns > 1) {   // the first stage's twiddles are all 1
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw(r * k * stride);
          if (SIGN > 0) w.y = -w.y;
          v[u][r] = cmul(v[u][r], w);
        }
      }
      dft<R, SIGN>(v[u]);
      const int d = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) x[at<PAD>(d + r * Ns, C, c)] = v[u][r];
    }
  }
  __syncthreads();
}

// Stages radix[0 .. nstages) after earlier ones whose radices multiply to Ns0.
template <int SIGN, bool PAD, int NT, class TW>
__device__ void fft(float2* x, int n, int C, const int* radix, int nstages, TW tw, int Ns0 = 1) {
  int Ns = Ns0;
  for (int s = 0; s < nstages; ++s) {
    const int R = radix[s];
    switch (R) {
      case 2: stage<2, SIGN, PAD, NT>(x, n, C, Ns, tw); break;
      case 3: stage<3, SIGN, PAD, NT>(x, n, C, Ns, tw); break;
      case 4: stage<4, SIGN, PAD, NT>(x, n, C, Ns, tw); break;
      case 5: stage<5, SIGN, PAD, NT>(x, n, C, Ns, tw); break;
      default: stage<16, SIGN, PAD, NT>(x, n, C, Ns, tw); break;
    }
    Ns *= R;
  }
}

// The row transforms' split twiddle tables (w = exp(-2 pi i / L)): thread j
// loads entry j of both (fetch), then writes them to LDS (put), so that the
// loads can be in flight together with the kernel's own.
struct SplitTwLoad {
  float2 lo, hi;
  __device__ __forceinline__ void fetch(const float2* twr, int L) {
    const int j = threadIdx.x, nh = L > kTwSplit ? L / kTwSplit : 1;
    lo = twr[min(j, L - 1)];
    hi = twr[min(j, nh - 1) * kTwSplit];
  }
  __device__ __forceinline__ void put(int L, float2* th, float2* tl) const {
    const int j = threadIdx.x, nh = L > kTwSplit ? L / kTwSplit : 1;
    if (j < kTwSplit) tl[j] = j < L ? lo : make_float2(0.0f, 0.0f);
    if (j < nh) th[j] = hi;
  }
};
static_assert(kLpThreads >= kTwSplit && kLpThreads >= kLpMaxL / kTwSplit, "split twiddles");

// ---------------------------------------------------------------------------
// Plan.
// ---------------------------------------------------------------------------

__global__ void lp_twiddle_kernel(float2* tw, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  const double a = -2.0 * (double)m / (double)n;
  tw[m] = make_float2((float)cospi(a), (float)sinpi(a));
}

// Node i: R e^{rho_i} as a bin position on both sides of the detector,
// v = +-R e^{rho_i} + n_det/2 - 1/2; its floor and the weight of the next bin.
__global__ void lp_nodes_kernel(LpNode* nodes, int n_rho, double R, double rho_first,
                                double drho, int nd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rho) return;
  const double r = R * exp(rho_first + (double)i * drho);
  const double c = 0.5 * (double)nd - 0.5;
  const double vp = c + r, vm = c - r;
  const double fp = floor(vp), fm = floor(vm);
  LpNode q;
  q.ip = (int)fp;
  q.wp = (float)(vp - fp);
  q.im = (int)fm;
  q.wm = (float)(vm - fm);
  nodes[i] = q;
}

__global__ void lp_header_kernel(LpHdr* h, int ny, int nx, int na, int nd) {
  if (threadIdx.x == 0) {
    h->ny = ny;
    h->nx = nx;
    h->na = na;
    h->nd = nd;
    h->magic = kLpMagic;
  }
}

// The kernel's spectrum for one tile of bins: the rho transform of ray j in
// closed form (weights w0, w1 at lags l0, l0 + 1 around the root of
// e^a cos phi_j = 1; nothing where cos phi_j <= 0 or the lag leaves the
// mesh), then the angle transform of each of the C columns, scaled.
__global__ __launch_bounds__(kLpThreads) void lp_kernel_spectrum_kernel(LpArgs a) {
  __shared__ float2 x[kLpElems];
  const int kt = blockIdx.x;
  const int n = a.n_phi, C = a.C;
  for (int e = threadIdx.x; e < n * C; e += kLpThreads) {
    const int j = e / C, c = e - j * C;
    const int k = kt * C + c;                  // rho frequency
    double re = 0.0, im = 0.0;
    const double cs = cospi((double)j / (double)a.na);
    if (k <= a.L / 2 && cs > 0.0) {
      const double xr = -log(cs) / a.drho;
      const double fl = floor(xr);
      if (fl <= (double)(a.n_rho - 1)) {
        const int l0 = (int)fl;
        const double w1 = xr - fl, w0 = 1.0 - w1;
        // exp(-2 pi i k l / L) with k l reduced modulo L
        const int64_t m0 = ((int64_t)k * l0) % a.L;
        re += w0 * cospi(-2.0 * (double)m0 / a.L);
        im += w0 * sinpi(-2.0 * (double)m0 / a.L);
        if (l0 + 1 <= a.n_rho - 1) {
          const int64_t m1 = ((int64_t)k * (l0 + 1)) % a.L;
          re += w1 * cospi(-2.0 * (double)m1 / a.L);
          im += w1 * sinpi(-2.0 * (double)m1 / a.L);
        }
      }
    }
    x[e] = make_float2((float)re, (float)im);
  }
  __syncthreads();
  fft<-1, false, kLpThreads>(x, n, C, a.radix, a.nstages, TwTable{a.twa});
  const float scale = (float)(a.dphi / ((double)a.L * (double)n));
  float2* out = a.k2 + (int64_t)kt * n * C;
  for (int e = threadIdx.x; e < n * C; e += kLpThreads) out[e] = cscale(x[e], scale);
}

// ---------------------------------------------------------------------------
// The transform.
// ---------------------------------------------------------------------------

// Both samples are loaded unconditionally (clamped indices) so that the
// loads of a batch are all in flight before the first use.
__device__ __forceinline__ float lp_interp(const float* row, int nd, int i0, float w) {
  const float r0 = row[min(max(i0, 0), nd - 1)];
  const float r1 = row[min(max(i0 + 1, 0), nd - 1)];
  const float s0 = (i0 >= 0 && i0 < nd) ? r0 : 0.0f;
  const float s1 = (i0 + 1 >= 0 && i0 + 1 < nd) ? r1 : 0.0f;
  return fmaf(w, s1, (1.0f - w) * s0);
}

// Step 1 for rays j0 and j0 + 1 and their rho transforms (see the file
// comment); bins 0 .. L/2 of both spectra into the tiles.
__global__ __launch_bounds__(kLpThreads) void lp_rows_forward_kernel(LpArgs a, const float* g) {
  __shared__ float2 x[kLpRowLds];
  __shared__ float2 twh[kLpMaxL / kTwSplit], twl[kTwSplit];
  const int j0 = 2 * blockIdx.x;
  const int L = a.L;
  const int ka = j0 < a.na ? j0 : j0 - a.na;
  const int kb = j0 + 1 < a.na ? j0 + 1 : j0 + 1 - a.na;
  const bool pa = j0 < a.na, pb = j0 + 1 < a.na;
  const float* ga = g + (int64_t)ka * a.nd;
  const float* gb = g + (int64_t)kb * a.nd;
  SplitTwLoad stw;
  stw.fetch(a.twr, L);
  const int nr = a.n_rho;
  auto sample = [&](const LpNode& q, int i) {
    const float va = pa ? lp_interp(ga, a.nd, q.ip, q.wp) : lp_interp(ga, a.nd, q.im, q.wm);
    const float vb = pb ? lp_interp(gb, a.nd, q.ip, q.wp) : lp_interp(gb, a.nd, q.im, q.wm);
    return i < nr ? make_float2(va, vb) : make_float2(0.0f, 0.0f);
  };
  if (a.rfused) {
    // First stage radix 16 (Ns = 1, no twiddles) on Step 1's values in
    // registers: butterfly j takes samples j + r L/16, of which r >= 8 lie
    // in the zero padding (N_rho <= L/2).
    const int m = L / 16, jb = threadIdx.x;
    LpNode q[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) q[r] = a.nodes[min(jb + r * m, nr - 1)];
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = sample(q[r], jb + r * m);
#pragma unroll
    for (int r = 8; r < 16; ++r) v[r] = make_float2(0.0f, 0.0f);
    if (jb < m) {
      dft16<-1>(v);
#pragma unroll
      for (int r = 0; r < 16; ++r) x[lds_at(16 * jb + r)] = v[r];
    }
  } else {
    // Batches of kLpRowBatch samples per thread: every node of the batch,
    // then every sinogram sample, then the LDS stores (one wait per batch).
    for (int i0 = 0; i0 < L; i0 += kLpRowBatch * kLpThreads) {
      LpNode q[kLpRowBatch];
#pragma unroll
      for (int u = 0; u < kLpRowBatch; ++u)
        q[u] = a.nodes[min(i0 + (int)threadIdx.x + u * kLpThreads, nr - 1)];
      float2 v[kLpRowBatch];
#pragma unroll
      for (int u = 0; u < kLpRowBatch; ++u) v[u] = sample(q[u], i0 + (int)threadIdx.x + u * kLpThreads);
#pragma unroll
      for (int u = 0; u < kLpRowBatch; ++u) {
        const int i = i0 + (int)threadIdx.x + u * kLpThreads;
        if (i < L) x[lds_at(i)] = v[u];
      }
    }
  }
  stw.put(L, twh, twl);
  __syncthreads();
  fft<-1, true, kLpThreads>(x, L, 1, a.rrest, a.rrest_n, TwSplit{twh, twl}, a.rfused ? 16 : 1);
  const int C = a.C;
  for (int k = threadIdx.x; k < L / 2; k += kLpThreads) {
    const float2 z1 = x[lds_at(k)];
    const float2 z2 = x[lds_at((L - k) & (L - 1))];
    // A = (z1 + conj z2) / 2, B = (z1 - conj z2) / (2 i)
    float2 A = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y));
    float2 B = make_float2(0.5f * (z1.y + z2.y), 0.5f * (z2.x - z1.x));
    if (k == 0) {
      // bins 0 and L/2 of both rays are real: bin L/2 rides in the
      // imaginary part of bin 0 (their angle convolutions are separated
      // again in lp_angle_conv_kernel)
      const float2 zn = x[lds_at(L / 2)];
      A = make_float2(z1.x, zn.x);
      B = make_float2(z1.y, zn.y);
    }
    const int kt = k / C, c = k - kt * C;
    float2* t = a.s + ((int64_t)kt * a.n_phi + j0) * C + c;
    t[0] = A;
    t[C] = B;
  }
}

// Step 3 along the angle for one tile of C bins.  The angle twiddles sit in
// LDS beside the tile (every stage reads R - 1 of them per butterfly).
// C (the tile's bins, a.C) is a template parameter: the butterflies' column
// and row indices are then shifts, cheap enough to recompute in every stage.
template <int C>
__global__ __launch_bounds__(kLpThreads) void lp_angle_conv_kernel(LpArgs a) {
  __shared__ float2 x[kLpElems];
  __shared__ float2 tw[kLpMaxPhi];
  const int n = a.n_phi;
  float2* t = a.s + (int64_t)blockIdx.x * n * C;
  const float2* kk = a.k2 + (int64_t)blockIdx.x * n * C;
  const int nc = n * C;
  {
    // every load of the tile and the twiddles in flight before the first
    // LDS store
    constexpr int kTw = kLpMaxPhi / kLpThreads;
    float2 r[kLpPer], w[kTw];
#pragma unroll
    for (int u = 0; u < kLpPer; ++u) r[u] = t[min((int)threadIdx.x + u * kLpThreads, nc - 1)];
#pragma unroll
    for (int u = 0; u < kTw; ++u) w[u] = a.twa[min((int)threadIdx.x + u * kLpThreads, n - 1)];
#pragma unroll
    for (int u = 0; u < kTw; ++u) {
      const int e = threadIdx.x + u * kLpThreads;
      if (e < n) tw[e] = w[u];
    }
#pragma unroll
    for (int u = 0; u < kLpPer; ++u) {
      const int e = threadIdx.x + u * kLpThreads;
      if (e < nc) x[e] = r[u];
    }
  }
  __syncthreads();
  fft<-1, false, kLpThreads>(x, n, C, a.radix, a.nstages, TwTable{tw});
  const bool packed = blockIdx.x == 0;
  {
    float2 r[kLpPer];
#pragma unroll
    for (int u = 0; u < kLpPer; ++u) r[u] = kk[min((int)threadIdx.x + u * kLpThreads, nc - 1)];
#pragma unroll
    for (int u = 0; u < kLpPer; ++u) {
      const int e = threadIdx.x + u * kLpThreads;
      if (e < nc && (!packed || e % C != 0)) x[e] = cmul(x[e], r[u]);
    }
  }
  if (packed) {
    // Column 0 holds z = x0 + i xN, the real sequences of bins 0 and L/2
    // over the angle.  With Z its transform, X0[m] = (Z[m] + conj Z[-m]) / 2
    // and XN[m] = (Z[m] - conj Z[-m]) / (2 i); each is multiplied by its own
    // kernel spectrum (bin L/2's sits in column 0 of the last tile) and the
    // two are recombined as X0 K0 + i XN KN, whose inverse transform is
    // (x0 * k0) + i (xN * kN).  Pairs (m, n - m) go to one thread.
    const float2* kn = a.k2 + (int64_t)(a.ntiles - 1) * n * C;
    auto one = [](float2 zm, float2 zmm, float2 k0, float2 kN) {
      const float2 x0 = make_float2(0.5f * (zm.x + zmm.x), 0.5f * (zm.y - zmm.y));
      const float2 xn = make_float2(0.5f * (zm.y + zmm.y), 0.5f * (zmm.x - zm.x));
      const float2 y0 = cmul(x0, k0), yn = cmul(xn, kN);
      return make_float2(y0.x - yn.y, y0.y + yn.x);
    };
    for (int m = threadIdx.x; m <= n / 2; m += kLpThreads) {
      const int mm = (n - m) % n;
      const float2 zm = x[m * C], zmm = x[mm * C];
      const float2 ym = one(zm, zmm, kk[m * C], kn[m * C]);
      const float2 ymm = one(zmm, zm, kk[mm * C], kn[mm * C]);
      x[m * C] = ym;
      if (mm != m) x[mm * C] = ymm;
    }
  }
  __syncthreads();
  fft<+1, false, kLpThreads>(x, n, C, a.radix, a.nstages, TwTable{tw});
  for (int e = threadIdx.x; e < n * C; e += kLpThreads) t[e] = x[e];
}

// Inverse rho transforms of rays j0 and j0 + 1 from their half spectra:
// Z = A + i B with Z[L - k] = conj(A[k]) + i conj(B[k]); the real and
// imaginary parts of the result are the two rays.
__global__ __launch_bounds__(kLpThreads) void lp_rows_inverse_kernel(LpArgs a) {
  __shared__ float2 x[kLpRowLds];
  __shared__ float2 twh[kLpMaxL / kTwSplit], twl[kTwSplit];
  const int j0 = 2 * blockIdx.x;
  const int L = a.L, C = a.C;
  SplitTwLoad stw;
  stw.fetch(a.twr, L);
  float2 A_[kLpHalfPer], B_[kLpHalfPer];
#pragma unroll
  for (int u = 0; u < kLpHalfPer; ++u) {
    // every load in flight before the first LDS store
    const int k = min((int)threadIdx.x + u * kLpThreads, L / 2 - 1);
    const int kt = k / C, c = k - kt * C;
    const float2* t = a.s + ((int64_t)kt * a.n_phi + j0) * C + c;
    A_[u] = t[0];
    B_[u] = t[C];
  }
#pragma unroll
  for (int u = 0; u < kLpHalfPer; ++u) {
    const int k = threadIdx.x + u * kLpThreads;
    if (k >= L / 2) break;
    const float2 A = A_[u], B = B_[u];
    if (k == 0) {
      // bins 0 and L/2 come packed (real parts bin 0, imaginary bin L/2)
      x[lds_at(0)] = make_float2(A.x, B.x);
      x[lds_at(L / 2)] = make_float2(A.y, B.y);
    } else {
      x[lds_at(k)] = make_float2(A.x - B.y, A.y + B.x);
      x[lds_at(L - k)] = make_float2(A.x + B.y, B.x - A.y);
    }
  }
  stw.put(L, twh, twl);
  __syncthreads();
  float* ra = a.bl + (int64_t)j0 * a.n_rho;
  float* rb = ra + a.n_rho;
  const TwSplit tw{twh, twl};
  fft<+1, true, kLpThreads>(x, L, 1, a.rrest, a.rrest_n, tw);
  if (a.rfused) {
    // The last stage (radix 16, Ns = L/16) in registers: butterfly j reads
    // and yields elements j + r L/16, stored straight to [B g]_L.
    const int m = L / 16, jb = threadIdx.x;
    if (jb < m) {
      float2 v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = x[lds_at(jb + r * m)];
#pragma unroll
      for (int r = 1; r < 16; ++r) {
        float2 w = tw(r * jb);
        w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
      dft16<+1>(v);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = jb + r * m;
        if (i < a.n_rho) {
          ra[i] = v[r].x;
          rb[i] = v[r].y;
        }
      }
    }
  } else {
    for (int i = threadIdx.x; i < a.n_rho; i += kLpThreads) {
      const float2 v = x[lds_at(i)];
      ra[i] = v.x;
      rb[i] = v.y;
    }
  }
}

// Step 4 for one pixel per thread (grid: column blocks by rows).  A
// workspace not planned for this geometry gives NaN everywhere.
__global__ __launch_bounds__(kMaxBlock) void lp_cartesian_kernel(LpArgs a, float* img) {
  const int col = blockIdx.x * kMaxBlock + threadIdx.x, row = blockIdx.y;
  if (col >= a.nx) return;
  const int64_t p = (int64_t)row * a.nx + col;
  const LpHdr* h = a.hdr;
  if (h->magic != kLpMagic || h->ny != a.ny || h->nx != a.nx || h->na != a.na ||
      h->nd != a.nd) {
    img[p] = __builtin_nanf("");
    return;
  }
  const double x = col + 0.5 - 0.5 * a.nx, y = row + 0.5 - 0.5 * a.ny;
  // ln(r / R) as ln(r^2) / 2 - ln R, and multiplications by 1/drho and
  // 1/dphi: no float64 square root or division per pixel
  double u = (0.5 * log(x * x + y * y) - a.lnR - a.rho_first) * a.inv_drho;   // -inf at the origin
  u = fmin(fmax(u, 0.0), (double)(a.n_rho - 1));
  double th = atan2(y, x);
  if (th < 0.0) th += 2.0 * M_PI;
  const double v = th * a.inv_dphi;
  int i0 = (int)floor(u);
  if (i0 > a.n_rho - 2) i0 = a.n_rho - 2;
  const float wu = (float)(u - i0);
  int j0 = (int)floor(v);
  const float wv = (float)(v - j0);
  j0 %= a.n_phi;
  const int j1 = j0 + 1 < a.n_phi ? j0 + 1 : 0;
  const float* b0 = a.bl + (int64_t)j0 * a.n_rho + i0;
  const float* b1 = a.bl + (int64_t)j1 * a.n_rho + i0;
  const float v0 = fmaf(wu, b0[1], (1.0f - wu) * b0[0]);
  const float v1 = fmaf(wu, b1[1], (1.0f - wu) * b1[0]);
  img[p] = fmaf(wv, v1, (1.0f - wv) * v0);
}

#define LP_TRY(call)                    \
  do {                                  \
    const int st_ = (call);             \
    if (st_ != TVPD_OK) return st_;     \
  } while (0)

int launched() { return hipGetLastError() == hipSuccess ? TVPD_OK : TVPD_ERR_HIP; }

bool geom_ok(const tvpd_tomo_geom* g) {
  if (!g) return false;
  return g->ny >= 1 && g->nx >= 1 && g->n_angles >= 1 && g->n_det >= 1 &&
         g->ny <= kTomoMaxSide && g->nx <= kTomoMaxSide && g->n_det <= kTomoMaxSide &&
         g->n_angles <= kTomoMaxAngles;
}

int ws_check(const LpLayout& Y, const void* ws, size_t bytes) {
  if (!ws) return TVPD_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return TVPD_ERR_ALIGNMENT;
  if (bytes < Y.bytes) return TVPD_ERR_WORKSPACE;
  return TVPD_OK;
}

LpArgs lp_args(const LpLayout& Y, void* ws) {
  char* base = static_cast<char*>(ws);
  LpArgs a{};
  a.hdr = reinterpret_cast<const LpHdr*>(base);
  a.nodes = reinterpret_cast<const LpNode*>(base + Y.off_nodes);
  a.twr = reinterpret_cast<const float2*>(base + Y.off_twr);
  a.twa = reinterpret_cast<const float2*>(base + Y.off_twa);
  a.k2 = reinterpret_cast<float2*>(base + Y.off_k2);
  a.s = reinterpret_cast<float2*>(base + Y.off_s);
  a.bl = reinterpret_cast<float*>(base + Y.off_bl);
  a.ny = Y.ny;
  a.nx = Y.nx;
  a.na = Y.na;
  a.nd = Y.nd;
  a.n_rho = Y.m.n_rho;
  a.n_phi = Y.m.n_phi;
  a.L = Y.m.L;
  a.C = Y.C;
  a.ntiles = Y.ntiles;
  a.R = Y.m.R;
  a.rho_first = Y.m.rho0 + Y.m.drho;
  a.drho = Y.m.drho;
  a.dphi = Y.m.dphi;
  a.lnR = std::log(Y.m.R);
  a.inv_drho = 1.0 / Y.m.drho;
  a.inv_dphi = 1.0 / Y.m.dphi;
  a.nstages = Y.nstages;
  a.rstages = Y.rstages;
  for (int i = 0; i < kLpMaxStages; ++i) {
    a.radix[i] = i < Y.nstages ? Y.radix[i] : 0;
    a.rradix[i] = i < Y.rstages ? Y.rradix[i] : 0;
    a.rrest[i] = 0;
  }
  int last16 = -1;
  for (int i = 0; i < Y.rstages; ++i)
    if (Y.rradix[i] == 16) last16 = i;
  a.rfused = last16 >= 0 && Y.m.L / 16 <= kLpThreads;
  a.rrest_n = 0;
  for (int i = 0; i < Y.rstages; ++i)
    if (!a.rfused || i != last16) a.rrest[a.rrest_n++] = Y.rradix[i];
  return a;
}

int prepare(const tvpd_tomo_geom* geom, void* ws, size_t ws_bytes, LpLayout* Y) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  *Y = lp_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  LP_TRY(lp_supported(*Y));
  return ws_check(*Y, ws, ws_bytes);
}

}  // namespace
}  // namespace tvpd

using namespace tvpd;

extern "C" {

int tvpd_lp_mesh(const tvpd_tomo_geom* geom, int32_t* n_rho, int32_t* n_phi, int32_t* L,
                 double* rho0, double* drho) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!n_rho || !n_phi || !L || !rho0 || !drho) return TVPD_ERR_INVALID_ARG;
  const LpLayout Y = lp_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  *n_rho = Y.m.n_rho;
  *n_phi = Y.m.n_phi;
  *L = Y.m.L;
  *rho0 = Y.m.rho0;
  *drho = Y.m.drho;
  return lp_supported(Y);
}

int tvpd_lp_workspace_size(const tvpd_tomo_geom* geom, size_t* bytes) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!bytes) return TVPD_ERR_INVALID_ARG;
  const LpLayout Y = lp_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  LP_TRY(lp_supported(Y));
  *bytes = Y.bytes;
  return TVPD_OK;
}

int tvpd_lp_plan(const tvpd_tomo_geom* geom, void* ws, size_t ws_bytes, void* stream) {
  LpLayout Y;
  LP_TRY(prepare(geom, ws, ws_bytes, &Y));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const LpArgs a = lp_args(Y, ws);
  char* base = static_cast<char*>(ws);
  lp_twiddle_kernel<<<(Y.m.L + 255) / 256, 256, 0, s>>>(
      reinterpret_cast<float2*>(base + Y.off_twr), Y.m.L);
  LP_TRY(launched());
  lp_twiddle_kernel<<<(Y.m.n_phi + 255) / 256, 256, 0, s>>>(
      reinterpret_cast<float2*>(base + Y.off_twa), Y.m.n_phi);
  LP_TRY(launched());
  lp_nodes_kernel<<<(Y.m.n_rho + 255) / 256, 256, 0, s>>>(
      reinterpret_cast<LpNode*>(base + Y.off_nodes), Y.m.n_rho, Y.m.R, a.rho_first, Y.m.drho,
      Y.nd);
  LP_TRY(launched());
  lp_kernel_spectrum_kernel<<<Y.ntiles, kLpThreads, 0, s>>>(a);
  LP_TRY(launched());
  lp_header_kernel<<<1, 64, 0, s>>>(reinterpret_cast<LpHdr*>(base), Y.ny, Y.nx, Y.na, Y.nd);
  return launched();
}

int tvpd_lp_backproject(const tvpd_tomo_geom* geom, const float* g, float* img,
                        float* lp_out, void* ws, size_t ws_bytes, void* stream) {
  LpLayout Y;
  LP_TRY(prepare(geom, ws, ws_bytes, &Y));
  if (!g || !img) return TVPD_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const LpArgs a = lp_args(Y, ws);
  lp_rows_forward_kernel<<<Y.m.n_phi / 2, kLpThreads, 0, s>>>(a, g);
  LP_TRY(launched());
  // (the last tile holds bin L/2 alone, which rides with bin 0)
  if (Y.C == 8)
    lp_angle_conv_kernel<8><<<Y.ntiles - 1, kLpThreads, 0, s>>>(a);
  else if (Y.C == 4)
    lp_angle_conv_kernel<4><<<Y.ntiles - 1, kLpThreads, 0, s>>>(a);
  else
    lp_angle_conv_kernel<2><<<Y.ntiles - 1, kLpThreads, 0, s>>>(a);
  LP_TRY(launched());
  lp_rows_inverse_kernel<<<Y.m.n_phi / 2, kLpThreads, 0, s>>>(a);
  LP_TRY(launched());
  lp_cartesian_kernel<<<dim3((unsigned)((Y.nx + kMaxBlock - 1) / kMaxBlock), (unsigned)Y.ny),
                        kMaxBlock, 0, s>>>(a, img);
  LP_TRY(launched());
  if (lp_out &&
      hipMemcpyAsync(lp_out, a.bl, 4 * (size_t)Y.m.n_phi * Y.m.n_rho, hipMemcpyDeviceToDevice,
                     s) != hipSuccess)
    return TVPD_ERR_HIP;
  return TVPD_OK;
}

}  // extern "C"
