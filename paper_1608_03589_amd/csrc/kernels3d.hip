// Plain-solver kernels of the 3D path: the fused sweep (one launch = one
// iteration over the whole volume, see tile3d.h), initialisation, read-out
// and the standalone energy/gap evaluation.
//
// Each sweep launch reads 24 bytes per voxel (f^k, f^{k-1}, p^k x3, g) and
// writes 16 (f^{k+1}, p^{k+1} x3), plus the halo rows and planes of the
// tiles (mostly L2 hits).  Completion works as in 2D: the last block
// advances the device-side iteration counter or applies the stopping rule.
#include "finish.h"
#include "tile3d.h"

namespace tvpd {
namespace {

using namespace dev;

template <int TH, bool GAP>
__global__ __launch_bounds__(kMaxBlock) void sweep3d_kernel(Sweep3DArgs a) {
  DevState* st = a.st;
  const int k = st->k;
  if (st->converged || k >= st->k_end) return;
  // (not wave_in_block(): measured 2-3 % slower in the 3D kernels)
  const int wave = threadIdx.x / kWave;
  // each XCD (blocks dispatched round-robin over 8) gets a contiguous run of
  // tiles: neighbouring bands and segments share halo rows in its L2
  const int nb = gridDim.x, b = blockIdx.x;
  const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
  const int bt = xcd * q8 + min(xcd, r8) + (b >> 3);
  const int wt = bt * a.wpb + wave;
  double acc_gap = 0.0, acc_P = 0.0;
  if (wt < a.ntiles) {
    const int per_seg = a.ntx * a.nty;
    const int tzi = wt / per_seg;
    const int rem = wt - tzi * per_seg;
    const int ty = rem / a.ntx;
    const int tx = rem - ty * a.ntx;
    const int64_t PL = a.plane;
    Tile3DCtx c;
    c.fk = a.base + plain3_f(k) * PL;
    c.fkm = a.base + plain3_f(k - 1) * PL;
    c.fn = a.base + plain3_f(k + 1) * PL;
    c.pk = a.base + plain3_p(k) * PL;
    c.pn = a.base + plain3_p(k + 1) * PL;
    c.g = a.base + kPlainG3D * PL;
    c.cs = PL;
    c.nz = a.nz;
    c.ny = a.ny;
    c.nx = a.nx;
    c.pitch = a.pitch;
    c.x0 = tx * kStripCols;
    c.y0 = ty * TH;
    c.z0 = tzi * a.tz;
    c.z1 = min(c.z0 + a.tz, a.nz);
    c.lam = a.lam;
    c.tau = a.tau;
    c.sig = a.sigma;
    c.th = a.theta;
    sweep_tile3d<TH, GAP>(c, acc_gap, acc_P);
  }
  finish_sweep<GAP>(st, a.partials, k, 1, acc_gap, acc_P, a.tau);
}

__global__ void init3d_kernel(float* base, int64_t plane, int nz, int ny,
                              int nx, int pitch, const float* __restrict__ g,
                              DevState* st) {
  const int64_t n = (int64_t)nz * ny * pitch;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / pitch;
    const int x = (int)(i - row * pitch);
    const float v = (x < nx) ? g[row * nx + x] : 0.0f;
    for (int s = 0; s < kPlainPlanes3D; ++s) base[s * plane + i] = 0.0f;
    base[plain3_f(0) * plane + i] = v;   // f^0
    base[plain3_f(-1) * plane + i] = v;  // f^{-1}
    base[kPlainG3D * plane + i] = v;     // g (p^0 = 0)
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->k = 0;
    st->k_end = 0x7fffffff;
    st->converged = 0;
    st->iters = 0;
    st->checks = 0;
    st->nblocks = 0;
    st->flags = 0;
    st->P = st->D = st->gap = 0.0;
    st->tol = -1.0;
    st->tau_prev = 0.0f;
    st->slot = 0;
    SyncArea* sa = reinterpret_cast<SyncArea*>(reinterpret_cast<char*>(st) +
                                               kSyncOffset);
    for (int i = 0; i < kSyncGroups; ++i) sa->sub[i].v = 0;
    sa->top.v = 0;
    sa->gen.v = 0;
  }
}

__global__ void read3d_kernel(const float* base, int64_t plane, int nz,
                              int ny, int nx, int pitch, const DevState* st,
                              float* f_out, float* p_out) {
  const int k = st->k;
  const float* f = base + plain3_f(k) * plane;
  const float* p = base + plain3_p(k) * plane;
  const int64_t n = (int64_t)nz * ny * nx;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / nx;
    const int x = (int)(i - row * nx);
    const int64_t s = row * pitch + x;
    f_out[i] = f[s];
    if (p_out) {
      p_out[i] = p[s];
      p_out[n + i] = p[plane + s];
      p_out[2 * n + i] = p[2 * plane + s];
    }
  }
}

// Gap density and primal energy of the current pair, one voxel per thread
// (neighbours read directly; used outside the iteration loop only).
__global__ __launch_bounds__(kMaxBlock) void energy3d_kernel(
    const float* base, int64_t plane, int nz, int ny, int nx, int pitch,
    float lam, const DevState* st, double* partials, int skip_if_converged) {
  if (skip_if_converged && st->converged) return;
  __shared__ double red[2][kMaxBlock / kWave];
  const int k = st->k;
  const float* f = base + plain3_f(k) * plane;
  const float* px = base + plain3_p(k) * plane;
  const float* py = px + plane;
  const float* pz = py + plane;
  const float* g = base + kPlainG3D * plane;
  const int64_t n = (int64_t)nz * ny * nx;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sg = 0.0, sp = 0.0;
  if (i < n) {
    const int64_t row = i / nx;
    const int x = (int)(i - row * nx);
    const int z = (int)(row / ny);
    const int y = (int)(row - (int64_t)z * ny);
    const int64_t SZ = (int64_t)ny * pitch;
    const int64_t s = row * pitch + x;
    const double fv = f[s];
    const double gx = (x < nx - 1) ? (double)f[s + 1] - fv : 0.0;
    const double gy = (y < ny - 1) ? (double)f[s + pitch] - fv : 0.0;
    const double gz = (z < nz - 1) ? (double)f[s + SZ] - fv : 0.0;
    const double dxl = (x > 0) ? (double)px[s - 1] : 0.0;
    const double dyl = (y > 0) ? (double)py[s - pitch] : 0.0;
    const double dzl = (z > 0) ? (double)pz[s - SZ] : 0.0;
    double d = ((double)px[s] - dxl) + ((double)py[s] - dyl);
    d = d + ((double)pz[s] - dzl);
    const double e = fv - (double)g[s];
    const double r = e - d;
    const double nrm = sqrt(gx * gx + gy * gy + gz * gz);
    sg = 0.5 * r * r + (double)lam * nrm -
         (gx * px[s] + gy * py[s] + gz * pz[s]);
    sp = 0.5 * e * e + (double)lam * nrm;
  }
  block_sum2(sg, sp, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sg;
    partials[2 * blockIdx.x + 1] = sp;
  }
}

}  // namespace

bool tile3d_ok(const Tile3D& t) {
  return (t.th == 2 || t.th == 4) && t.tz >= 1 &&
         (t.wpb == 1 || t.wpb == 2 || t.wpb == 4);
}

static void tile_counts3d(const Layout& L, const Tile3D& t, int* ntx, int* nty,
                          int* ntz) {
  *ntx = (L.nx + kStripCols - 1) / kStripCols;
  *nty = (L.ny + t.th - 1) / t.th;
  *ntz = (L.nz + t.tz - 1) / t.tz;
}

int sweep3d_blocks(const Layout& L, const Tile3D& t) {
  int ntx, nty, ntz;
  tile_counts3d(L, t, &ntx, &nty, &ntz);
  const int64_t nt = (int64_t)ntx * nty * ntz;
  return (int)((nt + t.wpb - 1) / t.wpb);
}

hipError_t launch_init3d(const Layout& L, const float* g, void* ws,
                         hipStream_t s) {
  hipLaunchKernelGGL(init3d_kernel,
                     dim3(grid_for((int64_t)L.nz * L.ny * L.pitch, 256)),
                     dim3(256), 0, s, planes_of(L, ws), L.plane, L.nz, L.ny,
                     L.nx, L.pitch, g, state_of(ws));
  return hipGetLastError();
}

hipError_t launch_sweep3d(const Layout& L, const Tile3D& t,
                          const tvpd_coeffs& c, bool with_gap, void* ws,
                          hipStream_t s) {
  if (!tile3d_ok(t)) return hipErrorInvalidValue;
  Sweep3DArgs a;
  a.base = planes_of(L, ws);
  a.plane = L.plane;
  a.nz = L.nz;
  a.ny = L.ny;
  a.nx = L.nx;
  a.pitch = L.pitch;
  a.tz = t.tz;
  a.wpb = t.wpb;
  tile_counts3d(L, t, &a.ntx, &a.nty, &a.ntz);
  const int64_t nt = (int64_t)a.ntx * a.nty * a.ntz;
  if (nt > INT32_MAX / 2) return hipErrorInvalidValue;
  a.ntiles = (int)nt;
  a.lam = c.lam;
  a.tau = c.tau;
  a.sigma = c.sigma;
  a.theta = c.theta;
  a.st = state_of(ws);
  a.partials = partials_of(L, ws);
  const int nb = (a.ntiles + t.wpb - 1) / t.wpb;
  if (nb > L.max_partials) return hipErrorInvalidValue;
  const dim3 grid(nb), block(t.wpb * kWave);
  if (t.th == 2) {
    if (with_gap)
      hipLaunchKernelGGL((sweep3d_kernel<2, true>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((sweep3d_kernel<2, false>), grid, block, 0, s, a);
  } else {
    if (with_gap)
      hipLaunchKernelGGL((sweep3d_kernel<4, true>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((sweep3d_kernel<4, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_read3d(const Layout& L, const void* ws, float* f_out,
                         float* p_out, hipStream_t s) {
  void* w = const_cast<void*>(ws);
  hipLaunchKernelGGL(read3d_kernel,
                     dim3(grid_for((int64_t)L.nz * L.ny * L.nx, 256)),
                     dim3(256), 0, s, planes_of(L, w), L.plane, L.nz, L.ny,
                     L.nx, L.pitch, state_of(w), f_out, p_out);
  return hipGetLastError();
}

hipError_t launch_energy3d(const Layout& L, float lam, void* ws,
                           bool skip_if_converged, hipStream_t s) {
  const int64_t n = (int64_t)L.nz * L.ny * L.nx;
  const int64_t nb = (n + kMaxBlock - 1) / kMaxBlock;
  if (nb > L.max_partials || nb > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(energy3d_kernel, dim3((unsigned)nb), dim3(kMaxBlock), 0,
                     s, planes_of(L, ws), L.plane, L.nz, L.ny, L.nx, L.pitch,
                     lam, state_of(ws), partials_of(L, ws),
                     skip_if_converged ? 1 : 0);
  return launch_energy_final(L, ws, (int)nb, skip_if_converged, s);
}

}  // namespace tvpd
