// Plain-solver kernels of the 2D path: the fused sweep (one launch = a pass
// of 1 .. kMaxPass iterations over the whole image, see tile2d_xs.h),
// initialisation, read-out and the standalone energy/gap evaluation.
//
// A pass of n iterations reads 16 bytes per pixel (f^k, p^k x2, g) and
// writes 12 (f^{k+n}, p^{k+n} x2).  The last block to finish advances the
// iteration counter kept in device memory, or on a gap check reduces the
// per-block partials in a fixed order and applies the stopping rule.
#include <atomic>

#include "finish.h"
#include "tile2d_pipe.h"
#include "tile2d_xs.h"

namespace tvpd {
namespace {

using namespace dev;

// S iterations per launch on overlapping strips of xs_owned(S) owned
// columns (tile2d_xs.h).
template <int S, bool GAP>
__global__ __launch_bounds__(kMaxBlock) void sweep2d_xs_kernel(Sweep2DArgs a) {
  DevState* st = a.st;
  const int k = st->k;
  if (st->converged || k + S > st->k_end) return;
  const float tau_prev = st->tau_prev;
  const int slot = st->slot;
  // (not wave_in_block(): with uniform tile coordinates the compiler's
  // schedule of the depth-5 walk needs more than 256 registers)
  const int wave = threadIdx.x / kWave;
  // Blocks are dispatched round-robin over the 8 XCDs; hand each XCD a
  // contiguous run of tiles so that vertically adjacent bands (which share
  // halo rows) meet in the same L2.
  const int nb = gridDim.x, b = blockIdx.x;
  const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
  const int bt = xcd * q8 + min(xcd, r8) + (b >> 3);
  const int wt = bt * a.wpb + wave;
  double acc_gap = 0.0, acc_P = 0.0;
  if (wt < a.ntiles) {
    TileCtxS c;
    const int64_t PL = a.plane;
    c.F = a.base + plain_f(slot) * PL;
    c.FN = a.base + plain_f(slot ^ 1) * PL;
    c.PX = a.base + plain_p(slot) * PL;
    c.PY = c.PX + PL;
    c.QX = a.base + plain_p(slot ^ 1) * PL;
    c.QY = c.QX + PL;
    c.G = a.base + kPlainG * PL;
    int tx, ty;
    if (a.order == 0) {
      ty = wt / a.ntx;
      tx = wt - ty * a.ntx;
    } else {
      tx = wt / a.nty;
      ty = wt - tx * a.nty;
    }
    c.ny = a.ny;
    c.nx = a.nx;
    c.pitch = a.pitch;
    c.x0 = tx * xs_owned(S);
    c.y0 = ty * a.th;
    c.y1 = min(c.y0 + a.th, a.ny);
    c.lam = a.lam;
    c.tau = a.tau;
    c.sig = a.sigma;
    c.th = a.theta;
    c.tau_prev = tau_prev;
    sweep_tile_xs<S, xs_margin(S), GAP>(c, acc_gap, acc_P);
  }
  finish_sweep<GAP>(st, a.partials, k, S, acc_gap, acc_P, a.tau);
}

// A pipelined pass of a.n iterations (tile2d_pipe.h): one block per tile of
// kPipeOwned columns and a.th rows, a.n waves (and one for the gap).
template <bool GAP>
__global__ __launch_bounds__(kPipeMaxThreads) void sweep2d_pipe_kernel(
    Sweep2DArgs a) {
  extern __shared__ __attribute__((aligned(16))) float pipe_lds[];
  DevState* st = a.st;
  const int k = st->k;
  const int n = a.n;
  if (st->converged || k + n > st->k_end) return;
  const float tau_prev = st->tau_prev;
  const int slot = st->slot;
  // contiguous runs of tiles per XCD, as in the walk
  const int nb = gridDim.x, b = blockIdx.x;
  const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
  const int bt = xcd * q8 + min(xcd, r8) + (b >> 3);
  const int ty = bt / a.ntx, tx = bt - ty * a.ntx;
  PipeCtx c;
  const int64_t PL = a.plane;
  c.F = a.base + plain_f(slot) * PL;
  c.FN = a.base + plain_f(slot ^ 1) * PL;
  c.PX = a.base + plain_p(slot) * PL;
  c.PY = c.PX + PL;
  c.QX = a.base + plain_p(slot ^ 1) * PL;
  c.QY = c.QX + PL;
  c.G = a.base + kPlainG * PL;
  c.ny = a.ny;
  c.nx = a.nx;
  c.pitch = a.pitch;
  c.x0 = tx * kPipeOwned;
  c.y0 = ty * a.th;
  c.y1 = min(c.y0 + a.th, a.ny);
  c.n = n;
  c.lam = a.lam;
  c.tau = a.tau;
  c.sig = a.sigma;
  c.th = a.theta;
  c.tau_prev = tau_prev;
  c.err = &st->flags;
  c.wait_limit = a.wait_limit;
  double acc_gap = 0.0, acc_P = 0.0;
  sweep_tile_pipe<GAP>(c, pipe_lds, acc_gap, acc_P);
  finish_sweep<GAP>(st, a.partials, k, n, acc_gap, acc_P, a.tau);
}

// A plain copy of n floats (n a multiple of 4) with 16-byte accesses, the
// reference transfer for byte counters.
__global__ __launch_bounds__(256) void tvpd_copy_kernel(const float4* __restrict__ src,
                                                        float4* __restrict__ dst,
                                                        int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void init2d_kernel(float* base, int64_t plane, int ny, int nx,
                              int pitch, const float* __restrict__ g,
                              DevState* st) {
  const int64_t n = (int64_t)ny * pitch;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / pitch);
    const int x = (int)(i - (int64_t)y * pitch);
    const float v = (x < nx) ? g[(int64_t)y * nx + x] : 0.0f;
    for (int s = 0; s < kPlainPlanes2D; ++s) base[s * plane + i] = 0.0f;
    base[plain_f(0) * plane + i] = v;   // f^0 (f^{-1} = f^0 is implied)
    base[kPlainG * plane + i] = v;      // g (p^0 = 0)
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

__global__ void set_params_kernel(DevState* st, int32_t k_end, double tol) {
  st->k_end = k_end;
  st->tol = tol;
  st->converged = 0;
  SyncArea* sa =
      reinterpret_cast<SyncArea*>(reinterpret_cast<char*>(st) + kSyncOffset);
  for (int i = 0; i < kSyncGroups; ++i) sa->sub[i].v = 0;
  sa->top.v = 0;
}

__global__ void read2d_kernel(const float* base, int64_t plane, int ny,
                              int nx, int pitch, const DevState* st,
                              float* f_out, float* p_out) {
  const int slot = st->slot;
  const float* f = base + plain_f(slot) * plane;
  const float* px = base + plain_p(slot) * plane;
  const float* py = px + plane;
  const int64_t n = (int64_t)ny * nx;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / nx);
    const int x = (int)(i - (int64_t)y * nx);
    const int64_t s = (int64_t)y * pitch + x;
    f_out[i] = f[s];
    if (p_out) {
      p_out[i] = px[s];
      p_out[n + i] = py[s];
    }
  }
}

// Gap density and primal energy of the current pair, one pixel per thread
// (neighbours read directly; used outside the iteration loop only).
__global__ __launch_bounds__(kMaxBlock) void energy2d_kernel(
    const float* base, int64_t plane, int ny, int nx, int pitch, float lam,
    const DevState* st, double* partials, int skip_if_converged) {
  if (skip_if_converged && st->converged) return;
  __shared__ double red[2][kMaxBlock / kWave];
  const int slot = st->slot;
  const float* f = base + plain_f(slot) * plane;
  const float* px = base + plain_p(slot) * plane;
  const float* py = px + plane;
  const float* g = base + kPlainG * plane;
  const int64_t n = (int64_t)ny * nx;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sg = 0.0, sp = 0.0;
  if (i < n) {
    const int y = (int)(i / nx);
    const int x = (int)(i - (int64_t)y * nx);
    const int64_t s = (int64_t)y * pitch + x;
    const double fv = f[s];
    const double gx = (x < nx - 1) ? (double)f[s + 1] - fv : 0.0;
    const double gy = (y < ny - 1) ? (double)f[s + pitch] - fv : 0.0;
    const double dxl = (x > 0) ? (double)px[s - 1] : 0.0;
    const double dyl = (y > 0) ? (double)py[s - pitch] : 0.0;
    const double d = ((double)px[s] - dxl) + ((double)py[s] - dyl);
    const double e = fv - (double)g[s];
    const double r = e - d;
    const double nrm = sqrt(gx * gx + gy * gy);
    sg = 0.5 * r * r + (double)lam * nrm - (gx * px[s] + gy * py[s]);
    sp = 0.5 * e * e + (double)lam * nrm;
  }
  block_sum2(sg, sp, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sg;
    partials[2 * blockIdx.x + 1] = sp;
  }
}

__global__ __launch_bounds__(kMaxBlock) void energy_final_kernel(
    DevState* st, const double* partials, int nparts, int skip_if_converged) {
  if (skip_if_converged && st->converged) return;
  __shared__ double red[2][kMaxBlock / kWave];
  double sg = 0.0, sp = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    sg += partials[2 * i];
    sp += partials[2 * i + 1];
  }
  block_sum2(sg, sp, red);
  if (threadIdx.x == 0) {
    st->gap = sg;
    st->P = sp;
    st->D = sp - sg;
  }
}

}  // namespace


hipError_t launch_init2d(const Layout& L, const float* g, void* ws,
                         hipStream_t s) {
  hipLaunchKernelGGL(init2d_kernel, dim3(grid_for((int64_t)L.ny * L.pitch, 256)),
                     dim3(256), 0, s, planes_of(L, ws), L.plane, L.ny, L.nx,
                     L.pitch, g, state_of(ws));
  return hipGetLastError();
}

hipError_t launch_stream_copy(const float* src, float* dst, int64_t n,
                              hipStream_t s) {
  const int64_t n4 = n / 4;
  const int64_t blocks = std::min<int64_t>((n4 + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(tvpd_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst), n4);
  return hipGetLastError();
}

hipError_t launch_set_params(void* ws, int32_t k_end, double tol,
                             hipStream_t s) {
  hipLaunchKernelGGL(set_params_kernel, dim3(1), dim3(1), 0, s, state_of(ws),
                     k_end, tol);
  return hipGetLastError();
}

// LDS beyond the default dynamic limit, requested for both instances of the
// pipelined kernel once per device (a function attribute is per device).
static hipError_t pipe_lds_ready() {
  constexpr int kMaxDevices = 64;
  static std::atomic<int> done[kMaxDevices];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const bool known = dev >= 0 && dev < kMaxDevices;
  if (known && done[dev].load(std::memory_order_acquire)) return hipSuccess;
  const int bytes = pipe_lds_floats(kPipeMaxPass) * (int)sizeof(float);
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(sweep2d_pipe_kernel<true>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(sweep2d_pipe_kernel<false>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  if (known) done[dev].store(1, std::memory_order_release);
  return hipSuccess;
}

static hipError_t launch_sweep2d_pipe(const Layout& L, const Tile2D& t,
                                      const tvpd_coeffs& c, bool with_gap, int n,
                                      void* ws, hipStream_t s) {
  if (n < 1 || n > kPipeMaxPass || t.th < 1) return hipErrorInvalidValue;
  if (n == 1) {
    // a one-iteration pass has nothing to pipeline: the walk computes the
    // same iterate
    Tile2D wt;
    wt.th = 16;
    wt.wpb = 4;
    wt.order = 0;
    return launch_sweep2d(L, wt, c, with_gap, 1, ws, s);
  }
  const hipError_t attr = pipe_lds_ready();
  if (attr != hipSuccess) return attr;
  Sweep2DArgs a;
  a.base = planes_of(L, ws);
  a.plane = L.plane;
  a.ny = L.ny;
  a.nx = L.nx;
  a.pitch = L.pitch;
  a.th = t.th;
  a.wpb = 0;
  a.order = kOrderPipe;
  a.wait_limit = pipe_wait_limit();
  a.ntx = (L.nx + kPipeOwned - 1) / kPipeOwned;
  a.nty = (L.ny + t.th - 1) / t.th;
  a.ntiles = a.ntx * a.nty;
  a.n = n;
  a.lam = c.lam;
  a.tau = c.tau;
  a.sigma = c.sigma;
  a.theta = c.theta;
  a.st = state_of(ws);
  a.partials = partials_of(L, ws);
  if (a.ntiles > L.max_partials) return hipErrorInvalidValue;
  const dim3 grid(a.ntiles), block((n + (with_gap ? 1 : 0)) * kWave);
  const size_t lds = (size_t)pipe_lds_floats(n) * sizeof(float);
  if (with_gap)
    hipLaunchKernelGGL((sweep2d_pipe_kernel<true>), grid, block, lds, s, a);
  else
    hipLaunchKernelGGL((sweep2d_pipe_kernel<false>), grid, block, lds, s, a);
  return hipGetLastError();
}

hipError_t launch_sweep2d(const Layout& L, const Tile2D& t,
                          const tvpd_coeffs& c, bool with_gap, int n,
                          void* ws, hipStream_t s) {
  if (t.order == kOrderPipe) return launch_sweep2d_pipe(L, t, c, with_gap, n, ws, s);
  if (n < 1 || n > kMaxPass) return hipErrorInvalidValue;
  Sweep2DArgs a;
  a.base = planes_of(L, ws);
  a.plane = L.plane;
  a.ny = L.ny;
  a.nx = L.nx;
  a.pitch = L.pitch;
  a.th = t.th;
  a.wpb = t.wpb;
  a.order = t.order;
  a.n = n;
  a.wait_limit = 0;  // (the walk has no waits)
  // every pass runs on overlapping strips of xs_owned(n) owned columns
  const int strip = xs_owned(n);
  a.ntx = (L.nx + strip - 1) / strip;
  a.nty = (L.ny + t.th - 1) / t.th;
  a.ntiles = a.ntx * a.nty;
  a.lam = c.lam;
  a.tau = c.tau;
  a.sigma = c.sigma;
  a.theta = c.theta;
  a.st = state_of(ws);
  a.partials = partials_of(L, ws);
  const int nb = (a.ntiles + t.wpb - 1) / t.wpb;
  if (nb > L.max_partials) return hipErrorInvalidValue;
  const dim3 grid(nb), block(t.wpb * kWave);
  if (with_gap) {
    switch (n) {
      case 1: hipLaunchKernelGGL((sweep2d_xs_kernel<1, true>), grid, block, 0, s, a); break;
      case 2: hipLaunchKernelGGL((sweep2d_xs_kernel<2, true>), grid, block, 0, s, a); break;
      case 3: hipLaunchKernelGGL((sweep2d_xs_kernel<3, true>), grid, block, 0, s, a); break;
      case 4: hipLaunchKernelGGL((sweep2d_xs_kernel<4, true>), grid, block, 0, s, a); break;
      case 5: hipLaunchKernelGGL((sweep2d_xs_kernel<5, true>), grid, block, 0, s, a); break;
      default: hipLaunchKernelGGL((sweep2d_xs_kernel<6, true>), grid, block, 0, s, a); break;
    }
  } else {
    switch (n) {
      case 1: hipLaunchKernelGGL((sweep2d_xs_kernel<1, false>), grid, block, 0, s, a); break;
      case 2: hipLaunchKernelGGL((sweep2d_xs_kernel<2, false>), grid, block, 0, s, a); break;
      case 3: hipLaunchKernelGGL((sweep2d_xs_kernel<3, false>), grid, block, 0, s, a); break;
      case 4: hipLaunchKernelGGL((sweep2d_xs_kernel<4, false>), grid, block, 0, s, a); break;
      case 5: hipLaunchKernelGGL((sweep2d_xs_kernel<5, false>), grid, block, 0, s, a); break;
      default: hipLaunchKernelGGL((sweep2d_xs_kernel<6, false>), grid, block, 0, s, a); break;
    }
  }
  return hipGetLastError();
}

int sweep2d_blocks(const Layout& L, const Tile2D& t, int n) {
  if (t.order == kOrderPipe)
    return ((L.nx + kPipeOwned - 1) / kPipeOwned) * ((L.ny + t.th - 1) / t.th);
  const int strip = xs_owned(n);
  const int ntx = (L.nx + strip - 1) / strip;
  const int nty = (L.ny + t.th - 1) / t.th;
  const int nt = ntx * nty;
  return (nt + t.wpb - 1) / t.wpb;
}

hipError_t launch_read2d(const Layout& L, const void* ws, float* f_out,
                         float* p_out, hipStream_t s) {
  void* w = const_cast<void*>(ws);
  hipLaunchKernelGGL(read2d_kernel, dim3(grid_for((int64_t)L.ny * L.nx, 256)),
                     dim3(256), 0, s, planes_of(L, w), L.plane, L.ny, L.nx,
                     L.pitch, state_of(w), f_out, p_out);
  return hipGetLastError();
}

hipError_t launch_energy_final(const Layout& L, void* ws, int nparts,
                               bool skip_if_converged, hipStream_t s) {
  hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(kMaxBlock), 0, s,
                     state_of(ws), partials_of(L, ws), nparts,
                     skip_if_converged ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_energy2d(const Layout& L, float lam, void* ws,
                           bool skip_if_converged, hipStream_t s) {
  const int64_t n = (int64_t)L.ny * L.nx;
  const int nb = (int)((n + kMaxBlock - 1) / kMaxBlock);
  if (nb > L.max_partials) return hipErrorInvalidValue;
  hipLaunchKernelGGL(energy2d_kernel, dim3(nb), dim3(kMaxBlock), 0, s,
                     planes_of(L, ws), L.plane, L.ny, L.nx, L.pitch, lam,
                     state_of(ws), partials_of(L, ws), skip_if_converged ? 1 : 0);
  hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(kMaxBlock), 0, s,
                     state_of(ws), partials_of(L, ws), nb,
                     skip_if_converged ? 1 : 0);
  return hipGetLastError();
}

}  // namespace tvpd
