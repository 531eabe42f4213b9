// C ABI of the tomographic data term: argument checks, workspace layout and
// the host side of the iteration (see include/tvpd.h for the semantics).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>

#include "tomo.h"

namespace tvpd {

TomoLayout tomo_layout(int ny, int nx, int na, int nd) {
  TomoLayout L;
  L.ny = ny;
  L.nx = nx;
  L.na = na;
  L.nd = nd;
  L.pitch_b = (int)round_up(nx + 2 * kTomoPad, 64);
  L.pitch_t = (int)round_up(ny + 2 * kTomoPad, 64);
  L.img = round_up((int64_t)ny * nx, 64);
  L.sino = round_up((int64_t)na * nd, 64);
  L.fb = round_up((int64_t)ny * L.pitch_b, 64);
  L.fbt = round_up((int64_t)nx * L.pitch_t, 64);
  const int64_t nproj = tomo_project_blocks(na, nd);
  const int64_t nreg = tomo_regsum_blocks(ny, nx);
  const int64_t ndot = tomo_dot_blocks((int64_t)ny * nx);
  L.max_partials = nproj + (nreg > ndot ? nreg : ndot) + 1;
  L.off_trig = kHeaderBytes;
  L.off_part = (size_t)round_up((int64_t)L.off_trig + 16 * (int64_t)na, (int64_t)kAlign);
  L.off_fbp = (size_t)round_up((int64_t)L.off_part + 16 * L.max_partials, (int64_t)kAlign);
  // FBP filter region: the taps (4 nd bytes) or the FFT twiddles (8 L bytes)
  const int64_t fbp_bytes = std::max<int64_t>(4 * (int64_t)nd, 8 * (int64_t)tomo_fbp_length(nd));
  L.off_planes = (size_t)round_up((int64_t)L.off_fbp + fbp_bytes, (int64_t)kAlign);
  L.bytes = L.off_planes +
            sizeof(float) * (size_t)(kTNumImg * L.img + kTNumSino * L.sino + L.fb + L.fbt);
  return L;
}

TomoPtrs tomo_ptrs(const TomoLayout& L, void* ws) {
  char* base = static_cast<char*>(ws);
  TomoPtrs p;
  p.st = reinterpret_cast<TomoState*>(base);
  p.trig = reinterpret_cast<double*>(base + L.off_trig);
  p.part = reinterpret_cast<double*>(base + L.off_part);
  p.fbp = reinterpret_cast<float*>(base + L.off_fbp);
  float* f = reinterpret_cast<float*>(base + L.off_planes);
  for (int i = 0; i < kTNumImg; ++i, f += L.img) p.img[i] = f;
  for (int i = 0; i < kTNumSino; ++i, f += L.sino) p.sino[i] = f;
  p.fb = f;
  p.fbt = f + L.fb;
  return p;
}

namespace {

#define TOMO_TRY(call)                    \
  do {                                    \
    const int st_ = (call);               \
    if (st_ != TVPD_OK) return st_;       \
  } while (0)

bool geom_ok(const tvpd_tomo_geom* g) {
  if (!g) return false;
  return g->ny >= 1 && g->nx >= 1 && g->n_angles >= 1 && g->n_det >= 1 &&
         g->ny <= kTomoMaxSide && g->nx <= kTomoMaxSide && g->n_det <= kTomoMaxSide &&
         g->n_angles <= kTomoMaxAngles;
}

int check_ws(const TomoLayout& L, const void* ws, size_t bytes) {
  if (!ws) return TVPD_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return TVPD_ERR_ALIGNMENT;
  if (bytes < L.bytes) return TVPD_ERR_WORKSPACE;
  return TVPD_OK;
}

int params_ok(const tvpd_tomo_params* p) {
  if (!p) return TVPD_ERR_INVALID_ARG;
  if (p->reg != TVPD_REG_TV && p->reg != TVPD_REG_TIKHONOV) return TVPD_ERR_INVALID_ARG;
  if (!(p->lam >= 0.0f) || !std::isfinite(p->lam)) return TVPD_ERR_INVALID_ARG;
  if (!(p->theta >= 0.0f && p->theta <= 1.0f)) return TVPD_ERR_INVALID_ARG;
  if (!(p->tau > 0.0f) || !std::isfinite(p->tau) || !(p->sigma_r > 0.0f) ||
      !std::isfinite(p->sigma_r))
    return TVPD_ERR_STEP;
  if (p->reg == TVPD_REG_TV && (!(p->sigma_p > 0.0f) || !std::isfinite(p->sigma_p)))
    return TVPD_ERR_STEP;
  return TVPD_OK;
}

// Staging of image rows in LDS by the projection (tvpd_set_projection_staging).
std::atomic<int> g_proj_staged{1};

ProjArgs proj_args(const TomoLayout& L, const TomoPtrs& P) {
  ProjArgs a{};
  a.staged = g_proj_staged.load();
  a.fb = P.fb;
  a.fbt = P.fbt;
  a.trig = P.trig;
  a.ny = L.ny;
  a.nx = L.nx;
  a.na = L.na;
  a.nd = L.nd;
  a.pitch_b = L.pitch_b;
  a.pitch_t = L.pitch_t;
  return a;
}

BpArgs bp_args(const TomoLayout& L, const TomoPtrs& P, const float* sino) {
  BpArgs a{};
  a.sino = sino;
  a.trig = P.trig;
  a.ny = L.ny;
  a.nx = L.nx;
  a.na = L.na;
  a.nd = L.nd;
  return a;
}

// A x into `sino` (x dense [ny][nx]); uses FB, FBT.
int forward(const TomoLayout& L, const TomoPtrs& P, const float* x, float* sino,
            hipStream_t s) {
  TOMO_TRY(launch_tomo_prep(L, x, x, nullptr, 0.0f, P.fb, P.fbt, nullptr, nullptr,
                            nullptr, nullptr, 0.0f, 0.0f, s));
  ProjArgs a = proj_args(L, P);
  a.out = sino;
  return launch_tomo_project(a, kProjWrite, s);
}

int backward(const TomoLayout& L, const TomoPtrs& P, const float* sino, float* img,
             hipStream_t s) {
  BpArgs a = bp_args(L, P, sino);
  a.out = img;
  return launch_tomo_backproject(a, kBpWrite, nullptr, nullptr, nullptr, nullptr,
                                 nullptr, s);
}

int one_iteration(const TomoLayout& L, const TomoPtrs& P, const float* g,
                  const tvpd_tomo_params& prm, hipStream_t s) {
  const bool tv = prm.reg == TVPD_REG_TV;
  float* const* I = P.img;
  // fbar (padded copies) and, for TV, p^{k+1}
  TOMO_TRY(launch_tomo_prep(L, I[kTF0], I[kTF1], &P.st->k, prm.theta, P.fb, P.fbt,
                            tv ? I[kTPX0] : nullptr, I[kTPY0], I[kTPX1], I[kTPY1],
                            prm.sigma_p, prm.lam, s));
  // r^{k+1} = (r^k + sigma_r (A fbar - g)) / (1 + sigma_r)
  ProjArgs pa = proj_args(L, P);
  pa.out = P.sino[kTR];
  pa.g = g;
  pa.sigma = prm.sigma_r;
  TOMO_TRY(launch_tomo_project(pa, kProjDual, s));
  // f^{k+1} from f^k, A^T r^{k+1} (and div p^{k+1})
  BpArgs ba = bp_args(L, P, P.sino[kTR]);
  ba.out = I[kTF0];
  ba.f = I[kTF0];
  ba.px = I[kTPX0];
  ba.py = I[kTPY0];
  ba.tau = prm.tau;
  ba.lam = prm.lam;
  TOMO_TRY(launch_tomo_backproject(ba, tv ? kBpTV : kBpTikhonov, &P.st->k, I[kTF1],
                                   I[kTF1], I[kTPX1], I[kTPY1], s));
  return launch_tomo_advance(P.st, s);
}

// Static scratch of tvpd_fbp_noalloc: the angle table (double2 per angle,
// room for kTomoMaxAngles), the filter taps (room for kTomoMaxSide) and the
// filtered sinogram (what is left of kNoAllocBytes).  Each device holds its
// own copy for the life of the process; every call on a device shares it.
constexpr size_t kNoAllocBytes = size_t(32) << 20;
constexpr size_t kNoAllocTrigOff = 0;
constexpr size_t kNoAllocTapOff = 65536 * 16;
constexpr size_t kNoAllocSinoOff = kNoAllocTapOff + 4 * size_t(kTomoMaxSide);
constexpr size_t kNoAllocSinoFloats = (kNoAllocBytes - kNoAllocSinoOff) / 4;
static_assert(16 * size_t(kTomoMaxAngles) <= kNoAllocTapOff, "angle table");
static_assert(8 * size_t(kFbpFftMaxLen) <= 4 * size_t(kTomoMaxSide), "FBP twiddles");
static_assert(kNoAllocSinoOff % 256 == 0, "sinogram alignment");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` on each device, looked up once per device
// with that device current (the symbol's host-side name is not a device
// address).
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TVPD_ERR_HIP;
  if (dev < 0 || dev >= kNoAllocMaxDevices) return TVPD_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return TVPD_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TVPD_OK;
}

// The regularised FBP's filtering into P.sino[kTS], with the factor dtheta
// of the backprojection: through the FFT for padded lengths up to
// kFbpFftMaxLen (P.fbp holds the twiddles), else a direct convolution with
// float64 taps (P.fbp holds the taps).
int fbp_filter(const TomoLayout& L, const float* g, const TomoPtrs& P, float lam,
               hipStream_t s) {
  const float dtheta = (float)(M_PI / (double)L.na);
  if (tomo_fbp_length(L.nd) <= kFbpFftMaxLen)
    return launch_fbp_fft_filter(g, P.sino[kTS], reinterpret_cast<float2*>(P.fbp), L.na, L.nd,
                                 lam, dtheta, s);
  TOMO_TRY(launch_tomo_fbp_taps(P.fbp, L.nd, lam, s));
  return launch_tomo_fbp_filter(g, P.sino[kTS], P.fbp, L.na, L.nd, dtheta, s);
}

}  // namespace
}  // namespace tvpd

using namespace tvpd;

extern "C" {

int tvpd_set_projection_staging(int32_t on) {
  if (on != 0 && on != 1) return TVPD_ERR_INVALID_ARG;
  g_proj_staged.store(on);
  return TVPD_OK;
}

int tvpd_tomo_workspace_size(const tvpd_tomo_geom* geom, size_t* bytes) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!bytes) return TVPD_ERR_INVALID_ARG;
  *bytes = tomo_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det).bytes;
  return TVPD_OK;
}

int tvpd_radon_forward(const tvpd_tomo_geom* geom, const float* f, float* sino,
                       void* ws, size_t ws_bytes, void* stream) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!f || !sino) return TVPD_ERR_INVALID_ARG;
  const TomoLayout L = tomo_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  TOMO_TRY(check_ws(L, ws, ws_bytes));
  const TomoPtrs P = tomo_ptrs(L, ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  TOMO_TRY(launch_tomo_trig(P.trig, L.na, s));
  return forward(L, P, f, sino, s);
}

int tvpd_radon_backward(const tvpd_tomo_geom* geom, const float* sino, float* img,
                        void* ws, size_t ws_bytes, void* stream) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!sino || !img) return TVPD_ERR_INVALID_ARG;
  const TomoLayout L = tomo_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  TOMO_TRY(check_ws(L, ws, ws_bytes));
  const TomoPtrs P = tomo_ptrs(L, ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  TOMO_TRY(launch_tomo_trig(P.trig, L.na, s));
  return backward(L, P, sino, img, s);
}

int tvpd_tomo_init(const tvpd_tomo_geom* geom, const float* f0, void* ws,
                   size_t ws_bytes, void* stream) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  const TomoLayout L = tomo_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  TOMO_TRY(check_ws(L, ws, ws_bytes));
  const TomoPtrs P = tomo_ptrs(L, ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = (int64_t)L.ny * L.nx;
  TOMO_TRY(launch_tomo_trig(P.trig, L.na, s));
  TOMO_TRY(launch_tomo_set_k(P.st, 0, s));
  if (f0) {
    if (hipMemcpyAsync(P.img[kTF0], f0, n * sizeof(float), hipMemcpyDeviceToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(P.img[kTF1], f0, n * sizeof(float), hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
      return TVPD_ERR_HIP;
  } else {
    TOMO_TRY(launch_tomo_fill(P.img[kTF0], n, 0.0f, s));
    TOMO_TRY(launch_tomo_fill(P.img[kTF1], n, 0.0f, s));
  }
  TOMO_TRY(launch_tomo_fill(P.img[kTPX0], n, 0.0f, s));
  TOMO_TRY(launch_tomo_fill(P.img[kTPY0], n, 0.0f, s));
  return launch_tomo_fill(P.sino[kTR], (int64_t)L.na * L.nd, 0.0f, s);
}

int tvpd_tomo_step(const tvpd_tomo_geom* geom, const float* g,
                   const tvpd_tomo_params* prm, int32_t n_iter, void* ws,
                   size_t ws_bytes, void* stream) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!g || n_iter < 0) return TVPD_ERR_INVALID_ARG;
  TOMO_TRY(params_ok(prm));
  const TomoLayout L = tomo_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  TOMO_TRY(check_ws(L, ws, ws_bytes));
  const TomoPtrs P = tomo_ptrs(L, ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int it = 0; it < n_iter; ++it) TOMO_TRY(one_iteration(L, P, g, *prm, s));
  return TVPD_OK;
}

int tvpd_tomo_read(const tvpd_tomo_geom* geom, const void* ws, size_t ws_bytes,
                   float* f, float* r, float* p, int32_t* k, void* stream) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  const TomoLayout L = tomo_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  TOMO_TRY(check_ws(L, ws, ws_bytes));
  const TomoPtrs P = tomo_ptrs(L, const_cast<void*>(ws));
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the slot of f^k and p^k depends on k: read it first (synchronises)
  int32_t kh = 0;
  if (hipMemcpyAsync(&kh, &P.st->k, sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return TVPD_ERR_HIP;
  const int par = kh & 1;
  const size_t nb = (size_t)L.ny * L.nx * sizeof(float);
  if (f && hipMemcpyAsync(f, P.img[par ? kTF1 : kTF0], nb, hipMemcpyDeviceToDevice, s) !=
               hipSuccess)
    return TVPD_ERR_HIP;
  if (r && hipMemcpyAsync(r, P.sino[kTR], (size_t)L.na * L.nd * sizeof(float),
                          hipMemcpyDeviceToDevice, s) != hipSuccess)
    return TVPD_ERR_HIP;
  if (p) {
    if (hipMemcpyAsync(p, P.img[par ? kTPX1 : kTPX0], nb, hipMemcpyDeviceToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(reinterpret_cast<char*>(p) + nb, P.img[par ? kTPY1 : kTPY0], nb,
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
      return TVPD_ERR_HIP;
  }
  if (k) *k = kh;
  return TVPD_OK;
}

int tvpd_tomo_energy(const tvpd_tomo_geom* geom, const float* g, float lam,
                     int32_t reg, void* ws, size_t ws_bytes, double* out,
                     void* stream) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!g || !out || (reg != TVPD_REG_TV && reg != TVPD_REG_TIKHONOV) || !(lam >= 0.0f) ||
      !std::isfinite(lam))
    return TVPD_ERR_INVALID_ARG;
  const TomoLayout L = tomo_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  TOMO_TRY(check_ws(L, ws, ws_bytes));
  const TomoPtrs P = tomo_ptrs(L, ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  TOMO_TRY(launch_tomo_trig(P.trig, L.na, s));
  // the slot of f^k depends on k (synchronises)
  int32_t kh = 0;
  if (hipMemcpyAsync(&kh, &P.st->k, sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return TVPD_ERR_HIP;
  const float* fk = P.img[(kh & 1) ? kTF1 : kTF0];
  TOMO_TRY(launch_tomo_prep(L, fk, fk, nullptr, 0.0f, P.fb, P.fbt, nullptr, nullptr,
                            nullptr, nullptr, 0.0f, 0.0f, s));
  ProjArgs pa = proj_args(L, P);
  pa.g = g;
  pa.part = P.part;
  TOMO_TRY(launch_tomo_project(pa, kProjResid, s));
  const int64_t nproj = tomo_project_blocks(L.na, L.nd);
  TOMO_TRY(launch_tomo_reduce(P.part, 0, nproj, &P.st->red[0], nullptr, s));
  TOMO_TRY(launch_tomo_regsum(fk, L.ny, L.nx, reg == TVPD_REG_TV ? 0 : 1,
                              P.part + 2 * nproj, s));
  TOMO_TRY(launch_tomo_reduce(P.part, nproj, tomo_regsum_blocks(L.ny, L.nx),
                              &P.st->red[1], nullptr, s));
  double red[2];
  if (hipMemcpyAsync(red, P.st->red, sizeof(red), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return TVPD_ERR_HIP;
  const double data = 0.5 * red[0];
  const double regv = (reg == TVPD_REG_TV ? (double)lam : 0.5 * (double)lam) * red[1];
  out[0] = data;
  out[1] = regv;
  out[2] = data + regv;
  return TVPD_OK;
}

int tvpd_tomo_opnorm(const tvpd_tomo_geom* geom, int32_t iters, void* ws,
                     size_t ws_bytes, double* out, void* stream) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!out || iters < 1) return TVPD_ERR_INVALID_ARG;
  const TomoLayout L = tomo_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  TOMO_TRY(check_ws(L, ws, ws_bytes));
  const TomoPtrs P = tomo_ptrs(L, ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = (int64_t)L.ny * L.nx;
  float* v = P.img[kTV];
  float* w = P.img[kTW];
  TOMO_TRY(launch_tomo_trig(P.trig, L.na, s));
  TOMO_TRY(launch_tomo_fill(v, n, (float)(1.0 / std::sqrt((double)n)), s));
  for (int it = 0; it < iters; ++it) {
    TOMO_TRY(forward(L, P, v, P.sino[kTS], s));
    TOMO_TRY(backward(L, P, P.sino[kTS], w, s));
    TOMO_TRY(launch_tomo_dot(v, w, n, P.part, s));
    TOMO_TRY(launch_tomo_reduce(P.part, 0, tomo_dot_blocks(n), &P.st->red[2],
                                &P.st->red[3], s));
    TOMO_TRY(launch_tomo_scale(v, w, n, &P.st->red[3], s));
  }
  double est = 0.0;
  if (hipMemcpyAsync(&est, &P.st->red[2], sizeof(double), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return TVPD_ERR_HIP;
  *out = est;
  return TVPD_OK;
}

int tvpd_fbp(const tvpd_tomo_geom* geom, const float* g, float lam, float* f_out,
             void* ws, size_t ws_bytes, void* stream) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!g || !f_out || !(lam >= 0.0f) || !std::isfinite(lam)) return TVPD_ERR_INVALID_ARG;
  const TomoLayout L = tomo_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  TOMO_TRY(check_ws(L, ws, ws_bytes));
  const TomoPtrs P = tomo_ptrs(L, ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  TOMO_TRY(launch_tomo_trig(P.trig, L.na, s));
  TOMO_TRY(fbp_filter(L, g, P, lam, s));
  return backward(L, P, P.sino[kTS], f_out, s);
}

int tvpd_fbp_noalloc(const tvpd_tomo_geom* geom, const float* g, float lam,
                     float* f_out, void* stream) {
  if (!geom_ok(geom)) return TVPD_ERR_SHAPE;
  if (!g || !f_out || !(lam >= 0.0f) || !std::isfinite(lam)) return TVPD_ERR_INVALID_ARG;
  if ((int64_t)geom->n_angles * geom->n_det > (int64_t)kNoAllocSinoFloats)
    return TVPD_ERR_SCRATCH;
  void* base = nullptr;
  TOMO_TRY(scratch_address(&base));
  char* b = static_cast<char*>(base);
  const TomoLayout L = tomo_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  TomoPtrs P{};
  P.trig = reinterpret_cast<double*>(b + kNoAllocTrigOff);
  P.fbp = reinterpret_cast<float*>(b + kNoAllocTapOff);
  P.sino[kTS] = reinterpret_cast<float*>(b + kNoAllocSinoOff);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // every scratch word the kernels read is written first in this call: no
  // clearing is needed
  TOMO_TRY(launch_tomo_trig(P.trig, L.na, s));
  TOMO_TRY(fbp_filter(L, g, P, lam, s));
  return backward(L, P, P.sino[kTS], f_out, s);
}

int tvpd_tomo_solve(const tvpd_tomo_geom* geom, const float* g,
                    const tvpd_tomo_params* prm, int32_t n_iter, float* f_out,
                    void* ws, size_t ws_bytes, void* stream) {
  if (!f_out) return TVPD_ERR_INVALID_ARG;
  TOMO_TRY(params_ok(prm));
  TOMO_TRY(tvpd_tomo_init(geom, nullptr, ws, ws_bytes, stream));
  TOMO_TRY(tvpd_tomo_step(geom, g, prm, n_iter, ws, ws_bytes, stream));
  // after n_iter iterations from k = 0, f^n sits in slot n & 1
  const TomoLayout L = tomo_layout(geom->ny, geom->nx, geom->n_angles, geom->n_det);
  const TomoPtrs P = tomo_ptrs(L, ws);
  if (hipMemcpyAsync(f_out, P.img[(n_iter & 1) ? kTF1 : kTF0],
                     (size_t)L.ny * L.nx * sizeof(float), hipMemcpyDeviceToDevice,
                     static_cast<hipStream_t>(stream)) != hipSuccess)
    return TVPD_ERR_HIP;
  return TVPD_OK;
}

}  // extern "C"
