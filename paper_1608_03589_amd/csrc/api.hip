// C ABI of the primal-dual sweep library: argument checks, workspace
// layout, and the host side of the iteration loop.
#include <climits>
#include <cmath>
#include <cstring>
#include <atomic>
#include <mutex>

#include "common.h"

namespace tvpd {
namespace {

constexpr int kVersion = 10000;  // 1.0.0

// Floats added to every plane so that consecutive planes do not start at
// the same offset modulo large powers of two (a multiple of 64).
#ifndef TVPD_PLANE_PAD
#define TVPD_PLANE_PAD 0
#endif

bool shape_ok(const tvpd_shape* s) {
  if (!s) return false;
  if (s->ndim == 2) {
    if (s->nz != 1) return false;
  } else if (s->ndim == 3) {
    if (s->nz < 1) return false;
  } else {
    return false;
  }
  if (s->ny < 1 || s->nx < 1) return false;
  // every index fits in int32 along an axis; planes are addressed in int64
  return s->nx <= (INT_MAX - 1024) && s->ny <= (INT_MAX - 1024);
}

// ||grad||^2 on the grid: the largest eigenvalue of the Neumann Laplacian,
// a sum over axes of 4 sin^2(pi (n-1) / (2n)).
double grad_norm2(const tvpd_shape& s) {
  auto term = [](int n) {
    const double a = std::sin(M_PI * (n - 1) / (2.0 * n));
    return 4.0 * a * a;
  };
  double v = term(s.nx) + term(s.ny);
  if (s.ndim == 3) v += term(s.nz);
  return v;
}

int coeffs_ok(const tvpd_shape& s, const tvpd_coeffs* c) {
  if (!c) return TVPD_ERR_INVALID_ARG;
  if (!(c->lam >= 0.0f) || !std::isfinite(c->lam)) return TVPD_ERR_INVALID_ARG;
  if (!(c->theta >= 0.0f && c->theta <= 1.0f)) return TVPD_ERR_INVALID_ARG;
  if (!(c->tau > 0.0f) || !(c->sigma > 0.0f) || !std::isfinite(c->tau) ||
      !std::isfinite(c->sigma))
    return TVPD_ERR_STEP;
  if ((double)c->tau * (double)c->sigma * grad_norm2(s) >= 1.0)
    return TVPD_ERR_STEP;
  return TVPD_OK;
}

Layout make_layout(const tvpd_shape& s) {
  Layout L;
  L.ndim = s.ndim;
  L.nz = s.nz;
  L.ny = s.ny;
  L.nx = s.nx;
  L.pitch = (int)round_up(s.nx, kColsPerLane);
  L.plane = round_up((int64_t)s.nz * s.ny * L.pitch, 64) + TVPD_PLANE_PAD;
  L.nplanes = s.ndim == 2 ? kPlainPlanes2D : kPlainPlanes3D;
  // enough reduction slots for one block per (strip, row) and for the
  // one-pixel-per-thread energy kernel
  // (the deepest passes own the narrowest strips)
  const int64_t ntx = (s.nx + kXsOwnedMin - 1) / kXsOwnedMin;
  const int64_t a = ntx * (int64_t)s.ny * s.nz;
  const int64_t b = ((int64_t)s.nz * s.ny * s.nx + kMaxBlock - 1) / kMaxBlock;
  L.max_partials = (a > b ? a : b) + 1;
  L.partial_off = kHeaderBytes;
  L.plane_off = (size_t)round_up((int64_t)L.partial_off + L.max_partials * 16,
                                 (int64_t)kAlign);
  L.bytes = L.plane_off + (size_t)L.nplanes * (size_t)L.plane * sizeof(float);
  return L;
}

int ws_ok(const Layout& L, const void* ws, size_t bytes) {
  if (!ws) return TVPD_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return TVPD_ERR_ALIGNMENT;
  if (bytes < L.bytes) return TVPD_ERR_WORKSPACE;
  return TVPD_OK;
}

// Per-thread host resources for polling the device convergence flag while
// the next chunk of iterations is already queued.
thread_local HostPoll t_poll;

}  // namespace

void host_poll_release(HostPoll& p) {
  int cur = -1;
  const bool switch_dev = p.device >= 0 && hipGetDevice(&cur) == hipSuccess &&
                          cur != p.device &&
                          hipSetDevice(p.device) == hipSuccess;
  if (p.capture) (void)hipStreamDestroy(p.capture);
  for (int i = 0; i < 2; ++i)
    if (p.ev[i]) (void)hipEventDestroy(p.ev[i]);
  if (p.host) (void)hipHostFree(p.host);
  if (switch_dev) (void)hipSetDevice(cur);
  p = HostPoll{};
}

int host_poll_get(HostPoll& p, size_t host_bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TVPD_ERR_HIP;
  if (p.ok && p.device == dev) return TVPD_OK;
  host_poll_release(p);
  p.device = dev;
  bool good = hipHostMalloc(&p.host, host_bytes, hipHostMallocDefault) ==
              hipSuccess;
  for (int i = 0; i < 2 && good; ++i)
    good = hipEventCreateWithFlags(&p.ev[i], hipEventDisableTiming) ==
           hipSuccess;
  good = good && hipStreamCreateWithFlags(&p.capture, hipStreamNonBlocking) ==
                     hipSuccess;
  if (!good) {
    host_poll_release(p);
    return TVPD_ERR_HIP;
  }
  p.ok = true;
  return TVPD_OK;
}

namespace {

#define TVPD_HIP(call)                                    \
  do {                                                    \
    if ((call) != hipSuccess) return TVPD_ERR_HIP;        \
  } while (0)

// Enqueue iterations k_first .. k_first+n-1.  2D: two-iteration passes
// wherever no gap check falls on a pass's second iteration (checks are
// evaluated at the first iteration of a pass only).  3D: one iteration per
// launch.
int enqueue_sweeps(const Layout& L, const tvpd_coeffs& c, int64_t k_first,
                   int n, int check_every, bool blocked, void* ws,
                   hipStream_t s) {
  if (L.ndim == 3) {
    const Tile3D t = tile3d_for(L);
    for (int i = 0; i < n; ++i) {
      const int64_t kk = k_first + i;
      const bool gap = check_every > 0 && (kk % check_every) == 0;
      TVPD_HIP(launch_sweep3d(L, t, c, gap, ws, s));
    }
    return TVPD_OK;
  }
  const Tile2D t = tile2d_for(L);
  const int depth =
      blocked ? (t.order == kOrderPipe ? pipe_depth() : walk_depth()) : 1;
  int i = 0;
  while (i < n) {
    const int64_t kk = k_first + i;
    const bool gap = check_every > 0 && (kk % check_every) == 0;
    int64_t len = std::min<int64_t>(depth, n - i);
    if (check_every > 0) {
      // a check may only fall on the first iteration of a pass
      const int64_t next = (kk / check_every + 1) * check_every;
      len = std::min<int64_t>(len, next - kk);
    }
    TVPD_HIP(launch_sweep2d(L, t, c, gap, (int)len, ws, s));
    i += (int)len;
  }
  return TVPD_OK;
}

hipError_t launch_init(const Layout& L, const float* g, void* ws,
                       hipStream_t s) {
  return L.ndim == 2 ? launch_init2d(L, g, ws, s) : launch_init3d(L, g, ws, s);
}

hipError_t launch_energy(const Layout& L, float lam, void* ws,
                         bool skip_if_converged, hipStream_t s) {
  return L.ndim == 2 ? launch_energy2d(L, lam, ws, skip_if_converged, s)
                     : launch_energy3d(L, lam, ws, skip_if_converged, s);
}

hipError_t launch_read(const Layout& L, const void* ws, float* f_out,
                       float* p_out, hipStream_t s) {
  return L.ndim == 2 ? launch_read2d(L, ws, f_out, p_out, s)
                     : launch_read3d(L, ws, f_out, p_out, s);
}

// Longest pass of the temporally blocked 2D sweep, process-wide
// (tvpd_set_pass_depth; 0: each kernel's default, the walk's kWalkDepth and
// the pipelined passes' kPipeMaxPass; tvpd_set_blocking(0) means 1).
constexpr int kWalkDepth = 5;
std::atomic<int> g_depth{0};
// Polls after which a bounded wait inside a pipelined pass gives up
// (tvpd_set_wait_limit; 0: the default, about half a second).
constexpr int64_t kDefaultWaitLimit = 1LL << 24;
std::atomic<int64_t> g_wait_limit{0};

}  // namespace

int64_t pipe_wait_limit() {
  const int64_t v = g_wait_limit.load();
  return v == 0 ? kDefaultWaitLimit : v;
}

int pass_depth() { return g_depth.load(); }
int walk_depth() {
  const int d = g_depth.load();
  return d == 0 ? kWalkDepth : std::min(d, kMaxPass);
}
int pipe_depth() {
  const int d = g_depth.load();
  return d == 0 ? kPipeMaxPass : std::min(d, kPipeMaxPass);
}

namespace {

int solve_plain(const Layout& L, const float* g, float* f_out,
                const tvpd_params& prm, void* ws, tvpd_result* res,
                hipStream_t s) {
  HostPoll* poll = &t_poll;
  int rc = host_poll_get(*poll, 2 * sizeof(DevState));
  if (rc) return rc;
  TVPD_HIP(launch_init(L, g, ws, s));
  TVPD_HIP(launch_set_params(ws, prm.max_iter, prm.gap_tol, s));

  const int ce = prm.check_every;
  const bool can_stop = ce > 0 && prm.gap_tol >= 0.0;
  const bool blocked = pass_depth() != 1;
  // chunk of iterations between host polls: a multiple of check_every
  int chunk = 64;
  if (ce > 0) chunk = ce * ((64 + ce - 1) / ce);
  bool use_graph = prm.use_graph == 1;
  if (prm.use_graph < 0) {
    // graphs pay off when launches are short and many: small images with one
    // iteration per launch.  With passes of several iterations the launches
    // are few and a replay measured slower than launching them directly
    // (1000 iterations: 256^2 3.34 against 3.25 ms, 512^2 3.77 against 3.69)
    use_graph = !blocked && (int64_t)L.nz * L.ny * L.nx <= (1 << 20) &&
                prm.max_iter >= 2 * chunk;
  }
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  if (use_graph && prm.max_iter >= chunk) {
    TVPD_HIP(hipStreamBeginCapture(poll->capture, hipStreamCaptureModeThreadLocal));
    rc = enqueue_sweeps(L, prm.c, 0, chunk, ce, blocked, ws, poll->capture);
    hipGraph_t gtmp = nullptr;
    const hipError_t e = hipStreamEndCapture(poll->capture, &gtmp);
    if (rc || e != hipSuccess) {
      if (gtmp) (void)hipGraphDestroy(gtmp);
      return rc ? rc : TVPD_ERR_HIP;
    }
    graph = gtmp;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return TVPD_ERR_HIP;
    }
  }
  auto cleanup = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  };

  int64_t launched = 0;
  int slot = 0, inflight = 0;
  const DevState* dst = reinterpret_cast<const DevState*>(ws);
  DevState* hst = reinterpret_cast<DevState*>(poll->host);
  bool stop = false;
  while (launched < prm.max_iter && !stop) {
    const int n = (int)std::min<int64_t>(chunk, prm.max_iter - launched);
    if (exec && n == chunk) {
      if (hipGraphLaunch(exec, s) != hipSuccess) {
        cleanup();
        return TVPD_ERR_HIP;
      }
    } else {
      rc = enqueue_sweeps(L, prm.c, launched, n, ce, blocked, ws, s);
      if (rc) {
        cleanup();
        return rc;
      }
    }
    launched += n;
    if (can_stop) {
      if (hipMemcpyAsync(&hst[slot], dst, sizeof(DevState),
                         hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipEventRecord(poll->ev[slot], s) != hipSuccess) {
        cleanup();
        return TVPD_ERR_HIP;
      }
      ++inflight;
      if (inflight == 2) {
        // wait for the previous chunk only; the current one keeps the
        // device busy meanwhile
        const int prev = slot ^ 1;
        if (hipEventSynchronize(poll->ev[prev]) != hipSuccess) {
          cleanup();
          return TVPD_ERR_HIP;
        }
        if (hst[prev].converged || hst[prev].flags) stop = true;
        inflight = 1;
      }
      slot ^= 1;
    }
  }
  cleanup();
  // final pair energies when no check passed
  TVPD_HIP(launch_energy(L, prm.c.lam, ws, true, s));
  TVPD_HIP(launch_read(L, ws, f_out, nullptr, s));
  TVPD_HIP(hipMemcpyAsync(&hst[0], dst, sizeof(DevState),
                          hipMemcpyDeviceToHost, s));
  TVPD_HIP(hipStreamSynchronize(s));
  if (res) {
    res->converged = hst[0].converged;
    res->iters = hst[0].converged ? hst[0].iters : hst[0].k;
    res->primal = hst[0].P;
    res->dual = hst[0].D;
    res->gap = hst[0].gap;
  }
  return hst[0].flags ? TVPD_ERR_DEVICE : TVPD_OK;
}

}  // namespace
}  // namespace tvpd

using namespace tvpd;

extern "C" {

const char* tvpd_status_string(int status) {
  switch (status) {
    case TVPD_OK: return "ok";
    case TVPD_ERR_INVALID_ARG: return "invalid argument";
    case TVPD_ERR_SHAPE: return "invalid shape";
    case TVPD_ERR_ALIGNMENT: return "workspace not 256-byte aligned";
    case TVPD_ERR_WORKSPACE: return "workspace too small";
    case TVPD_ERR_HIP: return "HIP runtime error";
    case TVPD_ERR_UNSUPPORTED: return "unsupported request";
    case TVPD_ERR_STEP: return "step sizes violate tau*sigma*||grad||^2 < 1";
    case TVPD_ERR_DEVICE: return "device-side check failed";
    case TVPD_ERR_SCRATCH: return "request exceeds the static scratch area";
    default: return "unknown status";
  }
}

int tvpd_version(void) { return kVersion; }

int tvpd_release_thread_resources(void) {
  host_poll_release(t_poll);
  release_batch_thread_resources();
  return TVPD_OK;
}

int tvpd_stream_copy(const float* src, float* dst, int64_t n, void* stream) {
  if (!src || !dst || n <= 0 || n % 4 != 0) return TVPD_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
    return TVPD_ERR_INVALID_ARG;
  TVPD_HIP(launch_stream_copy(src, dst, n, static_cast<hipStream_t>(stream)));
  return TVPD_OK;
}

int tvpd_workspace_size(const tvpd_shape* shape, size_t* bytes) {
  if (!bytes) return TVPD_ERR_INVALID_ARG;
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  *bytes = make_layout(*shape).bytes;
  return TVPD_OK;
}

int tvpd_init(const tvpd_shape* shape, const float* g, void* ws,
              size_t ws_bytes, void* stream) {
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  if (!g) return TVPD_ERR_INVALID_ARG;
  const Layout L = make_layout(*shape);
  if (int rc = ws_ok(L, ws, ws_bytes)) return rc;
  return launch_init(L, g, ws, (hipStream_t)stream) == hipSuccess
             ? TVPD_OK
             : TVPD_ERR_HIP;
}

int tvpd_step(const tvpd_shape* shape, const tvpd_coeffs* c, int32_t n_iter,
              void* ws, size_t ws_bytes, void* stream) {
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  if (n_iter < 0) return TVPD_ERR_INVALID_ARG;
  if (int rc = coeffs_ok(*shape, c)) return rc;
  const Layout L = make_layout(*shape);
  if (int rc = ws_ok(L, ws, ws_bytes)) return rc;
  hipStream_t s = (hipStream_t)stream;
  TVPD_HIP(launch_set_params(ws, INT_MAX, -1.0, s));
  return enqueue_sweeps(L, *c, 0, n_iter, 0, pass_depth() != 1, ws, s);
}

int tvpd_read_state(const tvpd_shape* shape, const void* ws, size_t ws_bytes,
                    float* f_out, float* p_out, void* stream) {
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  if (!f_out) return TVPD_ERR_INVALID_ARG;
  const Layout L = make_layout(*shape);
  if (int rc = ws_ok(L, ws, ws_bytes)) return rc;
  return launch_read(L, ws, f_out, p_out, (hipStream_t)stream) == hipSuccess
             ? TVPD_OK
             : TVPD_ERR_HIP;
}

int tvpd_iteration(const tvpd_shape* shape, const void* ws, size_t ws_bytes,
                   int32_t* k, void* stream) {
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  if (!k) return TVPD_ERR_INVALID_ARG;
  const Layout L = make_layout(*shape);
  if (int rc = ws_ok(L, ws, ws_bytes)) return rc;
  hipStream_t s = (hipStream_t)stream;
  int32_t v = 0;
  TVPD_HIP(hipMemcpyAsync(&v, ws, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TVPD_HIP(hipStreamSynchronize(s));
  *k = v;
  return TVPD_OK;
}

int tvpd_energy_gap(const tvpd_shape* shape, float lam, void* ws,
                    size_t ws_bytes, double out[3], void* stream) {
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  if (!out || !(lam >= 0.0f)) return TVPD_ERR_INVALID_ARG;
  const Layout L = make_layout(*shape);
  if (int rc = ws_ok(L, ws, ws_bytes)) return rc;
  hipStream_t s = (hipStream_t)stream;
  TVPD_HIP(launch_energy(L, lam, ws, false, s));
  DevState h;
  TVPD_HIP(hipMemcpyAsync(&h, ws, sizeof(DevState), hipMemcpyDeviceToHost, s));
  TVPD_HIP(hipStreamSynchronize(s));
  out[0] = h.P;
  out[1] = h.D;
  out[2] = h.gap;
  return h.flags ? TVPD_ERR_DEVICE : TVPD_OK;
}

int tvpd_solve(const tvpd_shape* shape, const float* g, float* f_out,
               const tvpd_params* prm, void* ws, size_t ws_bytes,
               tvpd_result* res, void* stream) {
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  if (!g || !f_out || !prm) return TVPD_ERR_INVALID_ARG;
  if (prm->max_iter < 0 || prm->check_every < 0) return TVPD_ERR_INVALID_ARG;
  if (std::isnan(prm->gap_tol)) return TVPD_ERR_INVALID_ARG;
  if (int rc = coeffs_ok(*shape, &prm->c)) return rc;
  const Layout L = make_layout(*shape);
  if (int rc = ws_ok(L, ws, ws_bytes)) return rc;
  return solve_plain(L, g, f_out, *prm, ws, res, (hipStream_t)stream);
}

int tvpd_set_tile(const tvpd_shape* shape, int32_t th, int32_t wpb,
                  int32_t order) {
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  if (shape->ndim != 2) return TVPD_ERR_UNSUPPORTED;
  if (th < 1 || th > 65536) return TVPD_ERR_INVALID_ARG;
  if (order != 0 && order != 1 && order != kOrderPipe) return TVPD_ERR_INVALID_ARG;
  if (order != kOrderPipe && wpb != 1 && wpb != 2 && wpb != 4)
    return TVPD_ERR_INVALID_ARG;
  Tile2D t;
  t.th = th;
  t.wpb = wpb;
  t.order = order;
  remember_tile2d(*shape, t);
  return TVPD_OK;
}

int tvpd_get_tile(const tvpd_shape* shape, int32_t* th, int32_t* wpb,
                  int32_t* order) {
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  if (shape->ndim != 2) return TVPD_ERR_UNSUPPORTED;
  if (!th || !wpb || !order) return TVPD_ERR_INVALID_ARG;
  const Tile2D t = tile2d_for(make_layout(*shape));
  *th = t.th;
  *wpb = t.wpb;
  *order = t.order;
  return TVPD_OK;
}

int tvpd_set_tile3d(const tvpd_shape* shape, int32_t th, int32_t tz,
                    int32_t wpb) {
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  if (shape->ndim != 3) return TVPD_ERR_UNSUPPORTED;
  Tile3D t;
  t.th = th;
  t.tz = tz;
  t.wpb = wpb;
  if (!tile3d_ok(t) || tz > 65536) return TVPD_ERR_INVALID_ARG;
  remember_tile3d(*shape, t);
  return TVPD_OK;
}

int tvpd_get_tile3d(const tvpd_shape* shape, int32_t* th, int32_t* tz,
                    int32_t* wpb) {
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  if (shape->ndim != 3) return TVPD_ERR_UNSUPPORTED;
  if (!th || !tz || !wpb) return TVPD_ERR_INVALID_ARG;
  const Tile3D t = tile3d_for(make_layout(*shape));
  *th = t.th;
  *tz = t.tz;
  *wpb = t.wpb;
  return TVPD_OK;
}

int tvpd_autotune(const tvpd_shape* shape, void* ws, size_t ws_bytes,
                  const char* cache_path, int32_t* th, int32_t* wpb,
                  int32_t* order, float* us, void* stream) {
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  const Layout L = make_layout(*shape);
  if (int rc = ws_ok(L, ws, ws_bytes)) return rc;
  if (shape->ndim == 3) {
    Tile3D best;
    float best_us = 0.0f;
    if (int rc = autotune3d(*shape, L, ws, (hipStream_t)stream, &best, &best_us))
      return rc;
    if (cache_path) {
      if (int rc = tune_save3d(cache_path, *shape, best, best_us)) return rc;
    }
    if (th) *th = best.th;
    if (wpb) *wpb = best.wpb;
    if (order) *order = best.tz;
    if (us) *us = best_us;
    return TVPD_OK;
  }
  Tile2D best;
  float best_us = 0.0f;
  if (int rc = autotune2d(*shape, L, ws, (hipStream_t)stream, &best, &best_us))
    return rc;
  if (cache_path) {
    if (int rc = tune_save(cache_path, *shape, best, best_us)) return rc;
  }
  if (th) *th = best.th;
  if (wpb) *wpb = best.wpb;
  if (order) *order = best.order;
  if (us) *us = best_us;
  return TVPD_OK;
}

int tvpd_tune_load(const char* cache_path, int32_t* count) {
  if (!cache_path || !count) return TVPD_ERR_INVALID_ARG;
  int n = 0;
  if (int rc = tune_load(cache_path, &n)) return rc;
  *count = n;
  return TVPD_OK;
}

int tvpd_set_blocking(int32_t on) {
  if (on != 0 && on != 1) return TVPD_ERR_INVALID_ARG;
  g_depth.store(on ? 0 : 1);
  return TVPD_OK;
}

int tvpd_set_pass_depth(int32_t depth) {
  if (depth < 0 || depth > kPipeMaxPass) return TVPD_ERR_INVALID_ARG;
  g_depth.store(depth);
  return TVPD_OK;
}

int tvpd_set_wait_limit(int64_t polls) {
  if (polls < 0) return TVPD_ERR_INVALID_ARG;
  g_wait_limit.store(polls);
  return TVPD_OK;
}

int tvpd_get_pass_depth(int32_t* depth) {
  if (!depth) return TVPD_ERR_INVALID_ARG;
  *depth = g_depth.load();
  return TVPD_OK;
}

int tvpd_pass_length(const tvpd_shape* shape, int32_t* n) {
  if (!n) return TVPD_ERR_INVALID_ARG;
  if (!shape_ok(shape)) return TVPD_ERR_SHAPE;
  if (shape->ndim != 2) return TVPD_ERR_UNSUPPORTED;
  const Tile2D t = tile2d_for(make_layout(*shape));
  *n = t.order == kOrderPipe ? pipe_depth() : walk_depth();
  return TVPD_OK;
}

}  // extern "C"
