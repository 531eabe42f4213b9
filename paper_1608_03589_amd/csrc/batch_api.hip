// C ABI of the batched solver: workspace layout, tile table, the two
// drivers (persistent launch, graph-replayed iteration blocks) and the
// batch tile autotuner.
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "batch.h"

namespace tvpd {
namespace {

struct BatchLayout {
  int n;
  int64_t tmax;              // tile slots (enough for th = 1)
  size_t off_imgs, off_state, off_offs, off_tiles, off_active, off_part;
  size_t off_fpart, off_arena;
  size_t bytes;
  std::vector<int64_t> img_off;    // float offset of each plane block
  std::vector<int64_t> img_plane;  // floats per plane
  std::vector<int> img_pitch;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool shapes_ok(int n, const tvpd_shape* s) {
  if (n < 1 || !s) return false;
  for (int i = 0; i < n; ++i) {
    if (s[i].ndim != 2 || s[i].nz != 1 || s[i].ny < 1 || s[i].nx < 1 ||
        s[i].ny > (1 << 20) || s[i].nx > (1 << 20))
      return false;
  }
  return true;
}

BatchLayout make_batch_layout(int n, const tvpd_shape* s) {
  BatchLayout L;
  L.n = n;
  L.tmax = 0;
  int64_t arena = 0;
  for (int i = 0; i < n; ++i) {
    const int pitch = (int)round_up(s[i].nx, kColsPerLane);
    const int64_t plane = round_up((int64_t)s[i].ny * pitch, 64);
    L.img_pitch.push_back(pitch);
    L.img_plane.push_back(plane);
    L.img_off.push_back(arena);
    arena += kBatchPlanes * plane;
    // each tile table holds at most ny tiles per strip (bands of >= 1 row)
    L.tmax += (int64_t)((s[i].nx + kBatchStrip - 1) / kBatchStrip) *
              kBatchTables * s[i].ny;
  }
  size_t o = kHeaderBytes;
  L.off_imgs = o;
  o = align_up(o + n * sizeof(ImgDesc), kAlign);
  L.off_state = o;
  o = align_up(o + n * sizeof(ImgState), kAlign);
  L.off_offs = o;
  o = align_up(o + n * sizeof(int64_t), kAlign);
  L.off_tiles = o;
  o = align_up(o + L.tmax * sizeof(TileDesc), kAlign);
  L.off_active = o;
  o = align_up(o + L.tmax * sizeof(int32_t), kAlign);
  L.off_part = o;
  o = align_up(o + L.tmax * 4 * sizeof(double), kAlign);
  L.off_fpart = o;
  o = align_up(o + (size_t)n * kFinalBlocks * 2 * sizeof(double), kAlign);
  L.off_arena = o;
  L.bytes = o + (size_t)arena * sizeof(float);
  return L;
}

std::mutex g_btile_mu;
int g_btile_th = 16, g_btile_wpb = 8;

int params_ok(int n, const tvpd_shape* s, const tvpd_params* prm) {
  if (!prm) return TVPD_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    if (prm[i].max_iter != prm[0].max_iter ||
        prm[i].check_every != prm[0].check_every)
      return TVPD_ERR_INVALID_ARG;
    if (prm[i].max_iter < 0 || prm[i].check_every < 0 ||
        std::isnan(prm[i].gap_tol))
      return TVPD_ERR_INVALID_ARG;
    const tvpd_coeffs& c = prm[i].c;
    if (!(c.lam >= 0.0f) || !std::isfinite(c.lam)) return TVPD_ERR_INVALID_ARG;
    if (!(c.theta >= 0.0f && c.theta <= 1.0f)) return TVPD_ERR_INVALID_ARG;
    if (!(c.tau > 0.0f) || !(c.sigma > 0.0f) || !std::isfinite(c.tau) ||
        !std::isfinite(c.sigma))
      return TVPD_ERR_STEP;
    auto term = [](int m) {
      const double a = std::sin(M_PI * (m - 1) / (2.0 * m));
      return 4.0 * a * a;
    };
    if ((double)c.tau * c.sigma * (term(s[i].nx) + term(s[i].ny)) >= 1.0)
      return TVPD_ERR_STEP;
  }
  return TVPD_OK;
}

#define BHIP(call)                                   \
  do {                                               \
    if ((call) != hipSuccess) return TVPD_ERR_HIP;   \
  } while (0)

// Host image of the descriptor region [hdr .. partials) and kernel args.
struct BatchSetup {
  std::vector<char> host;  // bytes [0, off_part) of the workspace
  BatchArgs args;
  int ntiles;
};

// Rows per band of the first short-band table; the later ones halve it
// (a band walk of a pass of n iterations covers 2n extra rows, so short
// bands pay off only once few images are left).
constexpr int kShortBand = 8;

void build_setup(const BatchLayout& L, int n, const tvpd_shape* s,
                 const int64_t* offsets, const tvpd_params* prm, int th,
                 int th_short, int wpb, int slots, char* ws, BatchSetup& B) {
  B.host.assign(L.off_part, 0);
  char* h = B.host.data();
  ImgDesc* imgs = reinterpret_cast<ImgDesc*>(h + L.off_imgs);
  int64_t* offs = reinterpret_cast<int64_t*>(h + L.off_offs);
  TileDesc* tiles = reinterpret_cast<TileDesc*>(h + L.off_tiles);
  int32_t* active = reinterpret_cast<int32_t*>(h + L.off_active);
  int ths[kBatchTables];
  ths[0] = th;
  ths[1] = std::min(th, th_short > 0 ? th_short : kShortBand);
  for (int j = 2; j < kBatchTables; ++j) ths[j] = std::max(1, ths[j - 1] / 2);
  int t = 0;
  for (int tbl = 0; tbl < kBatchTables; ++tbl) {
    for (int i = 0; i < n; ++i) {
      ImgDesc& D = imgs[i];
      D.tile_first[tbl] = t;
      const int ntx = (s[i].nx + kBatchStrip - 1) / kBatchStrip;
      const int nty = (s[i].ny + ths[tbl] - 1) / ths[tbl];
      for (int ty = 0; ty < nty; ++ty)
        for (int tx = 0; tx < ntx; ++tx) {
          tiles[t].img = i;
          tiles[t].x0 = tx * kBatchStrip;
          tiles[t].y0 = ty * ths[tbl];
          tiles[t].y1 = std::min((ty + 1) * ths[tbl], s[i].ny);
          ++t;
        }
      D.tile_count[tbl] = t - D.tile_first[tbl];
    }
  }
  for (int i = 0; i < n; ++i) {
    ImgDesc& D = imgs[i];
    D.off = L.img_off[i];
    D.plane = L.img_plane[i];
    D.ny = s[i].ny;
    D.nx = s[i].nx;
    D.pitch = L.img_pitch[i];
    D.lam = prm[i].c.lam;
    D.tau = prm[i].c.tau;
    D.sigma = prm[i].c.sigma;
    D.theta = prm[i].c.theta;
    D.tol = prm[i].gap_tol;
    offs[i] = offsets[i];
  }
  // start on short bands when the tall ones cannot fill the grid (the rule
  // of compact_active)
  auto tiles_of = [&](int tbl) {
    int c = 0;
    for (int i = 0; i < n; ++i) c += imgs[i].tile_count[tbl];
    return c;
  };
  int tbl0 = tiles_of(0) < slots ? 1 : 0;
  while (tbl0 >= 1 && tbl0 + 1 < kBatchTables && tiles_of(tbl0 + 1) <= slots) ++tbl0;
  int na = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < imgs[i].tile_count[tbl0]; ++j)
      active[na++] = imgs[i].tile_first[tbl0] + j;
  BatchHdr* hdr = reinterpret_cast<BatchHdr*>(h);
  hdr->n_active = na;
  hdr->table = tbl0;
  B.ntiles = t;
  BatchArgs& a = B.args;
  a.hdr = reinterpret_cast<BatchHdr*>(ws);
  a.imgs = reinterpret_cast<const ImgDesc*>(ws + L.off_imgs);
  a.state = reinterpret_cast<ImgState*>(ws + L.off_state);
  a.tiles = reinterpret_cast<const TileDesc*>(ws + L.off_tiles);
  a.active = reinterpret_cast<int32_t*>(ws + L.off_active);
  a.partials = reinterpret_cast<double*>(ws + L.off_part);
  a.fparts = reinterpret_cast<double*>(ws + L.off_fpart);
  a.arena = reinterpret_cast<float*>(ws + L.off_arena);
  a.nimg = n;
  a.ntiles = t;
  a.max_iter = prm[0].max_iter;
  a.check_every = prm[0].check_every;
  a.wpb = wpb;
  a.switch_tiles = slots;
  a.depth = walk_depth() < kBatchMaxPass ? walk_depth() : kBatchMaxPass;
}

thread_local HostPoll t_pin;

// Launches of iterations k0 .. k0+n-1: passes as batch_pass_len schedules
// them (the same schedule as the persistent driver), a check on the first
// iteration of a pass whenever it is due.
hipError_t enqueue_batch_iters(const BatchArgs& a, int grid, int k0, int n,
                               hipStream_t s) {
  const int ce = a.check_every;
  int i = 0;
  while (i < n) {
    const int k = k0 + i;
    const bool check = ce > 0 && (k % ce) == 0;
    const int len = batch_pass_len(k, k0 + n, ce, a.depth);
    const hipError_t e = launch_batch_sweep(a, grid, check, len, s);
    if (e != hipSuccess) return e;
    i += len;
  }
  return hipSuccess;
}

int run_graph_blocks(const BatchArgs& a, int grid, hipStream_t s) {
  HostPoll* pin = &t_pin;
  if (int rc = host_poll_get(*pin, 2 * sizeof(BatchHdr))) return rc;
  BatchHdr* hst = static_cast<BatchHdr*>(pin->host);
  const int ce = a.check_every;
  const int chunk = ce > 0 ? ce * ((32 + ce - 1) / ce) : 32;
  // one graph of `chunk` iterations, checks at multiples of check_every
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BHIP(hipStreamBeginCapture(pin->capture, hipStreamCaptureModeThreadLocal));
  const hipError_t err = enqueue_batch_iters(a, grid, 0, chunk, pin->capture);
  const hipError_t e2 = hipStreamEndCapture(pin->capture, &graph);
  if (err != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return TVPD_ERR_HIP;
  }
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return TVPD_ERR_HIP;
  }
  int rc = TVPD_OK;
  int64_t launched = 0;
  int slot = 0, inflight = 0;
  bool all_stopped = false;
  while (launched + chunk <= a.max_iter) {
    if (hipGraphLaunch(exec, s) != hipSuccess) {
      rc = TVPD_ERR_HIP;
      break;
    }
    launched += chunk;
    if (hipMemcpyAsync(&hst[slot], a.hdr, sizeof(BatchHdr),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(pin->ev[slot], s) != hipSuccess) {
      rc = TVPD_ERR_HIP;
      break;
    }
    if (++inflight == 2) {
      const int prev = slot ^ 1;
      if (hipEventSynchronize(pin->ev[prev]) != hipSuccess) {
        rc = TVPD_ERR_HIP;
        break;
      }
      inflight = 1;
      if (hst[prev].n_active == 0) {
        all_stopped = true;
        break;
      }
    }
    slot ^= 1;
  }
  // the iterations of max_iter beyond the last whole block, launched
  // directly; none once every image has stopped
  if (rc == TVPD_OK && !all_stopped && launched < a.max_iter &&
      enqueue_batch_iters(a, grid, (int)launched, (int)(a.max_iter - launched),
                          s) != hipSuccess)
    rc = TVPD_ERR_HIP;
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  return rc;
}

int solve_batched_impl(int n, const tvpd_shape* shapes, const int64_t* offsets,
                       const float* g, float* f, const tvpd_params* prm,
                       int mode, int th, int th_short, int wpb, void* ws,
                       size_t ws_bytes, tvpd_result* res, hipStream_t s) {
  const BatchLayout L = make_batch_layout(n, shapes);
  if (L.tmax > INT32_MAX) return TVPD_ERR_UNSUPPORTED;  // tile indices are int32
  if (!ws) return TVPD_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return TVPD_ERR_ALIGNMENT;
  if (ws_bytes < L.bytes) return TVPD_ERR_WORKSPACE;
  // grid of the driver: one block per CU for the persistent kernel (capped by
  // co-residency), two (one of 8 waves) for the launch drivers; the waves
  // share the active tiles out (tile_share).  One persistent block per CU is
  // faster on the 64
  // uneven images (61.7 against 66.4 ms with two of 4 waves): the grid
  // barrier costs by the block; one block of 8 waves, two per SIMD, takes
  // 55.7 ms against 59.1 with 4 waves, the extra waves shortening the
  // latency-bound walks at no barrier cost.
  int cus = 0;
  {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipGetDeviceProperties(&p, dev) != hipSuccess)
      return TVPD_ERR_HIP;
    cus = p.multiProcessorCount;
  }
  // (launch drivers: two blocks per CU of up to 4 waves, one of 8 waves;
  // either way two waves per SIMD, all resident at once)
  int grid = (wpb >= 8 ? 1 : 2) * cus;
  if (mode == 0) {
    const int cap = batch_persistent_grid(wpb);
    if (cap <= 0) return TVPD_ERR_HIP;
    grid = std::min(cus, cap);
  }
  BatchSetup B;
  // Short-band tables are taken while their tiles fit one wave per SIMD: a
  // walk is issue-bound once few images are left, and two waves sharing a
  // SIMD double its time, more than the longer walk of the next taller band.
  const int slots = std::min(grid * wpb, 4 * cus);
  build_setup(L, n, shapes, offsets, prm, th, th_short, wpb, slots,
              static_cast<char*>(ws), B);
  BHIP(hipMemcpyAsync(ws, B.host.data(), B.host.size(), hipMemcpyHostToDevice,
                      s));
  const int64_t* offs_dev = reinterpret_cast<const int64_t*>(
      static_cast<char*>(ws) + L.off_offs);
  BHIP(launch_batch_init(B.args, g, offs_dev, s));
  if (B.args.max_iter > 0) {
    if (mode == 0) {
      BHIP(launch_batch_persistent(B.args, grid, s));
    } else if (mode == 1) {
      if (int rc = run_graph_blocks(B.args, grid, s)) return rc;
    } else {
      BHIP(enqueue_batch_iters(B.args, grid, 0, B.args.max_iter, s));
    }
  }
  BHIP(launch_batch_final(B.args, f, offs_dev, s));
  std::vector<ImgState> st(n);
  BatchHdr hdr;
  BHIP(hipMemcpyAsync(st.data(), static_cast<char*>(ws) + L.off_state,
                      n * sizeof(ImgState), hipMemcpyDeviceToHost, s));
  BHIP(hipMemcpyAsync(&hdr, ws, sizeof(BatchHdr), hipMemcpyDeviceToHost, s));
  BHIP(hipStreamSynchronize(s));
  if (hdr.flags & kBatchErrBarrier) return TVPD_ERR_DEVICE;
  if (res)
    for (int i = 0; i < n; ++i) {
      res[i].iters = st[i].iters;
      res[i].converged = st[i].converged;
      res[i].primal = st[i].P;
      res[i].dual = st[i].D;
      res[i].gap = st[i].gap;
    }
  return TVPD_OK;
}

int batch_args_ok(int n, const tvpd_shape* shapes, const int64_t* offsets,
                  const float* g, const float* f, const tvpd_params* prm) {
  if (!shapes_ok(n, shapes)) return TVPD_ERR_SHAPE;
  if (!offsets || !g || !f) return TVPD_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i)
    if (offsets[i] < 0) return TVPD_ERR_INVALID_ARG;
  return params_ok(n, shapes, prm);
}

}  // namespace

void release_batch_thread_resources() { host_poll_release(t_pin); }

}  // namespace tvpd

using namespace tvpd;

extern "C" {

int tvpd_batch_workspace_size(int32_t n, const tvpd_shape* shapes,
                              size_t* bytes) {
  if (!bytes) return TVPD_ERR_INVALID_ARG;
  if (!shapes_ok(n, shapes)) return TVPD_ERR_SHAPE;
  const BatchLayout L = make_batch_layout(n, shapes);
  if (L.tmax > INT32_MAX) return TVPD_ERR_UNSUPPORTED;  // tile indices are int32
  *bytes = L.bytes;
  return TVPD_OK;
}

int tvpd_solve_batched(int32_t n, const tvpd_shape* shapes,
                       const int64_t* offsets, const float* g_arena,
                       float* f_arena, const tvpd_params* prm,
                       const tvpd_batch_opts* opts, void* ws, size_t ws_bytes,
                       tvpd_result* res, void* stream) {
  if (int rc = batch_args_ok(n, shapes, offsets, g_arena, f_arena, prm))
    return rc;
  int mode = 0, th = 0, wpb = 0, th_short = 0;
  if (opts) {
    mode = opts->mode;
    th = opts->th;
    wpb = opts->wpb;
    th_short = opts->th_short;
  }
  if (mode < 0 || mode > 2) return TVPD_ERR_INVALID_ARG;
  if (th < 0 || th > 4096 || th_short < 0 || th_short > 4096 ||
      !(wpb == 0 || wpb == 1 || wpb == 2 || wpb == 4 || wpb == 8))
    return TVPD_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> gl(g_btile_mu);
    if (th == 0) th = g_btile_th;
    if (wpb == 0) wpb = g_btile_wpb;
  }
  return solve_batched_impl(n, shapes, offsets, g_arena, f_arena, prm, mode,
                            th, th_short, wpb, ws, ws_bytes, res,
                            (hipStream_t)stream);
}

int tvpd_batch_autotune(int32_t n, const tvpd_shape* shapes,
                        const int64_t* offsets, const float* g_arena,
                        float* f_arena, const tvpd_params* prm, void* ws,
                        size_t ws_bytes, int32_t* th_out, int32_t* wpb_out,
                        float* ms_out, void* stream) {
  if (int rc = batch_args_ok(n, shapes, offsets, g_arena, f_arena, prm))
    return rc;
  hipStream_t s = (hipStream_t)stream;
  std::vector<tvpd_params> p(prm, prm + n);
  for (auto& q : p) {
    q.max_iter = 30;
    q.check_every = 10;
    q.gap_tol = -1.0;
  }
  hipEvent_t e0, e1;
  BHIP(hipEventCreate(&e0));
  BHIP(hipEventCreate(&e1));
  static const int ths[] = {8, 16, 32, 64, 128};
  static const int wpbs[] = {1, 2, 4, 8};
  float best = 1e30f;
  int bth = 32, bwpb = 4;
  int rc = TVPD_OK;
  for (int th : ths) {
    for (int w : wpbs) {
      float ms = 0.0f;
      for (int rep = 0; rep < 2 && rc == TVPD_OK; ++rep) {
        if (hipEventRecord(e0, s) != hipSuccess) rc = TVPD_ERR_HIP;
        if (!rc)
          rc = solve_batched_impl(n, shapes, offsets, g_arena, f_arena,
                                  p.data(), 0, th, 0, w, ws, ws_bytes,
                                  nullptr, s);
        if (!rc && (hipEventRecord(e1, s) != hipSuccess ||
                    hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          rc = TVPD_ERR_HIP;
      }
      if (rc) break;
      if (ms < best) {
        best = ms;
        bth = th;
        bwpb = w;
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> gl(g_btile_mu);
    g_btile_th = bth;
    g_btile_wpb = bwpb;
  }
  if (th_out) *th_out = bth;
  if (wpb_out) *wpb_out = bwpb;
  if (ms_out) *ms_out = best;
  return TVPD_OK;
}

}  // extern "C"
