// Tile selection for the fused 2D sweep: a process-wide table of chosen
// tiles, a default rule, a measuring autotuner and a small text cache.
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace tvpd {
namespace {

struct TileEntry {
  tvpd_shape s;
  Tile2D t;
};

struct TileEntry3 {
  tvpd_shape s;
  Tile3D t;
};

std::mutex g_mu;
std::vector<TileEntry> g_table;
std::vector<TileEntry3> g_table3;

bool same(const tvpd_shape& a, const Layout& L) {
  return a.ndim == L.ndim && a.nz == L.nz && a.ny == L.ny && a.nx == L.nx;
}

int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipGetDeviceProperties(&p, dev) == hipSuccess && p.multiProcessorCount > 0)
      cus = p.multiProcessorCount;
    else
      cus = 256;
  }
  return cus;
}

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipGetDeviceProperties(&p, dev) == hipSuccess) {
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
  }
  return "unknown";
}

}  // namespace

// Default: blocks of 4 side-by-side waves.  One-iteration and two-iteration
// passes: bands tall enough for about one block per compute unit (few
// concurrent row streams keep HBM pages open).  Deeper passes: the shortest
// bands whose blocks all fit on the GPU at once, one block per CU from
// passes of 5 on (two per CU for passes of 3 and 4).  At depth 5 one block
// per CU (one wave per SIMD) beat two: its bands are twice as tall, so the
// 2 depth + 1 halo rows each band recomputes cost half as much -- 4096^2:
// 74-row bands 642 000 Mpixel-iterations/s against 617 000 with 37 rows;
// 2048^2: 19 rows 495 000 against 420 000 with 10; 1024^2: 6 rows 209 000
// against 186 000 with 3.  (One block more than the CUs is a second round
// for some CUs: 70-row bands at 4096^2 gave 488 000.)  The search starts at
// bands of 2 rows: on images too small to fill the GPU a pass costs one band
// walk of th + 2 depth - 1 steps, and at 256^2 (1000 iterations, depth 5)
// bands of 2 rows took 3.7 ms against 4.3 and 5.3 ms with 4 and 8.
// Pipelined passes (tile2d_pipe.h) are not a default: at 4096^2 they ran
// 3% behind the walk (288 against 280 us per ten iterations), bound by the
// issue of their longer per-row instruction chains; the autotuner tries them.
Tile2D default_tile2d(const Layout& L) {
  Tile2D t;
  t.wpb = 4;
  t.order = 0;
  const int depth = walk_depth();
  const int cus = device_cus();
  int64_t th;
  if (depth >= 3) {
    const int64_t ntx = (L.nx + xs_owned(depth) - 1) / xs_owned(depth);
    const int64_t max_blocks = (depth >= 5 ? 1LL : 2LL) * cus;
    th = 2;
    while (th < 256 &&
           (ntx * ((L.ny + th - 1) / th) + t.wpb - 1) / t.wpb > max_blocks)
      ++th;
  } else {
    const int64_t ntx = (L.nx + xs_owned(depth) - 1) / xs_owned(depth);
    const int64_t target_waves = 4LL * cus;
    th = (ntx * L.ny + target_waves - 1) / target_waves;
    if (th < 8) th = 8;
    if (th > 256) th = 256;
  }
  t.th = (int)th;
  return t;
}

Tile2D tile2d_for(const Layout& L) {
  std::lock_guard<std::mutex> g(g_mu);
  for (const TileEntry& e : g_table)
    if (same(e.s, L)) return e.t;
  return default_tile2d(L);
}

void remember_tile2d(const tvpd_shape& s, const Tile2D& t) {
  std::lock_guard<std::mutex> g(g_mu);
  for (TileEntry& e : g_table) {
    if (e.s.ndim == s.ndim && e.s.nz == s.nz && e.s.ny == s.ny &&
        e.s.nx == s.nx) {
      e.t = t;
      return;
    }
  }
  g_table.push_back({s, t});
}

// Default 3D tile: bands of 4 rows, blocks of 4 waves, segments deep enough
// for about 4 waves (one block) per CU: deeper segments re-read fewer
// prologue planes, and the rolling prefetch of each wave hides the latency.
Tile3D default_tile3d(const Layout& L) {
  Tile3D t;
  t.th = 4;
  t.wpb = 4;
  const int64_t ntx = (L.nx + kStripCols - 1) / kStripCols;
  const int64_t cols = ntx * ((L.ny + t.th - 1) / t.th);
  const int64_t target_waves = 4LL * device_cus();
  int64_t tz = (cols * L.nz + target_waves - 1) / target_waves;
  if (tz < 4) tz = 4;
  if (tz > L.nz) tz = L.nz;
  t.tz = (int)tz;
  return t;
}

Tile3D tile3d_for(const Layout& L) {
  std::lock_guard<std::mutex> g(g_mu);
  for (const TileEntry3& e : g_table3)
    if (same(e.s, L)) return e.t;
  return default_tile3d(L);
}

void remember_tile3d(const tvpd_shape& s, const Tile3D& t) {
  std::lock_guard<std::mutex> g(g_mu);
  for (TileEntry3& e : g_table3) {
    if (e.s.ndim == s.ndim && e.s.nz == s.nz && e.s.ny == s.ny &&
        e.s.nx == s.nx) {
      e.t = t;
      return;
    }
  }
  g_table3.push_back({s, t});
}

// Time one tile: warm up, then enough launches for about 2 ms of work, each
// a pass of n iterations; the result is per iteration.
static int time_tile(const Layout& L, const Tile2D& t, int n, void* ws,
                     hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* us) {
  tvpd_coeffs c;
  c.lam = 0.1f;
  c.tau = c.sigma = 0.35355339f;
  c.theta = 1.0f;
  if (sweep2d_blocks(L, t, n) > L.max_partials) return TVPD_ERR_INVALID_ARG;
  for (int i = 0; i < 2; ++i)
    if (launch_sweep2d(L, t, c, false, n, ws, s) != hipSuccess) return TVPD_ERR_HIP;
  int reps = 2;
  float ms = 0.0f;
  for (int round = 0; round < 2; ++round) {
    if (hipEventRecord(e0, s) != hipSuccess) return TVPD_ERR_HIP;
    for (int i = 0; i < reps; ++i)
      if (launch_sweep2d(L, t, c, false, n, ws, s) != hipSuccess) return TVPD_ERR_HIP;
    if (hipEventRecord(e1, s) != hipSuccess) return TVPD_ERR_HIP;
    if (hipEventSynchronize(e1) != hipSuccess) return TVPD_ERR_HIP;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return TVPD_ERR_HIP;
    if (round == 0) {
      const float per = ms / reps;
      reps = per > 0.0f ? (int)(2.0f / per) : 50;
      if (reps < 3) reps = 3;
      if (reps > 200) reps = 200;
    }
  }
  *us = ms * 1000.0f / reps / (float)n;
  return TVPD_OK;
}

int autotune2d(const tvpd_shape& sh, const Layout& L, void* ws, hipStream_t s,
               Tile2D* best, float* best_us) {
  if (launch_set_params(ws, 0x7fffffff, -1.0, s) != hipSuccess) return TVPD_ERR_HIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return TVPD_ERR_HIP;
  static const int ths[] = {2, 4, 8, 12, 16, 24, 32, 36, 40, 44, 48, 64, 96, 128,
                            192, 256};
  static const int wpbs[] = {1, 2, 4};
  float bu = 1e30f;
  Tile2D bt = default_tile2d(L);
  int rc = TVPD_OK;
  for (int th : ths) {
    if (th > L.ny && th != ths[0]) break;
    for (int w : wpbs) {
      for (int order = 0; order < 2; ++order) {
        Tile2D t;
        t.th = th;
        t.wpb = w;
        t.order = order;
        float us = 0.0f;
        rc = time_tile(L, t, walk_depth(), ws, s, e0, e1, &us);
        if (rc == TVPD_ERR_INVALID_ARG) {
          rc = TVPD_OK;
          continue;
        }
        if (rc) break;
        if (us < bu) {
          bu = us;
          bt = t;
        }
      }
      if (rc) break;
    }
    if (rc) break;
  }
  // pipelined passes: bands for one, two and three tiles per CU and a few
  // fixed heights
  if (rc == TVPD_OK && pass_depth() != 1) {
    const int cus = device_cus();
    const int ntx = (L.nx + kPipeOwned - 1) / kPipeOwned;
    int pths[8];
    int np = 0;
    for (int m = 1; m <= 3; ++m) {
      const int nty = m * cus / ntx;
      if (nty >= 1) pths[np++] = (L.ny + nty - 1) / nty;
    }
    for (int th : {64, 128, 256}) pths[np++] = th;
    for (int i = 0; i < np && rc == TVPD_OK; ++i) {
      const int th = pths[i];
      if (th < 1 || (th > L.ny && i >= 3)) continue;
      Tile2D t;
      t.th = th;
      t.wpb = 1;
      t.order = kOrderPipe;
      float us = 0.0f;
      rc = time_tile(L, t, pipe_depth(), ws, s, e0, e1, &us);
      if (rc == TVPD_ERR_INVALID_ARG) {
        rc = TVPD_OK;
        continue;
      }
      if (rc == TVPD_OK && us < bu) {
        bu = us;
        bt = t;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  remember_tile2d(sh, bt);
  *best = bt;
  *best_us = bu;
  return TVPD_OK;
}

// Per-iteration time of one 3D tile (same scheme as time_tile).
static int time_tile3d(const Layout& L, const Tile3D& t, void* ws,
                       hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* us) {
  tvpd_coeffs c;
  c.lam = 0.1f;
  c.tau = c.sigma = 0.28867513f;
  c.theta = 1.0f;
  if (sweep3d_blocks(L, t) > L.max_partials) return TVPD_ERR_INVALID_ARG;
  for (int i = 0; i < 2; ++i)
    if (launch_sweep3d(L, t, c, false, ws, s) != hipSuccess) return TVPD_ERR_HIP;
  int n = 2;
  float ms = 0.0f;
  for (int round = 0; round < 2; ++round) {
    if (hipEventRecord(e0, s) != hipSuccess) return TVPD_ERR_HIP;
    for (int i = 0; i < n; ++i)
      if (launch_sweep3d(L, t, c, false, ws, s) != hipSuccess) return TVPD_ERR_HIP;
    if (hipEventRecord(e1, s) != hipSuccess) return TVPD_ERR_HIP;
    if (hipEventSynchronize(e1) != hipSuccess) return TVPD_ERR_HIP;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return TVPD_ERR_HIP;
    if (round == 0) {
      const float per = ms / n;
      n = per > 0.0f ? (int)(2.0f / per) : 50;
      if (n < 3) n = 3;
      if (n > 200) n = 200;
    }
  }
  *us = ms * 1000.0f / n;
  return TVPD_OK;
}

int autotune3d(const tvpd_shape& sh, const Layout& L, void* ws, hipStream_t s,
               Tile3D* best, float* best_us) {
  if (launch_set_params(ws, 0x7fffffff, -1.0, s) != hipSuccess) return TVPD_ERR_HIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return TVPD_ERR_HIP;
  static const int ths[] = {2, 4};
  static const int tzs[] = {2, 4, 8, 16, 32, 64, 128};
  static const int wpbs[] = {1, 2, 4};
  float bu = 1e30f;
  Tile3D bt = default_tile3d(L);
  int rc = TVPD_OK;
  for (int th : ths) {
    for (int tz : tzs) {
      if (tz > L.nz && tz != tzs[0]) break;
      for (int w : wpbs) {
        Tile3D t;
        t.th = th;
        t.tz = tz;
        t.wpb = w;
        float us = 0.0f;
        rc = time_tile3d(L, t, ws, s, e0, e1, &us);
        if (rc == TVPD_ERR_INVALID_ARG) {
          rc = TVPD_OK;
          continue;
        }
        if (rc) break;
        if (us < bu) {
          bu = us;
          bt = t;
        }
      }
      if (rc) break;
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  remember_tile3d(sh, bt);
  *best = bt;
  *best_us = bu;
  return TVPD_OK;
}

// Cache file: one line per entry,
//   <arch> <ndim> <nz> <ny> <nx> <th> <wpb> <order> <us>      (ndim 2)
//   <arch> <ndim> <nz> <ny> <nx> <th> <wpb> <tz> <us>         (ndim 3)
int tune_save(const char* path, const tvpd_shape& s, const Tile2D& t,
              float us) {
  FILE* f = std::fopen(path, "a");
  if (!f) return TVPD_ERR_INVALID_ARG;
  std::fprintf(f, "%s %d %d %d %d %d %d %d %.3f\n", device_arch().c_str(),
               s.ndim, s.nz, s.ny, s.nx, t.th, t.wpb, t.order, us);
  std::fclose(f);
  return TVPD_OK;
}

int tune_save3d(const char* path, const tvpd_shape& s, const Tile3D& t,
                float us) {
  FILE* f = std::fopen(path, "a");
  if (!f) return TVPD_ERR_INVALID_ARG;
  std::fprintf(f, "%s %d %d %d %d %d %d %d %.3f\n", device_arch().c_str(),
               s.ndim, s.nz, s.ny, s.nx, t.th, t.wpb, t.tz, us);
  std::fclose(f);
  return TVPD_OK;
}

int tune_load(const char* path, int* count) {
  FILE* f = std::fopen(path, "r");
  if (!f) return TVPD_ERR_INVALID_ARG;
  const std::string arch = device_arch();
  char line[512];
  int n = 0;
  while (std::fgets(line, sizeof line, f)) {
    char a[128];
    tvpd_shape s;
    Tile2D t;
    float us;
    if (std::sscanf(line, "%127s %d %d %d %d %d %d %d %f", a, &s.ndim, &s.nz,
                    &s.ny, &s.nx, &t.th, &t.wpb, &t.order, &us) != 9)
      continue;
    if (arch != a) continue;
    if (s.ndim == 3) {
      Tile3D t3;
      t3.th = t.th;
      t3.wpb = t.wpb;
      t3.tz = t.order;
      if (!tile3d_ok(t3)) continue;
      remember_tile3d(s, t3);
      ++n;
      continue;
    }
    if (s.ndim != 2 || t.th < 1 ||
        (t.order != 0 && t.order != 1 && t.order != kOrderPipe) ||
        (t.order != kOrderPipe && t.wpb != 1 && t.wpb != 2 && t.wpb != 4))
      continue;
    remember_tile2d(s, t);  // later lines override earlier ones
    ++n;
  }
  std::fclose(f);
  *count = n;
  return TVPD_OK;
}

}  // namespace tvpd
