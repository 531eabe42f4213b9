// Data structures of the batched solver (device side and host side).
#pragma once

#include "common.h"

namespace tvpd {

constexpr int kBatchErrBarrier = 1;  // a grid barrier wait ran out
constexpr int kBatchStopped = 2;     // an image stopped at the last check
// Tile tables: tall bands, then bands of 8, 4 and 2 rows (by default).
constexpr int kBatchTables = 4;

// Per-image description (device, read-only during a solve).
struct ImgDesc {
  int64_t off;       // float offset of the image's plane block in the arena
  int64_t plane;     // floats per plane
  int32_t ny, nx, pitch;
  int32_t tile_first[kBatchTables], tile_count[kBatchTables];  // per table
  float lam, tau, sigma, theta;
  double tol;        // relative gap tolerance (< 0: never stop)
};

// Plane block of an image in the batch arena: f in three slots, the dual
// (x, y) in two, and g.  Pass j (iterations k -> k+n) reads f slot j mod 3
// and dual slot j mod 2 and writes the next ones.  The third f slot lets the
// persistent driver decide a gap check while the next pass already runs:
// that pass writes f slot j+2 mod 3, so the f^k of an image stopped at the
// check of pass j survives until the stop is known, one grid barrier later.
constexpr int kBatchPlanes = 8;
constexpr int kBatchG = 7;
__host__ __device__ inline int batch_f(int fslot) { return fslot; }
__host__ __device__ inline int batch_p(int pslot) { return 3 + 2 * pslot; }
__host__ __device__ inline int batch_fslot(int pass) { return pass % 3; }
__host__ __device__ inline int batch_pslot(int pass) { return pass & 1; }

// Per-image result (device).
struct ImgState {
  int32_t converged;
  int32_t iters;
  int32_t fslot;     // f slot of the returned iterate once stopped
  int32_t pad;
  double P, D, gap;
};

struct TileDesc {
  int32_t img, x0, y0, y1;
};

// Batch header at the workspace start (device).
// Arrival counters and the barrier generation live in a SyncArea (sync.h)
// at byte kSyncOffset of the header.
struct BatchHdr {
  int32_t k;             // iteration of the running images
  int32_t n_active;      // entries of the active tile list
  int32_t flags;         // error bits
  int32_t table;         // tile table in use: 0 tall bands, then shorter ones
  int32_t pass;          // passes made: the plane slots of f^k and p^k
};

struct BatchArgs {
  BatchHdr* hdr;
  const ImgDesc* imgs;
  ImgState* state;
  const TileDesc* tiles;
  int32_t* active;
  double* partials;  // 4 per tile: (gap, P) of a check, by pass parity
  double* fparts;    // 2 per (image, final block)
  float* arena;
  int32_t nimg, ntiles;
  int32_t max_iter, check_every;
  int32_t wpb;
  int32_t switch_tiles;  // SIMD slots: short bands once fewer tall tiles are active
  int32_t depth;         // longest pass (iterations per sweep), 1 .. kBatchMaxPass
};

// Batch passes are 1, 2 or 5 iterations long: the drivers contain every
// pass length they can launch, and their register count is that of the
// longest; with lengths 3 and 4 as well it would exceed two waves per SIMD.
// Passes of 5 fit the usual check interval of 10 exactly.
constexpr int kBatchMaxPass = 5;

// Batch tiles: 256-column strips that own their middle kBatchStrip columns
// (margins of kBatchMargin > every pass length, tile2d_xs.h).
constexpr int kBatchMargin = 8;
constexpr int kBatchStrip = kStripCols - 2 * kBatchMargin;
static_assert(kBatchMargin >= kMaxPass + 1, "batch strip margin");

// Iterations of the pass that starts at iteration k: at most `depth`, never
// past max_iter, and ending before the next gap check (a check falls on the
// first iteration of a pass only).
__host__ __device__ inline int batch_pass_len(int k, int max_iter, int ce,
                                              int depth) {
  int n = max_iter - k < depth ? max_iter - k : depth;
  if (ce > 0) {
    const int to_check = (k / ce + 1) * ce - k;
    if (to_check < n) n = to_check;
  }
  return (n == 3 || n == 4) ? 2 : n;  // lengths 1, 2 and 5 only
}

constexpr int kFinalBlocks = 32;  // blocks per image of the final pass

// Threads per block of the batched drivers: up to 8 waves, so that one
// block per CU holds two waves per SIMD (the grid barrier costs by the
// block, the tile walks gain from the waves).
constexpr int kBatchBlock = 512;

hipError_t launch_batch_init(const BatchArgs& a, const float* g,
                             const int64_t* offs_dev, hipStream_t s);
int batch_persistent_grid(int wpb);
hipError_t launch_batch_persistent(const BatchArgs& a, int grid,
                                   hipStream_t s);
hipError_t launch_batch_sweep(const BatchArgs& a, int grid, bool check,
                              int n, hipStream_t s);
hipError_t launch_batch_final(const BatchArgs& a, float* f_out,
                              const int64_t* offs_dev, hipStream_t s);
int batch_max_blocks_per_cu(int wpb);

}  // namespace tvpd
