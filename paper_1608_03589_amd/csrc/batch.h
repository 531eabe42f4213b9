// Data structures of the batched solver (device side and host side).
#pragma once

#include "common.h"

namespace tvpd {

constexpr int kBatchErrBarrier = 1;  // a grid barrier wait ran out

// Per-image description (device, read-only during a solve).
struct ImgDesc {
  int64_t off;       // float offset of the image's plane block in the arena
  int64_t plane;     // floats per plane
  int32_t ny, nx, pitch;
  int32_t tile_first, tile_count;
  float lam, tau, sigma, theta;
  int32_t pad;
  double tol;        // relative gap tolerance (< 0: never stop)
};

// Per-image result (device).
struct ImgState {
  int32_t converged;
  int32_t iters;
  int32_t pad[2];
  double P, D, gap;
};

struct TileDesc {
  int32_t img, x0, y0, y1;
};

// Batch header at the workspace start (device).
struct BatchHdr {
  int32_t k;             // iteration of the running images
  int32_t n_active;      // entries of the active tile list
  uint32_t bar_count;    // grid barrier arrivals
  uint32_t bar_gen;      // grid barrier generation
  uint32_t blocks_done;  // completion counter (graph-block driver)
  int32_t flags;         // error bits
  int32_t pad[2];
};

struct BatchArgs {
  BatchHdr* hdr;
  const ImgDesc* imgs;
  ImgState* state;
  const TileDesc* tiles;
  int32_t* active;
  double* partials;  // 2 per tile
  float* arena;
  int32_t nimg, ntiles;
  int32_t max_iter, check_every;
  int32_t wpb;
};

hipError_t launch_batch_init(const BatchArgs& a, const float* g,
                             const int64_t* offs_dev, hipStream_t s);
int batch_persistent_grid(int wpb);
hipError_t launch_batch_persistent(const BatchArgs& a, int grid,
                                   hipStream_t s);
hipError_t launch_batch_sweep(const BatchArgs& a, int grid, bool check,
                              hipStream_t s);
hipError_t launch_batch_final(const BatchArgs& a, float* f_out,
                              const int64_t* offs_dev, hipStream_t s);

}  // namespace tvpd
