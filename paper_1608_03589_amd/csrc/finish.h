// Completion of a plain-solver sweep launch (2D and 3D kernels).
#pragma once

#include "common.h"
#include "sync.h"
#include "tile2d.h"

namespace tvpd {
namespace dev {

// Completion of a sweep of `step` iterations: the last block to finish
// advances k and records the step tau of the iterations made, or on a gap
// check reduces the per-block partials (fixed order, float64), records the
// energies and either freezes k (converged) or advances it.
constexpr int kMaxBlockWaves = kPipeMaxThreads / kWave;
template <bool GAP>
__device__ __forceinline__ void finish_sweep(DevState* st, double* partials,
                                             int k, int step, double acc_gap,
                                             double acc_P, float tau) {
  __shared__ double red[2][kMaxBlockWaves];
  __shared__ int s_last;
  const unsigned nb = gridDim.x;
  if constexpr (GAP) {
    block_sum2(acc_gap, acc_P, red);
    if (threadIdx.x == 0) {
      store_agent(&partials[2 * blockIdx.x], acc_gap);
      store_agent(&partials[2 * blockIdx.x + 1], acc_P);
    }
  }
  // Every wave of the block has read k and finished.  Only thread 0 stored
  // data the last block reads (the partials): its release covers them, and
  // the planes reach the next launch across the kernel boundary.
  __syncthreads();
  if (threadIdx.x == 0) {
    release_agent();
    SyncArea* sa = reinterpret_cast<SyncArea*>(reinterpret_cast<char*>(st) +
                                               kSyncOffset);
    s_last = arrive_last(sa, nb) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  if constexpr (!GAP) {
    if (threadIdx.x == 0) {
      st->k = k + step;
      st->tau_prev = tau;
      st->slot ^= 1;
    }
  } else {
    double sg = 0.0, sp = 0.0;
    for (unsigned i = threadIdx.x; i < nb; i += blockDim.x) {
      sg += load_agent(&partials[2 * i]);
      sp += load_agent(&partials[2 * i + 1]);
    }
    block_sum2(sg, sp, red);
    if (threadIdx.x == 0) {
      st->gap = sg;
      st->P = sp;
      st->D = sp - sg;
      st->checks += 1;
      st->nblocks = (int)nb;
      if (st->tol >= 0.0 && sg <= st->tol * sp) {
        st->converged = 1;
        st->iters = k;
      } else {
        st->k = k + step;
        st->tau_prev = tau;
        st->slot ^= 1;
      }
    }
  }
}

}  // namespace dev

// Workspace regions of the plain solver.
inline DevState* state_of(void* ws) { return reinterpret_cast<DevState*>(ws); }

inline float* planes_of(const Layout& L, void* ws) {
  return reinterpret_cast<float*>(static_cast<char*>(ws) + L.plane_off);
}

inline double* partials_of(const Layout& L, void* ws) {
  return reinterpret_cast<double*>(static_cast<char*>(ws) + L.partial_off);
}

// Blocks for a grid-stride loop over n items.
inline int grid_for(int64_t n, int block, int cap = 8192) {
  const int64_t b = (n + block - 1) / block;
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace tvpd
