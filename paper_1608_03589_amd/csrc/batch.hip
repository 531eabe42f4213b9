// Batched solver: many 2D images of different sizes solved together, each
// exactly as the plain solver would solve it alone (same per-pixel
// arithmetic, same stopping rule, its own stopping iteration).
//
// All images live in one arena; a tile table lists every (image, strip,
// band) tile, and an active list holds the tiles of the images that have not
// stopped.  All running images are at the same iteration k, so the plane
// slots are shared (batch.h); an image that stops at k keeps f^k in its slot
// and is dropped from the active list before a pass could overwrite it.
//
// Two drivers share the tile code:
//  - persistent: one cooperative launch runs every iteration; waves take
//    shares of the active tiles and a grid barrier separates passes.  The
//    gaps of a check are reduced and the stopping rule applied by one wave
//    per image during the next pass, and the stopped images leave the active
//    list after that pass's barrier, so a check costs no barrier of its own;
//  - graph blocks: one launch per iteration over the active list, the last
//    block to finish doing the per-image bookkeeping; launches are replayed
//    from HIP graphs of check_every iterations.
#include "batch.h"
#include "sync.h"
#include "tile2d.h"
#include "tile2d_xs.h"

namespace tvpd {
namespace {

using namespace dev;

constexpr long kSpinLimit = 1L << 22;  // polls (seconds of them) before giving up
// Set in the barrier generation word by a block whose wait ran out, so that
// every waiting block leaves at its next poll.
constexpr unsigned kGenError = 0x80000000u;

__device__ __forceinline__ int load_i32(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ SyncArea* sync_of(BatchHdr* h) {
  return reinterpret_cast<SyncArea*>(reinterpret_cast<char*>(h) + kSyncOffset);
}

// Grid-wide barrier for a co-resident grid (hierarchical arrival, one
// generation word polled with a short sleep; the ordering of sync.h: every
// wave's stores in L2, one release per block before arriving, one acquire
// per block after the generation moves).  Every wait is bounded: after
// kSpinLimit polls the barrier flags an error, marks the generation word and
// every block leaves.
__device__ bool grid_barrier(BatchHdr* h, unsigned& gen) {
  __shared__ int s_ok;
  wait_vmem();
  __syncthreads();
  if (threadIdx.x == 0) {
    SyncArea* sa = sync_of(h);
    release_agent();
    const unsigned g = gen;
    unsigned seen;
    if (arrive_last(sa, gridDim.x)) {
      seen = atomicAdd(&sa->gen.v, 1u) + 1u;
    } else {
      long spins = 0;
      while ((seen = __hip_atomic_load(&sa->gen.v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT)) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          atomicOr(&h->flags, kBatchErrBarrier);
          atomicOr(&sa->gen.v, kGenError);
          seen = kGenError;
          break;
        }
      }
      acquire_agent();
    }
    gen = g + 1;
    s_ok = (seen & kGenError) ? 0 : 1;
  }
  __syncthreads();
  return s_ok != 0;
}

// Sweep one tile by pass `pass` of n iterations k -> k+n (tile2d_xs.h,
// strips of kBatchStrip owned columns), reading the pass's plane slots and
// writing the next ones (batch.h); on check iterations lane 0 stores the
// tile's partials (the gap of (f^k, p^k)) in the pass parity's pair.
template <int N, bool CHECK>
__device__ __forceinline__ void tile_pass(const BatchArgs& a,
                                          const TileDesc& T, int pass,
                                          double& sg, double& sp) {
  const ImgDesc& D = a.imgs[T.img];
  float* base = a.arena + D.off;
  const int64_t PL = D.plane;
  const int fs = batch_fslot(pass), ps = batch_pslot(pass);
  TileCtxS c;
  c.F = base + batch_f(fs) * PL;
  c.FN = base + batch_f(fs == 2 ? 0 : fs + 1) * PL;
  c.PX = base + batch_p(ps) * PL;
  c.PY = c.PX + PL;
  c.QX = base + batch_p(ps ^ 1) * PL;
  c.QY = c.QX + PL;
  c.G = base + kBatchG * PL;
  c.ny = D.ny;
  c.nx = D.nx;
  c.pitch = D.pitch;
  c.x0 = T.x0;
  c.y0 = T.y0;
  c.y1 = T.y1;
  c.lam = D.lam;
  c.tau = D.tau;
  c.sig = D.sigma;
  c.th = D.theta;
  c.tau_prev = D.tau;   // every step of an image has its tau (at k = 0 any value)
  sweep_tile_xs<N, kBatchMargin, CHECK, false>(c, sg, sp);
}

// The waves' share of the active list.  The list is cut into one
// contiguous chunk per XCD (blocks are dealt to the 8 XCDs round-robin), so
// that bands sharing halo rows meet in one L2; inside a chunk consecutive
// tiles go to the XCD's blocks before their further waves, so that a short
// list (the last images of a batch) spreads over every CU at one wave per
// SIMD instead of stacking the waves of a few CUs.  A wave sweeps tiles
// active[base + j] for j = first, first + step, ... below end.
struct TileShare {
  int base, first, step, end;
};

__device__ __forceinline__ TileShare tile_share(int nact, int wave, int wpb) {
  const int nb = gridDim.x;
  const int nx = (nb % kSyncGroups == 0) ? kSyncGroups : 1;
  const int per = (nact + nx - 1) / nx;  // tiles per chunk
  const int bx = nb / nx;                // blocks per chunk
  TileShare r;
  r.base = (blockIdx.x % nx) * per;
  r.first = wave * bx + blockIdx.x / nx;
  r.step = wpb * bx;
  r.end = min(per, nact - r.base);
  return r;
}

// Partials of tile t from a check in a pass of parity `par`: (gap, P).
__device__ __forceinline__ double* tile_partials(const BatchArgs& a, int t,
                                                 int par) {
  return a.partials + 4 * (int64_t)t + 2 * par;
}

template <bool CHECK>
__device__ __forceinline__ void do_tile(const BatchArgs& a, int t, int pass,
                                        int n) {
  const TileDesc T = a.tiles[t];
  double sg = 0.0, sp = 0.0;
  switch (n) {
    case 1: tile_pass<1, CHECK>(a, T, pass, sg, sp); break;
    case 2: tile_pass<2, CHECK>(a, T, pass, sg, sp); break;
    default: tile_pass<5, CHECK>(a, T, pass, sg, sp); break;
  }
  static_assert(kBatchMaxPass == 5, "one case per pass length");
  if (CHECK) {
    sg = wave_sum(sg);
    sp = wave_sum(sp);
    if ((threadIdx.x & (kWave - 1)) == 0) {
      double* q = tile_partials(a, t, pass & 1);
      store_agent(q, sg);
      store_agent(q + 1, sp);
    }
  }
}

// Reduce the gap partials of image i from the check at iteration k, made
// in pass `pass` with tile table `tbl`, in a fixed order (one wave), and
// apply the stopping rule; lane 0 updates the image state.
__device__ void reduce_image(const BatchArgs& a, int i, int k, int pass,
                             int tbl) {
  const ImgDesc& D = a.imgs[i];
  const int first = D.tile_first[tbl], count = D.tile_count[tbl];
  const int lane = threadIdx.x & (kWave - 1);
  double sg = 0.0, sp = 0.0;
  for (int j = lane; j < count; j += kWave) {
    const double* q = tile_partials(a, first + j, pass & 1);
    sg += load_agent(q);
    sp += load_agent(q + 1);
  }
  sg = wave_sum(sg);
  sp = wave_sum(sp);
  if (lane == 0) {
    ImgState& S = a.state[i];
    S.gap = sg;
    S.P = sp;
    S.D = sp - sg;
    if (D.tol >= 0.0 && sg <= D.tol * sp) {
      S.converged = 1;
      S.iters = k;
      S.fslot = batch_fslot(pass);
      atomicOr(&a.hdr->flags, kBatchStopped);  // the active list must shrink
    }
  }
}

// Tiles of table `tbl` over the images that still run.
__device__ int running_tiles(const BatchArgs& a, int tbl) {
  int n = 0;
  for (int i = 0; i < a.nimg; ++i)
    if (!a.state[i].converged) n += a.imgs[i].tile_count[tbl];
  return n;
}

// Rebuild the active tile list from the images that still run (one block).
// Once fewer tall-band tiles than SIMD slots (switch_tiles) remain, switch
// for good to the first short-band table, and from there to a table of
// shorter bands whenever its tiles still fit the slots: the iterates do not depend on the
// tiling, and a shorter band is a shorter serial walk for its wave, which
// is what a pass costs while only a few images are left.
__device__ void compact_active(const BatchArgs& a) {
  __shared__ int s_pos;
  __shared__ int s_tbl;
  if (threadIdx.x == 0) {
    int tbl = a.hdr->table;
    if (tbl == 0 && running_tiles(a, 0) < a.switch_tiles) tbl = 1;
    while (tbl >= 1 && tbl + 1 < kBatchTables &&
           running_tiles(a, tbl + 1) <= a.switch_tiles)
      ++tbl;
    a.hdr->table = tbl;
    s_tbl = tbl;
    s_pos = 0;
  }
  __syncthreads();
  const int tbl = s_tbl;
  for (int i = 0; i < a.nimg; ++i) {
    const ImgDesc& D = a.imgs[i];
    const int conv = a.state[i].converged;
    const int pos = s_pos;
    const int first = D.tile_first[tbl], count = D.tile_count[tbl];
    if (!conv)
      for (int j = threadIdx.x; j < count; j += blockDim.x)
        a.active[pos + j] = first + j;
    __syncthreads();
    if (threadIdx.x == 0 && !conv) s_pos = pos + count;
    __syncthreads();
  }
  // (the grid barrier or the kernel boundary that follows a rebuild
  // publishes the list and its length)
  if (threadIdx.x == 0)
    __hip_atomic_store(&a.hdr->n_active, s_pos, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
}

__global__ __launch_bounds__(kBatchBlock) void batch_persistent_kernel(
    BatchArgs a) {
  BatchHdr* h = a.hdr;
  unsigned gen = __hip_atomic_load(&sync_of(h)->gen.v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
  const int wave = wave_in_block();
  int k = 0, pass = 0;
  // the active list and its table change only when an image stops
  int nact = load_i32(&h->n_active);
  int tbl = load_i32(&h->table);
  // the check whose stopping decisions are being made: iteration, pass and
  // tile table (ck < 0: none)
  int ck = -1, cpass = 0, ctbl = 0;
  while (k < a.max_iter) {
    if (nact == 0) break;
    const bool check = a.check_every > 0 && (k % a.check_every) == 0;
    const int n = batch_pass_len(k, a.max_iter, a.check_every, a.depth);
    // the last wave of a block decides its images before taking tiles; the
    // pass writes f slot pass+1 mod 3, so f^ck of a stopped image survives
    if (ck >= 0 && wave == a.wpb - 1)
      for (int i = blockIdx.x; i < a.nimg; i += gridDim.x)
        if (!a.state[i].converged) reduce_image(a, i, ck, cpass, ctbl);
    if (wave < a.wpb) {
      const TileShare r = tile_share(nact, wave, a.wpb);
      for (int j = r.first; j < r.end; j += r.step) {
        if (check)
          do_tile<true>(a, a.active[r.base + j], pass, n);
        else
          do_tile<false>(a, a.active[r.base + j], pass, n);
      }
    }
    if (!grid_barrier(h, gen)) return;
    if (ck >= 0) {
      // the decisions are out: rebuild the active list if an image stopped
      ck = -1;
      if (load_i32(&h->flags) & kBatchStopped) {
        if (!grid_barrier(h, gen)) return;  // every block has read the flag
        if (blockIdx.x == 0) {
          compact_active(a);
          if (threadIdx.x == 0) atomicAnd(&h->flags, ~kBatchStopped);
        }
        if (!grid_barrier(h, gen)) return;
        nact = load_i32(&h->n_active);
        tbl = load_i32(&h->table);
      }
    }
    if (check) {
      ck = k;
      cpass = pass;
      ctbl = tbl;
    }
    k += n;
    ++pass;
  }
  // a check in the last pass is decided here (the final kernel follows)
  if (ck >= 0 && wave == a.wpb - 1)
    for (int i = blockIdx.x; i < a.nimg; i += gridDim.x)
      if (!a.state[i].converged) reduce_image(a, i, ck, cpass, ctbl);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    h->k = k;
    h->pass = pass;
  }
}

// One pass of n iterations over the active list (graph-block driver).  The
// last block to finish advances k and, on check iterations, reduces every
// running image, stops the converged ones and rebuilds the active list.
template <bool CHECK>
__global__ __launch_bounds__(kBatchBlock) void batch_sweep_kernel(BatchArgs a,
                                                                  int n) {
  __shared__ int s_last;
  BatchHdr* h = a.hdr;
  const int k = h->k;
  if (k + n > a.max_iter) return;
  const int pass = h->pass;
  const int nact = h->n_active;
  if (nact == 0) return;
  const int wave = wave_in_block();
  if (wave < a.wpb) {
    const TileShare r = tile_share(nact, wave, a.wpb);
    for (int j = r.first; j < r.end; j += r.step)
      do_tile<CHECK>(a, a.active[r.base + j], pass, n);
  }
  // the partials of every wave in L2, one release per block (sync.h); the
  // last block acquires in arrive_last, the planes reach the next launch
  // across the kernel boundary
  wait_vmem();
  __syncthreads();
  if (threadIdx.x == 0) {
    release_agent();
    s_last = arrive_last(sync_of(h), gridDim.x) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  if (CHECK) {
    const int tbl = h->table;
    if (wave < a.wpb)
      for (int i = wave; i < a.nimg; i += a.wpb)
        if (!a.state[i].converged) reduce_image(a, i, k, pass, tbl);
    wait_vmem();
    __syncthreads();
    if (load_i32(&h->flags) & kBatchStopped) {
      compact_active(a);
      if (threadIdx.x == 0) atomicAnd(&h->flags, ~kBatchStopped);
    }
  }
  if (threadIdx.x == 0) {
    h->k = k + n;
    h->pass = pass + 1;
  }
}

__global__ void batch_init_kernel(BatchArgs a, const float* __restrict__ g,
                                  const int64_t* __restrict__ offs) {
  const int i = blockIdx.y;
  const ImgDesc& D = a.imgs[i];
  float* base = a.arena + D.off;
  const int64_t PL = D.plane;
  const int64_t n = (int64_t)D.ny * D.pitch;
  const float* gi = g + offs[i];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(e / D.pitch);
    const int x = (int)(e - (int64_t)y * D.pitch);
    const float v = (x < D.nx) ? gi[(int64_t)y * D.nx + x] : 0.0f;
    for (int s = 0; s < kBatchPlanes; ++s) base[s * PL + e] = 0.0f;
    base[batch_f(batch_fslot(0)) * PL + e] = v;  // f^0
    base[kBatchG * PL + e] = v;                  // g
  }
}

// Energies of the final pair of every image that did not stop, and the
// read-out of every image's returned iterate: kFinalBlocks blocks per image
// write float64 partials, then one block per image sums them in order.
__global__ __launch_bounds__(kMaxBlock) void batch_final_kernel(
    BatchArgs a, float* __restrict__ f_out, const int64_t* __restrict__ offs) {
  __shared__ double red[2][kMaxBlock / kWave];
  const int i = blockIdx.y;
  const ImgDesc& D = a.imgs[i];
  const ImgState& S = a.state[i];
  const int conv = S.converged;
  const int pass = a.hdr->pass;
  const float* base = a.arena + D.off;
  const int64_t PL = D.plane;
  const float* f = base + batch_f(conv ? S.fslot : batch_fslot(pass)) * PL;
  const float* px = base + batch_p(batch_pslot(pass)) * PL;  // (running only)
  const float* py = px + PL;
  const float* g = base + kBatchG * PL;
  const int64_t n = (int64_t)D.ny * D.nx;
  const int P = D.pitch;
  double sg = 0.0, sp = 0.0;
  float* fo = f_out + offs[i];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(e / D.nx);
    const int x = (int)(e - (int64_t)y * D.nx);
    const int64_t s = (int64_t)y * P + x;
    fo[e] = f[s];
    if (!conv) {
      const double fv = f[s];
      const double gx = (x < D.nx - 1) ? (double)f[s + 1] - fv : 0.0;
      const double gy = (y < D.ny - 1) ? (double)f[s + P] - fv : 0.0;
      const double dxl = (x > 0) ? (double)px[s - 1] : 0.0;
      const double dyl = (y > 0) ? (double)py[s - P] : 0.0;
      const double d = ((double)px[s] - dxl) + ((double)py[s] - dyl);
      const double ee = fv - (double)g[s];
      const double r = ee - d;
      const double nrm = sqrt(gx * gx + gy * gy);
      sg += 0.5 * r * r + (double)D.lam * nrm - (gx * px[s] + gy * py[s]);
      sp += 0.5 * ee * ee + (double)D.lam * nrm;
    }
  }
  block_sum2(sg, sp, red);
  if (threadIdx.x == 0) {
    a.fparts[2 * (i * kFinalBlocks + blockIdx.x)] = sg;
    a.fparts[2 * (i * kFinalBlocks + blockIdx.x) + 1] = sp;
  }
}

__global__ void batch_final_reduce_kernel(BatchArgs a) {
  const int i = blockIdx.x;
  if (threadIdx.x != 0) return;
  ImgState& S = a.state[i];
  if (S.converged) return;
  double sg = 0.0, sp = 0.0;
  for (int b = 0; b < kFinalBlocks; ++b) {
    sg += a.fparts[2 * (i * kFinalBlocks + b)];
    sp += a.fparts[2 * (i * kFinalBlocks + b) + 1];
  }
  S.gap = sg;
  S.P = sp;
  S.D = sp - sg;
  S.iters = a.hdr->k;
}

}  // namespace

hipError_t launch_batch_init(const BatchArgs& a, const float* g,
                             const int64_t* offs_dev, hipStream_t s) {
  dim3 grid(64, a.nimg);
  hipLaunchKernelGGL(batch_init_kernel, grid, dim3(256), 0, s, a, g, offs_dev);
  return hipGetLastError();
}

int batch_persistent_grid(int wpb) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(batch_persistent_kernel),
          wpb * kWave, 0) != hipSuccess)
    return 0;
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipGetDeviceProperties(&p, dev) != hipSuccess)
    return 0;
  return per_cu * p.multiProcessorCount;
}

hipError_t launch_batch_persistent(const BatchArgs& a, int grid,
                                   hipStream_t s) {
  BatchArgs arg = a;
  void* params[] = {&arg};
  return hipLaunchCooperativeKernel(
      reinterpret_cast<const void*>(batch_persistent_kernel), dim3(grid),
      dim3(a.wpb * kWave), params, 0, s);
}

hipError_t launch_batch_sweep(const BatchArgs& a, int grid, bool check,
                              int n, hipStream_t s) {
  if (n != 1 && n != 2 && n != kBatchMaxPass) return hipErrorInvalidValue;
  const dim3 g(grid), blk(a.wpb * kWave);
  if (check)
    hipLaunchKernelGGL((batch_sweep_kernel<true>), g, blk, 0, s, a, n);
  else
    hipLaunchKernelGGL((batch_sweep_kernel<false>), g, blk, 0, s, a, n);
  return hipGetLastError();
}

hipError_t launch_batch_final(const BatchArgs& a, float* f_out,
                              const int64_t* offs_dev, hipStream_t s) {
  hipLaunchKernelGGL(batch_final_kernel, dim3(kFinalBlocks, a.nimg),
                     dim3(kMaxBlock), 0, s, a, f_out, offs_dev);
  hipLaunchKernelGGL(batch_final_reduce_kernel, dim3(a.nimg), dim3(64), 0, s,
                     a);
  return hipGetLastError();
}

int batch_max_blocks_per_cu(int wpb) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(batch_persistent_kernel),
          wpb * kWave, 0) != hipSuccess)
    return 0;
  return per_cu;
}

}  // namespace tvpd
