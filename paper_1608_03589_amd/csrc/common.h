// Internal definitions shared by the HIP kernels and the host entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tvpd.h"

namespace tvpd {

constexpr int kWave = 64;               // CDNA wavefront width
constexpr int kColsPerLane = 4;         // one float4 per lane and row
constexpr int kStripCols = kWave * kColsPerLane;  // columns per wave strip
constexpr int kMaxBlock = 256;          // threads per block (4 waves)
constexpr size_t kHeaderBytes = 4096;   // state header at the workspace start
constexpr size_t kAlign = 256;

// Index of the calling wave in its block as a wave-uniform value.  The
// compiler cannot prove threadIdx.x / 64 uniform, so tile coordinates and
// descriptors derived from it would be kept in vector registers (one copy
// per lane) and the loops bounded by them would be treated as divergent.
__device__ __forceinline__ int wave_in_block() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
}

// Solver state kept in device memory at the start of a workspace.  Kernels
// read k to find the ring slots of the iterates they read and write; the
// last block of every sweep advances k (or freezes it on convergence) and
// records the step tau of the iterations it made (the 2D sweeps form the
// extrapolation of f^k from it).
struct DevState {
  int32_t k;             // index of the current iterate
  int32_t k_end;         // sweeps do nothing once k >= k_end
  int32_t converged;     // set by a passing gap check (k is then frozen)
  int32_t iters;         // k at which the passing check happened
  uint32_t unused0;      // (arrival counters: SyncArea at kSyncOffset)
  int32_t checks;        // number of gap checks performed
  int32_t nblocks;       // block count of the last gap sweep
  int32_t flags;         // device-side error bits (kStateErr*)
  double P, D, gap;      // energies of the last evaluated pair
  double tol;            // relative gap tolerance (< 0: never stop)
  float tau_prev;        // step that produced f^k (0 after initialisation)
  int32_t slot;          // 2D: plane slot of f^k and p^k (flips with every pass)
  double pad[7];
};
static_assert(sizeof(DevState) <= 256, "state header");
// DevState.flags: a wait of a pipelined pass ran out (its iterates are not
// valid; the solve reports TVPD_ERR_DEVICE).
constexpr int32_t kStateErrPipeWait = 1;

// Workspace layout of the plain solver (2D and 3D share it).
struct Layout {
  int ndim;
  int nz, ny, nx;
  int pitch;              // floats per stored row (multiple of 4, >= nx)
  int64_t plane;          // floats per plane (multiple of 64)
  int nplanes;            // kPlainPlanes2D or kPlainPlanes3D
  int64_t max_partials;   // reduction slots (2 doubles each)
  size_t partial_off;     // byte offset of the partials
  size_t plane_off;       // byte offset of plane 0
  size_t bytes;           // total
};

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Longest pass (iterations per launch) of the 2D sweep.  Passes run on
// overlapping strips: a wave loads 256 columns and owns the middle
// xs_owned(n) of them (margins of xs_margin(n) >= n + 1 columns on each
// side, a multiple of 4 for aligned float4 access).
constexpr int kMaxPass = 6;
__host__ __device__ constexpr int xs_margin(int n) { return n <= 3 ? 4 : 8; }
__host__ __device__ constexpr int xs_owned(int n) {
  return kStripCols - 2 * xs_margin(n);
}
// Pipelined passes (tile2d_pipe.h): one block per tile whose waves run one
// stage each, up to kPipeMaxPass iterations per launch, on strips with
// margins of kPipeMargin >= kPipeMaxPass + 1 columns.
constexpr int kPipeMaxPass = 10;
constexpr int kPipeMargin = 12;
constexpr int kPipeOwned = kStripCols - 2 * kPipeMargin;
static_assert(kPipeMargin >= kPipeMaxPass + 1 && kPipeMargin % kColsPerLane == 0,
              "pipelined strip margin");
constexpr int kXsOwnedMin = kPipeOwned < kStripCols - 2 * xs_margin(kMaxPass)
                                ? kPipeOwned
                                : kStripCols - 2 * xs_margin(kMaxPass);
// Threads of a pipelined block: one wave per stage and one for the gap.
constexpr int kPipeMaxThreads = (kPipeMaxPass + 1) * kWave;

// Plane block of the plain 2D solver: two slots, f in plane `slot` and p in
// planes 2 + 2 slot (x) and 3 + 2 slot (y), and g in plane 6.  The slot of
// f^k and p^k is kept with the iteration count (DevState::slot; the batched
// solver's header and, for an image that stopped, its ImgState).  A pass of
// n iterations reads f^k, p^k from one slot and writes f^{k+n}, p^{k+n} to
// the other, so it never overwrites an input that another tile of the same
// pass still reads; the pass that advances k flips the slot.
constexpr int kPlainPlanes2D = 7;
constexpr int kPlainG = 6;
__host__ __device__ inline int plain_f(int slot) { return slot; }
__host__ __device__ inline int plain_p(int slot) { return 2 + 2 * slot; }

// Plane block of the plain 3D solver: f^k in slot k mod 3 (planes 0..2),
// p^k in slot k mod 2 (planes 3 + 3 (k mod 2), x, y, z), g in plane 9.
constexpr int kPlainPlanes3D = 10;
constexpr int kPlainG3D = 9;
__host__ __device__ inline int plain3_f(int k) { return ((k % 3) + 3) % 3; }
__host__ __device__ inline int plain3_p(int k) { return 3 + 3 * (k & 1); }

// Tile configuration of the 2D sweep: each wave owns a strip of 256 columns
// and a band of `th` rows; a block holds `wpb` consecutive wave tiles.
// order 0 numbers tiles band by band (consecutive tiles are horizontally
// adjacent strips: concurrent waves read long contiguous row segments);
// order 1 numbers them strip by strip (consecutive tiles are vertically
// adjacent bands).  order 2 selects the pipelined passes instead: one block
// per tile of kPipeOwned columns and `th` rows, numbered band by band (wpb
// is not used).
constexpr int kOrderPipe = 2;
struct Tile2D {
  int th;
  int wpb;
  int order;
};

// Arguments of the fused 2D sweep kernel (passed by value).
struct Sweep2DArgs {
  float* base;        // plane 0 of the workspace
  int64_t plane;      // floats per plane
  int32_t ny, nx, pitch;
  int32_t th, wpb, order;
  int32_t ntx, nty, ntiles;  // wave tiles: ntx strips by nty row bands
  int32_t n;                 // iterations of the pass (pipelined kernel)
  float lam, tau, sigma, theta;
  DevState* st;
  double* partials;   // 2 doubles per block (gap, P)
  int64_t wait_limit; // polls before a wait of the pipelined kernel gives up
};

// Tile configuration of the 3D sweep: each wave owns a strip of 256 columns,
// a band of `th` rows (2 or 4) and a segment of `tz` planes; a block holds
// `wpb` consecutive wave tiles, numbered strip fastest, then band, then
// segment.
struct Tile3D {
  int th;
  int tz;
  int wpb;
};

// Arguments of the fused 3D sweep kernel (passed by value).
struct Sweep3DArgs {
  float* base;
  int64_t plane;
  int32_t nz, ny, nx, pitch;
  int32_t tz, wpb;
  int32_t ntx, nty, ntz, ntiles;
  float lam, tau, sigma, theta;
  DevState* st;
  double* partials;
};

// Host launchers (kernels2d.hip).
hipError_t launch_init2d(const Layout& L, const float* g, void* ws,
                         hipStream_t s);
// One launch of n iterations (n = 1 .. kMaxPass, temporally blocked for
// n >= 2).  Gap check, if any, on the first iteration.
hipError_t launch_sweep2d(const Layout& L, const Tile2D& t,
                          const tvpd_coeffs& c, bool with_gap, int n,
                          void* ws, hipStream_t s);
hipError_t launch_read2d(const Layout& L, const void* ws, float* f_out,
                         float* p_out, hipStream_t s);
hipError_t launch_energy2d(const Layout& L, float lam, void* ws,
                           bool skip_if_converged, hipStream_t s);
hipError_t launch_stream_copy(const float* src, float* dst, int64_t n, hipStream_t s);
hipError_t launch_set_params(void* ws, int32_t k_end, double tol,
                             hipStream_t s);
int sweep2d_blocks(const Layout& L, const Tile2D& t, int n);
hipError_t launch_energy_final(const Layout& L, void* ws, int nparts,
                               bool skip_if_converged, hipStream_t s);

// Host launchers (kernels3d.hip).
hipError_t launch_init3d(const Layout& L, const float* g, void* ws,
                         hipStream_t s);
hipError_t launch_sweep3d(const Layout& L, const Tile3D& t,
                          const tvpd_coeffs& c, bool with_gap, void* ws,
                          hipStream_t s);
hipError_t launch_read3d(const Layout& L, const void* ws, float* f_out,
                         float* p_out, hipStream_t s);
hipError_t launch_energy3d(const Layout& L, float lam, void* ws,
                           bool skip_if_converged, hipStream_t s);
int sweep3d_blocks(const Layout& L, const Tile3D& t);
bool tile3d_ok(const Tile3D& t);

// Tile table and autotuner (autotune.hip).
Tile2D default_tile2d(const Layout& L);
Tile2D tile2d_for(const Layout& L);
void remember_tile2d(const tvpd_shape& s, const Tile2D& t);
int autotune2d(const tvpd_shape& sh, const Layout& L, void* ws, hipStream_t s,
               Tile2D* best, float* best_us);
Tile3D default_tile3d(const Layout& L);
Tile3D tile3d_for(const Layout& L);
void remember_tile3d(const tvpd_shape& s, const Tile3D& t);
int autotune3d(const tvpd_shape& sh, const Layout& L, void* ws, hipStream_t s,
               Tile3D* best, float* best_us);
int tune_save(const char* path, const tvpd_shape& s, const Tile2D& t, float us);
int tune_save3d(const char* path, const tvpd_shape& s, const Tile3D& t,
                float us);
int tune_load(const char* path, int* count);
// Longest pass of the plain 2D sweep (api.hip): 0 = each kernel's own
// default, else the process-wide setting, capped by the kernel in use.
int pass_depth();
int walk_depth();         // strip walks (tile2d_xs.h): 1 .. kMaxPass
int pipe_depth();         // pipelined passes (tile2d_pipe.h): 1 .. kPipeMaxPass
int64_t pipe_wait_limit();  // polls per bounded wait of the pipelined passes

// Host resources a driver keeps for polling device state while further work
// is queued: pinned staging for two copies of a header, two events and a
// stream for graph capture, all owned by one host thread and created on one
// device (api.hip).
struct HostPoll {
  int device = -1;
  void* host = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipStream_t capture = nullptr;
  bool ok = false;
};
// Make p hold resources for the current device with `host_bytes` of pinned
// staging; resources held for another device are released first (with that
// device current).  On failure everything is released.
int host_poll_get(HostPoll& p, size_t host_bytes);
// Release whatever p holds; p is then empty and may be reused.
void host_poll_release(HostPoll& p);
// Release the calling thread's batch-driver resources (batch_api.hip).
void release_batch_thread_resources();

}  // namespace tvpd
