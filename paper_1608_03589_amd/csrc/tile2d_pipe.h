// A pass of n iterations of the 2D sweep over one tile, pipelined across the
// waves of a block: wave w runs stage w+1 (iteration k+w -> k+w+1) of the
// strip walk of tile2d_xs.h and hands its rows to the next stage through
// LDS.  The arithmetic of every stage is the walk's, operation for
// operation, so a pipelined pass gives the walk's iterates bit for bit.
//
// Why: the walk keeps every stage of a wave's column strip in that wave's
// registers, which caps a pass at about five iterations; here a wave holds
// one stage, so a pass can span a whole check interval (up to kPipeMaxPass
// iterations), and the 28 bytes per pixel a pass moves are shared by that
// many iterations.  One block per tile also makes the bands tall (a few
// blocks per strip for the whole image), so the band halo of 2n + 1 rows
// costs little.
//
// Schedule.  At its step t wave 0 takes in row q = tb + t + 1 of f^k, p^k,
// g and runs stage 1 on row q - 1; wave w > 0 takes in row tb + t - 2w + 1
// of stage w's output and runs stage w+1 on row tb + t - 2w, two rows behind
// the stage before it.  Stage s is needed on rows [y0-n+s-1, y1+n-s-1]
// (tb = y0-n-1), exactly as in the walk, and the last stage stores
// f^{k+n}, p^{k+n} of the band's rows and owned columns.  A stage passes on
// its iterate, its fbar and g.  A gap check adds one wave that evaluates
// the gap density and primal energy of (f^k, p^k) on the band's rows.
//
// Loads.  Wave 0 keeps kPipeAhead rows of f^k, p^k, g in flight in
// registers (its loop is unrolled over the buffers, so the compiler waits
// for the oldest row only): with a pipeline stage per wave a step is short,
// and a memory latency takes several steps.  (A pass of one iteration runs
// as a walk instead, bit for bit the same.)
//
// Synchronisation is point to point, through a progress count per wave in
// LDS (steps finished): a wave starts step t once the wave feeding it has
// finished step t-1 and the waves it feeds have finished step t-1 (the ring
// slot it is about to write was last read at their step t-1).  Every (wave,
// step) waits only on neighbouring waves' earlier steps, so the block
// cannot deadlock; there is no block barrier inside the pass (a barrier
// would wait for the loads in flight).
//
// LDS (float rows of 256 columns): for each stage boundary two slots of
// five rows (f, p_x, p_y, g, fbar: a row written at step t is read at t+1
// and overwritten at t+2); with the gap, two slots of four rows (f^k,
// p_x^k, p_y^k, g) for the gap wave; then the progress counts.
#pragma once

#include "tile2d.h"

namespace tvpd {
namespace dev {

constexpr int kPipeRow = kStripCols;  // floats per LDS row
constexpr int kPipeAhead = 4;         // rows in flight ahead of the one taken in
constexpr int kPipeBufs = kPipeAhead + 1;  // wave 0's row buffers
constexpr int kPipeCounts = 16;       // progress counts (>= kPipeMaxPass + 1)
static_assert(kPipeCounts >= kPipeMaxPass + 2, "progress counts and abort flag");

constexpr int kPipeArrays = 5;        // rows per ring slot: f, p_x, p_y, g, fbar
constexpr int kPipeSlots = 2;         // slots per ring: a producer runs up to
                                      // kPipeSlots - 1 steps ahead of its
                                      // readers (three slots measured slower)

__host__ __device__ constexpr int pipe_lds_floats(int n) {
  return ((n - 1) * kPipeSlots * kPipeArrays + kPipeSlots * 4) * kPipeRow +
         kPipeCounts;
}

struct PipeCtx {
  const float* F;   // f^k
  const float* PX;  // p^k
  const float* PY;
  const float* G;
  float* FN;        // f^{k+n}
  float* QX;        // p^{k+n}
  float* QY;
  int ny, nx, pitch;
  int x0, y0, y1;   // owned columns [x0, x0+kPipeOwned), rows [y0, y1)
  int n;            // iterations of the pass, 1 .. kPipeMaxPass
  float lam, tau, sig, th;
  float tau_prev;   // the step that produced f^k (any value at k = 0)
  int* err;         // device error bits: kStateErrPipeWait if a wait ran out
  int64_t wait_limit;  // polls before a wait gives up
};

__device__ __forceinline__ void lds_st4(float* p, const F4& a) {
  *reinterpret_cast<float4*>(p) = make_float4(a.v[0], a.v[1], a.v[2], a.v[3]);
}
__device__ __forceinline__ F4 lds_ld4(const float* p) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  F4 r;
  r.v[0] = t.x;
  r.v[1] = t.y;
  r.v[2] = t.z;
  r.v[3] = t.w;
  return r;
}

// s_waitcnt with lgkmcnt 0 and the other counters at their maxima (vmcnt
// 63, expcnt 7): wait for this wave's LDS operations only.
constexpr int kWaitLgkm0 = 0xC07F;
// s_waitcnt with vmcnt v (6 bits: [3:0] and [15:14]) and the other counters
// at their maxima.
__host__ __device__ constexpr int waitcnt_vm(int v) {
  return (v & 0xF) | ((v >> 4) << 14) | (0x7 << 4) | (0xF << 8);
}

// One row of a stage's input: the iterate (f, p_x, p_y) and g.
struct PipeRowIn {
  F4 f, px, py, g;
};

template <bool GAP>
__device__ __forceinline__ void sweep_tile_pipe(const PipeCtx& c, float* lds,
                                                double& acc_gap,
                                                double& acc_P) {
  const int w = wave_in_block();
  const int lane = threadIdx.x & (kWave - 1);
  const int n = c.n;
  const int nx = c.nx, ny = c.ny, x0 = c.x0, y0 = c.y0, y1 = c.y1;
  const int64_t P = c.pitch;
  const int xg = x0 - kPipeMargin + kColsPerLane * lane;
  const int xcl = min(max(xg, 0), c.pitch - kColsPerLane);
  const bool owned = xg >= x0 && xg < x0 + kPipeOwned && xg < c.pitch;
  const float lam = c.lam, tau = c.tau, sig = c.sig, th = c.th;
  const float iopt = prox_factor(tau);
  const float thtau = th * tau;          // fbar of the iterates this pass makes
  const float thtau0 = th * c.tau_prev;  // fbar^k
  const int tb = y0 - n - 1;
  // the last stage finishes row y1-1 at step h + 3n - 2, the gap wave at
  // step h + n + 1 (later only for n = 1)
  const int h = y1 - y0;
  const int steps = (GAP && n == 1) ? h + 3 : h + 3 * n - 1;

  // LDS: stage rings, the gap wave's ring, progress counts (rows >= tb, so
  // the slots are non-negative)
  float* const in_ring = lds + (n - 1) * kPipeSlots * kPipeArrays * kPipeRow;
  int* const prog = reinterpret_cast<int*>(in_ring + kPipeSlots * 4 * kPipeRow);
  int* const abort_flag = prog + (kPipeCounts - 1);
  const int col = kColsPerLane * lane;
  auto ring_row = [&](int b, int row, int arr) {
    const int slot = (unsigned)(row - tb) % kPipeSlots;
    return lds + ((b * kPipeSlots + slot) * kPipeArrays + arr) * kPipeRow + col;
  };
  auto in_row = [&](int row, int arr) {
    return in_ring + (((unsigned)(row - tb) % kPipeSlots) * 4 + arr) * kPipeRow + col;
  };
  auto ld_ring = [&](int b, int row, PipeRowIn& R, F4& fb) {
    R.f = lds_ld4(ring_row(b, row, 0));
    R.px = lds_ld4(ring_row(b, row, 1));
    R.py = lds_ld4(ring_row(b, row, 2));
    R.g = lds_ld4(ring_row(b, row, 3));
    fb = lds_ld4(ring_row(b, row, 4));
  };

  // wait until wave v has finished `t` steps.  Bounded: a wait that runs
  // out raises the block's abort flag, after which no wait waits, so the
  // pass ends instead of hanging, and the block records the error in the
  // device state (its results are not valid).
  auto wait_for = [&](int v, int t) {
    int64_t spins = 0;
    while (__hip_atomic_load(&prog[v], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP) < t) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_WORKGROUP) != 0)
        break;
      if (++spins > c.wait_limit) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    // (no reads of the rings move above the poll)
    __asm__ __volatile__("" ::: "memory");
  };
  // publish that this wave has finished `t` steps: its LDS writes complete
  // first (LDS serves one CU's waves in order, so a count seen by another
  // wave comes after the rows).  Only LDS ordering is needed here: a
  // workgroup fence would also wait for the loads in flight.
  auto post = [&](int t) {
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __asm__ __volatile__("" ::: "memory");
    if (lane == 0)
      __hip_atomic_store(&prog[w], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  if (threadIdx.x < kPipeCounts) prog[threadIdx.x] = 0;
  __syncthreads();

  // fbar of row y from the row's iterate and g (R) and p_y of the row above
  // (pya): the extrapolation from the data prox, with the operations of the
  // stage that produced the row (thtau_r: theta tau of that stage).
  auto fbar_of = [&](int y, const PipeRowIn& R, const F4& pya, float thtau_r,
                     F4& out) {
    const bool up = y > 0;
    const float pl = from_left(R.px.v[3]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float lp = (j == 0) ? ((xg > 0) ? pl : 0.0f) : R.px.v[j - 1];
      const float d = (R.px.v[j] - lp) + (R.py.v[j] - (up ? pya.v[j] : 0.0f));
      out.v[j] = extrap_prox(R.f.v[j], R.g.v[j], d, thtau_r);
    }
  };

  // Stage on row r from fbar of rows r (cb) and r+1 (nb), the stage's input
  // row r (I) and p_y of row r-1 of this stage's own output (cyv): the
  // walk's per-stage update with its border masks.
  auto stage = [&](int r, const F4& cb, const F4& nb, const PipeRowIn& I,
                   const F4& cyv, F4& fnew, F4& fbnew, F4& npx, F4& npy) {
    const bool dn = r + 1 < ny;
    const float nbr = from_right(cb.v[0]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float right = (j < 3) ? cb.v[j + 1] : nbr;
      const float gx = (xg + j < nx - 1) ? right - cb.v[j] : 0.0f;
      const float gy = dn ? nb.v[j] - cb.v[j] : 0.0f;
      project2(dual_arg(I.px.v[j], sig, gx), dual_arg(I.py.v[j], sig, gy), lam,
               npx.v[j], npy.v[j]);
    }
    const float left = from_left(npx.v[3]);
    const bool up = r > 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float lp = (j == 0) ? ((xg > 0) ? left : 0.0f) : npx.v[j - 1];
      const float d = (npx.v[j] - lp) + (npy.v[j] - (up ? cyv.v[j] : 0.0f));
      fnew.v[j] = data_prox(I.f.v[j], I.g.v[j], d, tau, iopt);
      fbnew.v[j] = extrap_prox(fnew.v[j], I.g.v[j], d, thtau);
    }
  };

  // The last stage's rows inside the band go to HBM, the others to the ring.
  auto emit = [&](int s, int r, const F4& fnew, const F4& fbnew, const F4& npx,
                  const F4& npy, const F4& gv) {
    if (s == n) {
      if (owned && r >= y0 && r < y1) {
        const int64_t o = (int64_t)r * P + xg;
        st4(c.FN + o, fnew);
        st4(c.QX + o, npx);
        st4(c.QY + o, npy);
      }
    } else {
      lds_st4(ring_row(s - 1, r, 0), fnew);
      lds_st4(ring_row(s - 1, r, 1), npx);
      lds_st4(ring_row(s - 1, r, 2), npy);
      lds_st4(ring_row(s - 1, r, 3), gv);
      lds_st4(ring_row(s - 1, r, 4), fbnew);
    }
  };

  if (w == 0) {
    // Stage 1 (n >= 2, so it feeds the ring).  Row tb + j of f^k, p^k, g is
    // loaded into buf[j % kPipeBufs] kPipeAhead steps before it is taken in
    // and stays there while stage 1 runs on it; the loop is unrolled over the
    // buffers, so no loaded register is moved and the compiler waits for the
    // oldest row only (rows outside the image are clamped re-reads).
    auto load = [&](int y, PipeRowIn& L) {
      const int64_t o = (int64_t)min(max(y, 0), ny - 1) * P + xcl;
      L.f = ld4(c.F + o);
      L.px = ld4(c.PX + o);
      L.py = ld4(c.PY + o);
      L.g = ld4(c.G + o);
    };
    // the waves wave 0 feeds have read the slot it is about to write
    auto wait_readers = [&](int t) {
      wait_for(1, t + 2 - kPipeSlots);
      if (GAP) wait_for(n, t + 2 - kPipeSlots);
    };
    PipeRowIn buf[kPipeBufs];
#pragma unroll
    for (int i = 0; i < kPipeBufs; ++i) load(tb + i, buf[i]);
    F4 fbc, cy = zero4();
    fbar_of(tb, buf[0], zero4(), thtau0, fbc);
    // step t: take in row q = tb + t + 1 (in) and run stage 1 on row q - 1
    // (cur); then cur's buffer is refilled with row q + kPipeAhead
    auto step = [&](int t, const PipeRowIn& in, PipeRowIn& cur, bool run) {
      const int q = tb + t + 1;
      wait_readers(t);
      // rows q .. q+kPipeAhead-1 are in flight, row q the oldest (an explicit
      // count: the compiler's own falls back to zero after the polls)
      __builtin_amdgcn_s_waitcnt(waitcnt_vm(4 * (kPipeAhead - 1)));
      __builtin_amdgcn_sched_barrier(0);
      F4 fbq;
      fbar_of(q, in, cur.py, thtau0, fbq);
      if constexpr (GAP) {
        lds_st4(in_row(q, 0), in.f);
        lds_st4(in_row(q, 1), in.px);
        lds_st4(in_row(q, 2), in.py);
        lds_st4(in_row(q, 3), in.g);
      }
      if (run) {
        F4 fnew, fbnew, npx, npy;
        stage(q - 1, fbc, fbq, cur, cy, fnew, fbnew, npx, npy);
        emit(1, q - 1, fnew, fbnew, npx, npy, cur.g);
        cy = npy;
      }
      post(t + 1);
      fbc = fbq;
      load(q + kPipeAhead, cur);
    };
    step(0, buf[1], buf[0], false);  // row tb only starts the histories
    int t = 1;
    for (; t + kPipeBufs <= steps; t += kPipeBufs) {
#pragma unroll
      for (int i = 0; i < kPipeBufs; ++i)
        step(t + i, buf[(i + 2) % kPipeBufs], buf[(i + 1) % kPipeBufs], true);
    }
#pragma unroll
    for (int i = 0; i < kPipeBufs; ++i)
      if (t + i < steps)
        step(t + i, buf[(i + 2) % kPipeBufs], buf[(i + 1) % kPipeBufs], true);
  } else if (w < n) {
    // Stage s = w+1, two rows behind stage s-1: at step t it takes in row
    // r+1 of stage s-1's output and runs on row r.
    const int s = w + 1;
    const int lo = tb + s, hi = y1 + n - s - 1;      // rows of stage s
    const int plo = tb + s - 1, phi = y1 + n - s;    // rows of stage s-1
    // row r's input and fbar alternate between two register sets (no
    // copies): the set filled at step t is the current row at step t+1
    PipeRowIn ra, rb;
    ra.f = ra.px = ra.py = ra.g = zero4();
    rb = ra;
    F4 fa = zero4(), fbb = zero4(), cy = zero4();
    auto sstep = [&](int t, const PipeRowIn& cur, const F4& fcur, PipeRowIn& nxt,
                     F4& fnxt) {
      const int r = tb + t - 2 * w;
      wait_for(w - 1, t);
      if (w + 1 < n) wait_for(w + 1, t + 2 - kPipeSlots);
      if (r + 1 >= plo && r + 1 <= phi) ld_ring(w - 1, r + 1, nxt, fnxt);
      if (r >= lo && r <= hi) {
        F4 fnew, fbnew, npx, npy;
        stage(r, fcur, fnxt, cur, cy, fnew, fbnew, npx, npy);
        emit(s, r, fnew, fbnew, npx, npy, cur.g);
        cy = npy;
      }
      post(t + 1);
    };
    int t = 0;
    for (; t + 1 < steps; t += 2) {
      sstep(t, ra, fa, rb, fbb);
      sstep(t + 1, rb, fbb, ra, fa);
    }
    if (t < steps) sstep(t, ra, fa, rb, fbb);
  } else if (GAP) {
    // Gap density and primal energy of (f^k, p^k) on row r = tb + t - 1,
    // from the staging ring (the walk's evaluation, term for term); row r is
    // kept from the step before, with p_y^k of row r-1 (pyu).
    PipeRowIn cur;
    cur.f = cur.px = cur.py = cur.g = zero4();
    F4 pyu = zero4();
    for (int t = 0; t < steps; ++t) {
      const int r = tb + t - 1;
      wait_for(0, t);
      if (r >= tb && r <= y1) {
        PipeRowIn in;
        in.f = lds_ld4(in_row(r + 1, 0));
        in.px = lds_ld4(in_row(r + 1, 1));
        in.py = lds_ld4(in_row(r + 1, 2));
        in.g = lds_ld4(in_row(r + 1, 3));
        if (r >= y0 && r < y1) {
          const F4& B = cur.f;
          const F4& EX = cur.px;
          const F4& EY = cur.py;
          const F4& A = in.f;
          const F4& Gv = cur.g;
          const bool dn = r + 1 < ny;
          const bool up = r > 0;
          const float nfr = from_right(B.v[0]);
          const float lox = from_left(EX.v[3]);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (owned && xg + j < nx) {
              const float right = (j < 3) ? B.v[j + 1] : nfr;
              const float fv = B.v[j];
              const float gx = (xg + j < nx - 1) ? right - fv : 0.0f;
              const float gy = dn ? A.v[j] - fv : 0.0f;
              const float lo = (j == 0) ? ((xg > 0) ? lox : 0.0f) : EX.v[j - 1];
              const float uo = up ? pyu.v[j] : 0.0f;
              const float d = (EX.v[j] - lo) + (EY.v[j] - uo);
              const float e = fv - Gv.v[j];
              const float res = e - d;
              const float tv = lam * __builtin_amdgcn_sqrtf(fmaf(gx, gx, gy * gy));
              const float dot = fmaf(gx, EX.v[j], gy * EY.v[j]);
              acc_gap += (double)(0.5f * res * res) + ((double)tv - (double)dot);
              acc_P += (double)(0.5f * e * e) + (double)tv;
            }
          }
        }
        pyu = cur.py;
        cur = in;
      }
      post(t + 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && *abort_flag != 0) atomicOr(c.err, kStateErrPipeWait);
}

}  // namespace dev
}  // namespace tvpd
