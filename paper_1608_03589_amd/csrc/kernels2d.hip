// Fused 2D primal-dual sweep for gfx950 and its helper kernels.
//
// One launch performs one whole iteration k -> k+1 of the primal-dual method
// for 1/2 |f - g|^2 + lam TV(f) (the regularised problem of the paper's
// Section 6, eq. opt, with identity forward operator and a total-variation
// regulariser):
//     fbar = f^k + theta (f^k - f^{k-1})           (extrapolation)
//     p^{k+1} = P_lam(p^k + sigma grad fbar)        (dual ascent + prox)
//     f^{k+1} = (f^k + tau div p^{k+1} + tau g) / (1 + tau)   (primal + prox)
// and, on check iterations, the duality-gap density of (f^k, p^k), reduced
// in float64.  Every plane is read once and written once per pixel: 20 bytes
// in (f^k, f^{k-1}, p^k x2, g), 12 bytes out (f^{k+1}, p^{k+1} x2).
//
// Work decomposition.  A wave owns a strip of 256 columns (one float4 per
// lane) and a band of `th` rows, which it walks top to bottom keeping the
// previous row's new dual y-component in registers.  Neighbour columns come
// from the adjacent lane; the strip's outer columns (x0-1 on the left,
// x0+256 on the right) are read by the edge lanes, and the left one's new
// dual value is recomputed there with exactly the owner's arithmetic, so the
// iterates do not depend on the tiling.  The band's first row needs
// p^{k+1} of the row above, which is recomputed the same way.
//
// Planes are stored with a pitch that is a multiple of 4 floats; padding
// columns hold zeros and stay zero.
#include "common.h"

namespace tvpd {
namespace {

struct F4 {
  float v[4];
};

__device__ __forceinline__ F4 ld4(const float* p) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  F4 r;
  r.v[0] = t.x;
  r.v[1] = t.y;
  r.v[2] = t.z;
  r.v[3] = t.w;
  return r;
}

__device__ __forceinline__ void st4(float* p, const F4& a) {
  *reinterpret_cast<float4*>(p) = make_float4(a.v[0], a.v[1], a.v[2], a.v[3]);
}

__device__ __forceinline__ F4 zero4() {
  F4 r;
#pragma unroll
  for (int j = 0; j < 4; ++j) r.v[j] = 0.0f;
  return r;
}

// f^k and f^{k-1} of one row of a strip, with the strip's outer columns.
struct RowF {
  F4 f, m;
  float lf, lm, rf, rm;
};
// p^k and g of one row of a strip, with p^k of the left outer column.
struct RowP {
  F4 px, py, g;
  float lpx, lpy;
};

__device__ __forceinline__ RowF zeroF() {
  RowF r;
  r.f = zero4();
  r.m = zero4();
  r.lf = r.lm = r.rf = r.rm = 0.0f;
  return r;
}

__device__ __forceinline__ RowP zeroP() {
  RowP r;
  r.px = zero4();
  r.py = zero4();
  r.g = zero4();
  r.lpx = r.lpy = 0.0f;
  return r;
}

// Projection of q onto the disc of radius lam; |q| <= lam keeps q.
__device__ __forceinline__ void project2(float qx, float qy, float lam,
                                         float& px, float& py) {
  const float n = sqrtf(qx * qx + qy * qy);
  if (n > lam) {
    const float s = lam / n;
    px = qx * s;
    py = qy * s;
  } else {
    px = qx;
    py = qy;
  }
}

__device__ __forceinline__ float from_right(float v) {
  return __shfl_down(v, 1, kWave);
}
__device__ __forceinline__ float from_left(float v) {
  return __shfl_up(v, 1, kWave);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum (a, b) over the block in a fixed order; result valid in thread 0.
__device__ __forceinline__ void block_sum2(double& a, double& b,
                                           double (*red)[kMaxBlock / kWave]) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < nw; ++w) {
      sa += red[0][w];
      sb += red[1][w];
    }
    a = sa;
    b = sb;
  }
}

__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Completion of a sweep: the last block to finish advances k, or on a gap
// check reduces the per-block partials (fixed order, float64), records the
// energies and either freezes k (converged) or advances it.
template <bool GAP>
__device__ __forceinline__ void finish_sweep(DevState* st, double* partials,
                                             int k, double acc_gap,
                                             double acc_P) {
  __shared__ double red[2][kMaxBlock / kWave];
  __shared__ int s_last;
  const unsigned nb = gridDim.x;
  if constexpr (GAP) {
    block_sum2(acc_gap, acc_P, red);
    if (threadIdx.x == 0) {
      store_agent(&partials[2 * blockIdx.x], acc_gap);
      store_agent(&partials[2 * blockIdx.x + 1], acc_P);
    }
  }
  __syncthreads();  // every wave of the block has read k and finished
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(&st->blocks_done, 1u);
    s_last = (prev == nb - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if constexpr (!GAP) {
    if (threadIdx.x == 0) {
      st->blocks_done = 0;
      st->k = k + 1;
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
        st->k = k + 1;
      }
      st->blocks_done = 0;
    }
  }
}

template <bool GAP>
__global__ __launch_bounds__(kMaxBlock) void sweep2d_kernel(Sweep2DArgs a) {
  DevState* st = a.st;
  const int k = st->k;
  if (st->converged || k >= st->k_end) return;

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  // Blocks are dispatched round-robin over the 8 XCDs; hand each XCD a
  // contiguous run of tiles so that vertically adjacent bands (which share
  // halo rows) meet in the same L2.
  const int nb = gridDim.x, b = blockIdx.x;
  const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
  const int bt = xcd * q8 + min(xcd, r8) + (b >> 3);
  const int wt = bt * a.wpb + wave;

  double acc_gap = 0.0, acc_P = 0.0;
  if (wt < a.ntiles) {
    const int s0 = k % 3, s1 = (k + 1) % 3, sm = (k + 2) % 3;
    const int q0 = k & 1, q1 = q0 ^ 1;
    const int64_t PL = a.plane;
    const float* fk = a.base + s0 * PL;
    const float* fkm = a.base + sm * PL;
    float* fn = a.base + s1 * PL;
    const float* pxk = a.base + (3 + 2 * q0) * PL;
    const float* pyk = pxk + PL;
    float* pxn = a.base + (3 + 2 * q1) * PL;
    float* pyn = pxn + PL;
    const float* g = a.base + 7 * PL;

    int tx, ty;
    if (a.order == 0) {
      ty = wt / a.ntx;
      tx = wt - ty * a.ntx;
    } else {
      tx = wt / a.nty;
      ty = wt - tx * a.nty;
    }
    const int x0 = tx * kStripCols;
    const int y0 = ty * a.th;
    const int y1 = min(y0 + a.th, a.ny);
    const int nx = a.nx, ny = a.ny;
    const int64_t P = a.pitch;
    const int xc = x0 + kColsPerLane * lane;
    const bool lin = xc < a.pitch;
    const bool hl = (lane == 0) && (x0 > 0);
    const bool hr = (lane == kWave - 1) && (x0 + kStripCols < nx);
    const int xl = x0 - 1, xr = x0 + kStripCols;
    const float lam = a.lam, tau = a.tau, sig = a.sigma, th = a.theta;
    const float opt = 1.0f + tau;

    // Row data.  In the steady state every lane issues every load (padding
    // lanes and the edge columns read clamped, valid addresses; their values
    // are masked out below), so the loads prefetched for the next row stay
    // in flight while this row is computed.
    const int xcl = min(xc, a.pitch - kColsPerLane);
    const int xlc = max(xl, 0);
    const int xrc = min(xr, a.pitch - 1);
    auto loadF = [&](int y, RowF& r) {
      const int64_t ro = (int64_t)y * P;
      r.f = ld4(fk + ro + xcl);
      r.m = ld4(fkm + ro + xcl);
      r.lf = fk[ro + xlc];
      r.lm = fkm[ro + xlc];
      r.rf = fk[ro + xrc];
      r.rm = fkm[ro + xrc];
    };
    auto loadP = [&](int y, RowP& r) {
      const int64_t ro = (int64_t)y * P;
      r.px = ld4(pxk + ro + xcl);
      r.py = ld4(pyk + ro + xcl);
      r.g = ld4(g + (int64_t)max(y, y0) * P + xcl);
      r.lpx = pxk[ro + xlc];
      r.lpy = pyk[ro + xlc];
    };

    F4 up_pyn = zero4();  // p_y^{k+1} of the row above (0 above row 0)
    F4 up_pyo = zero4();  // p_y^k of the row above

    // Row y from `cur` (f of row y), `nxt` (f of row y+1, unused on the
    // last image row) and `pc` (p, g of row y).
    auto compute = [&](int y, const RowF& cur, const RowF& nxt,
                       const RowP& pc) {
      const bool dn = (y + 1 < ny);
      const bool own = (y >= y0);
      const int64_t o = (int64_t)y * P + xc;
      const F4& cf = cur.f;
      const F4& nf = nxt.f;
      const F4& opx = pc.px;
      const F4& opy = pc.py;
      const F4& gg = pc.g;
      // extrapolation of rows y and y+1 (and of the halo columns)
      F4 cb, nb4;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cb.v[j] = cur.f.v[j] + th * (cur.f.v[j] - cur.m.v[j]);
        nb4.v[j] = nxt.f.v[j] + th * (nxt.f.v[j] - nxt.m.v[j]);
      }
      const float lb = cur.lf + th * (cur.lf - cur.lm);
      const float rb = cur.rf + th * (cur.rf - cur.rm);
      const float lnb = nxt.lf + th * (nxt.lf - nxt.lm);
      const float rf = cur.rf;

      // dual ascent on the extrapolated gradient, then the projection
      F4 npx, npy;
      {
        const float nbr = from_right(cb.v[0]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float right =
              (j < 3) ? cb.v[(j + 1) & 3] : (lane == kWave - 1 ? rb : nbr);
          const float gx = (xc + j < nx - 1) ? right - cb.v[j] : 0.0f;
          const float gy = dn ? nb4.v[j] - cb.v[j] : 0.0f;
          project2(opx.v[j] + sig * gx, opy.v[j] + sig * gy, lam, npx.v[j],
                   npy.v[j]);
        }
      }
      // new p_x of the column to the left
      float left_n = from_left(npx.v[3]);
      float left_o = from_left(opx.v[3]);
      if (lane == 0) {
        if (hl) {
          const float gx = cb.v[0] - lb;
          const float gy = dn ? lnb - lb : 0.0f;
          float hx, hy;
          project2(pc.lpx + sig * gx, pc.lpy + sig * gy, lam, hx, hy);
          left_n = hx;
          left_o = pc.lpx;
        } else {
          left_n = 0.0f;
          left_o = 0.0f;
        }
      }

      if (own) {
        F4 fnew;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float lp = (j == 0) ? left_n : npx.v[(j + 3) & 3];
          const float d = (npx.v[j] - lp) + (npy.v[j] - up_pyn.v[j]);
          const float v = cf.v[j] + tau * d;
          fnew.v[j] = (v + tau * gg.v[j]) / opt;
        }
        if (lin) {
          st4(fn + o, fnew);
          st4(pxn + o, npx);
          st4(pyn + o, npy);
        }
        if constexpr (GAP) {
          const float nfr = from_right(cf.v[0]);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float right =
                (j < 3) ? cf.v[(j + 1) & 3] : (lane == kWave - 1 ? rf : nfr);
            if (xc + j < nx) {
              const double gx =
                  (xc + j < nx - 1) ? (double)right - (double)cf.v[j] : 0.0;
              const double gy =
                  dn ? (double)nf.v[j] - (double)cf.v[j] : 0.0;
              const double lo = (j == 0) ? left_o : opx.v[(j + 3) & 3];
              const double d = ((double)opx.v[j] - lo) +
                               ((double)opy.v[j] - (double)up_pyo.v[j]);
              const double e = (double)cf.v[j] - (double)gg.v[j];
              const double r = e - d;
              const double nrm = sqrt(gx * gx + gy * gy);
              acc_gap += 0.5 * r * r + (double)lam * nrm -
                         (gx * (double)opx.v[j] + gy * (double)opy.v[j]);
              acc_P += 0.5 * e * e + (double)lam * nrm;
            }
          }
        } else {
          (void)rf;
          (void)nf;
        }
      }

      up_pyn = npy;
      up_pyo = opy;
    };

    const int ys = y0 > 0 ? y0 - 1 : 0;
    // rows y < ymain have a next row in the band and a row y+2 in the image
    const int ymain = min(y1 - 1, ny - 2);
    RowF F0 = zeroF(), F1 = zeroF(), F2 = zeroF();
    RowP Q0 = zeroP(), Q1 = zeroP(), Q2 = zeroP();
    loadF(ys, F0);
    if (ys + 1 < ny) loadF(ys + 1, F1);
    loadP(ys, Q0);
    int y = ys;
    // steady state: whole groups of three rows, the row buffers rotating
    // roles by name, so that no register copy has to wait on a load
    const int ngroups = ymain > ys ? (ymain - ys) / 3 : 0;
    for (int grp = 0; grp < ngroups; ++grp, y += 3) {
      loadF(y + 2, F2);
      loadP(y + 1, Q1);
      compute(y, F0, F1, Q0);
      loadF(y + 3, F0);
      loadP(y + 2, Q2);
      compute(y + 1, F1, F2, Q1);
      loadF(y + 4, F1);
      loadP(y + 3, Q0);
      compute(y + 2, F2, F0, Q2);
    }
    RowF cur = F0, nxt = F1;
    RowP pc = Q0;
    // the remaining rows of the band (at most four)
    for (; y < y1; ++y) {
      RowF nn = zeroF();
      RowP pn = zeroP();
      if (y + 1 < y1) {
        if (y + 2 < ny) loadF(y + 2, nn);
        loadP(y + 1, pn);
      }
      compute(y, cur, nxt, pc);
      cur = nxt;
      nxt = nn;
      pc = pn;
    }
  }
  finish_sweep<GAP>(st, a.partials, k, acc_gap, acc_P);
}

__global__ void init2d_kernel(float* base, int64_t plane, int ny, int nx,
                              int pitch, const float* __restrict__ g,
                              DevState* st) {
  const int64_t n = (int64_t)ny * pitch;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / pitch);
    const int x = (int)(i - (int64_t)y * pitch);
    const float v = (x < nx) ? g[(int64_t)y * nx + x] : 0.0f;
    base[i] = v;                 // f^0    (slot 0)
    base[plane + i] = 0.0f;      // slot 1
    base[2 * plane + i] = v;     // f^{-1} (slot 2)
    base[3 * plane + i] = 0.0f;  // p^0
    base[4 * plane + i] = 0.0f;
    base[5 * plane + i] = 0.0f;
    base[6 * plane + i] = 0.0f;
    base[7 * plane + i] = v;     // g
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->k = 0;
    st->k_end = 0x7fffffff;
    st->converged = 0;
    st->iters = 0;
    st->blocks_done = 0;
    st->checks = 0;
    st->nblocks = 0;
    st->flags = 0;
    st->P = st->D = st->gap = 0.0;
    st->tol = -1.0;
  }
}

__global__ void set_params_kernel(DevState* st, int32_t k_end, double tol) {
  st->k_end = k_end;
  st->tol = tol;
  st->converged = 0;
  st->blocks_done = 0;
}

__global__ void read2d_kernel(const float* base, int64_t plane, int ny,
                              int nx, int pitch, const DevState* st,
                              float* f_out, float* p_out) {
  const int k = st->k;
  const float* f = base + (k % 3) * plane;
  const float* px = base + (3 + 2 * (k & 1)) * plane;
  const float* py = px + plane;
  const int64_t n = (int64_t)ny * nx;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / nx);
    const int x = (int)(i - (int64_t)y * nx);
    const int64_t s = (int64_t)y * pitch + x;
    f_out[i] = f[s];
    if (p_out) {
      p_out[i] = px[s];
      p_out[n + i] = py[s];
    }
  }
}

// Gap density and primal energy of the current pair, one pixel per thread
// (neighbours read directly; used outside the iteration loop only).
__global__ __launch_bounds__(kMaxBlock) void energy2d_kernel(
    const float* base, int64_t plane, int ny, int nx, int pitch, float lam,
    const DevState* st, double* partials, int skip_if_converged) {
  if (skip_if_converged && st->converged) return;
  __shared__ double red[2][kMaxBlock / kWave];
  const int k = st->k;
  const float* f = base + (k % 3) * plane;
  const float* px = base + (3 + 2 * (k & 1)) * plane;
  const float* py = px + plane;
  const float* g = base + 7 * plane;
  const int64_t n = (int64_t)ny * nx;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sg = 0.0, sp = 0.0;
  if (i < n) {
    const int y = (int)(i / nx);
    const int x = (int)(i - (int64_t)y * nx);
    const int64_t s = (int64_t)y * pitch + x;
    const double fv = f[s];
    const double gx = (x < nx - 1) ? (double)f[s + 1] - fv : 0.0;
    const double gy = (y < ny - 1) ? (double)f[s + pitch] - fv : 0.0;
    const double dxl = (x > 0) ? (double)px[s - 1] : 0.0;
    const double dyl = (y > 0) ? (double)py[s - pitch] : 0.0;
    const double d = ((double)px[s] - dxl) + ((double)py[s] - dyl);
    const double e = fv - (double)g[s];
    const double r = e - d;
    const double nrm = sqrt(gx * gx + gy * gy);
    sg = 0.5 * r * r + (double)lam * nrm - (gx * px[s] + gy * py[s]);
    sp = 0.5 * e * e + (double)lam * nrm;
  }
  block_sum2(sg, sp, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sg;
    partials[2 * blockIdx.x + 1] = sp;
  }
}

__global__ __launch_bounds__(kMaxBlock) void energy_final_kernel(
    DevState* st, const double* partials, int nparts, int skip_if_converged) {
  if (skip_if_converged && st->converged) return;
  __shared__ double red[2][kMaxBlock / kWave];
  double sg = 0.0, sp = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    sg += partials[2 * i];
    sp += partials[2 * i + 1];
  }
  block_sum2(sg, sp, red);
  if (threadIdx.x == 0) {
    st->gap = sg;
    st->P = sp;
    st->D = sp - sg;
  }
}

inline DevState* state_of(void* ws) { return reinterpret_cast<DevState*>(ws); }

inline float* planes_of(const Layout& L, void* ws) {
  return reinterpret_cast<float*>(static_cast<char*>(ws) + L.plane_off);
}

inline double* partials_of(const Layout& L, void* ws) {
  return reinterpret_cast<double*>(static_cast<char*>(ws) + L.partial_off);
}

inline int grid_for(int64_t n, int block, int cap = 8192) {
  const int64_t b = (n + block - 1) / block;
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

int sweep2d_blocks(const Layout& L, const Tile2D& t) {
  const int ntx = (L.nx + kStripCols - 1) / kStripCols;
  const int nty = (L.ny + t.th - 1) / t.th;
  const int nt = ntx * nty;
  return (nt + t.wpb - 1) / t.wpb;
}

hipError_t launch_init2d(const Layout& L, const float* g, void* ws,
                         hipStream_t s) {
  hipLaunchKernelGGL(init2d_kernel, dim3(grid_for((int64_t)L.ny * L.pitch, 256)),
                     dim3(256), 0, s, planes_of(L, ws), L.plane, L.ny, L.nx,
                     L.pitch, g, state_of(ws));
  return hipGetLastError();
}

hipError_t launch_set_params(void* ws, int32_t k_end, double tol,
                             hipStream_t s) {
  hipLaunchKernelGGL(set_params_kernel, dim3(1), dim3(1), 0, s, state_of(ws),
                     k_end, tol);
  return hipGetLastError();
}

hipError_t launch_sweep2d(const Layout& L, const Tile2D& t,
                          const tvpd_coeffs& c, bool with_gap, void* ws,
                          hipStream_t s) {
  Sweep2DArgs a;
  a.base = planes_of(L, ws);
  a.plane = L.plane;
  a.ny = L.ny;
  a.nx = L.nx;
  a.pitch = L.pitch;
  a.th = t.th;
  a.wpb = t.wpb;
  a.order = t.order;
  a.ntx = (L.nx + kStripCols - 1) / kStripCols;
  a.nty = (L.ny + t.th - 1) / t.th;
  a.ntiles = a.ntx * a.nty;
  a.lam = c.lam;
  a.tau = c.tau;
  a.sigma = c.sigma;
  a.theta = c.theta;
  a.st = state_of(ws);
  a.partials = partials_of(L, ws);
  const int nb = (a.ntiles + t.wpb - 1) / t.wpb;
  if (nb > L.max_partials) return hipErrorInvalidValue;
  if (with_gap)
    hipLaunchKernelGGL(sweep2d_kernel<true>, dim3(nb), dim3(t.wpb * kWave), 0,
                       s, a);
  else
    hipLaunchKernelGGL(sweep2d_kernel<false>, dim3(nb), dim3(t.wpb * kWave), 0,
                       s, a);
  return hipGetLastError();
}

hipError_t launch_read2d(const Layout& L, const void* ws, float* f_out,
                         float* p_out, hipStream_t s) {
  void* w = const_cast<void*>(ws);
  hipLaunchKernelGGL(read2d_kernel, dim3(grid_for((int64_t)L.ny * L.nx, 256)),
                     dim3(256), 0, s, planes_of(L, w), L.plane, L.ny, L.nx,
                     L.pitch, state_of(w), f_out, p_out);
  return hipGetLastError();
}

hipError_t launch_energy2d(const Layout& L, float lam, void* ws,
                           bool skip_if_converged, hipStream_t s) {
  const int64_t n = (int64_t)L.ny * L.nx;
  const int nb = (int)((n + kMaxBlock - 1) / kMaxBlock);
  if (nb > L.max_partials) return hipErrorInvalidValue;
  hipLaunchKernelGGL(energy2d_kernel, dim3(nb), dim3(kMaxBlock), 0, s,
                     planes_of(L, ws), L.plane, L.ny, L.nx, L.pitch, lam,
                     state_of(ws), partials_of(L, ws), skip_if_converged ? 1 : 0);
  hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(kMaxBlock), 0, s,
                     state_of(ws), partials_of(L, ws), nb,
                     skip_if_converged ? 1 : 0);
  return hipGetLastError();
}

}  // namespace tvpd
