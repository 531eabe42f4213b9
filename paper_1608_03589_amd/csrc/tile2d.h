// Device code of the fused 2D sweep over one tile (a 256-column strip by a
// band of rows) for the unrolled solver's forward step, which keeps every
// iterate and forms the extrapolation from the stored f^{k-1} (the plain and
// the batched solvers use tile2d_xs.h), and the per-row helpers that the
// other tiles share.
//
// One call performs iteration k -> k+1 of the primal-dual method on the
// tile's rows (the regularised problem of the paper's Section 6, eq. opt,
// with identity forward operator and total-variation regulariser):
//     fbar    = f^k + theta (f^k - f^{k-1})                  (extrapolation)
//     p^{k+1} = P_lam(p^k + sigma grad fbar)                  (dual prox)
//     f^{k+1} = (f^k + tau div p^{k+1} + tau g) / (1 + tau)   (data prox)
// and, with GAP, accumulates the duality-gap density and the primal energy
// of (f^k, p^k) in float64.
//
// A wave owns the strip (one float4 per lane) and walks the band top to
// bottom, keeping the previous row's new dual y-component in registers.
// Neighbour columns come from the adjacent lane; the strip's outer columns
// (x0-1, x0+256) are read by every lane at one shared address and used by the
// edge lanes, and the left one's new dual value is recomputed there with the
// owner's arithmetic, so the iterates do not depend on the tiling.  The
// band's first row needs p^{k+1} of the row above, recomputed the same way.
// Padding columns (x >= nx) hold zeros and stay zero.
#pragma once

#include "common.h"
#include "pointwise.h"

namespace tvpd {
namespace dev {

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

// Projection of q onto the disc of radius lam (lam2 = lam * lam).
__device__ __forceinline__ void project2(float qx, float qy, float lam,
                                         float lam2, float& px, float& py) {
  const float c = ball_scale(sq2(qx, qy), lam, lam2);
  px = qx * c;
  py = qy * c;
}

// Value of the next (from_right) or previous (from_left) lane of the wave,
// by a DPP wavefront shift (wave_shl:1 / wave_shr:1): a VALU operation with
// no LDS round trip, unlike a bpermute shuffle.  The edge lane keeps its own
// value, as a shuffle past the wave's end does; callers replace it.  All
// lanes of the wave must be active.
__device__ __forceinline__ float from_right(float v) {
  const int x = __float_as_int(v);
  return __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_left(float v) {
  const int x = __float_as_int(v);
  return __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x138, 0xF, 0xF, false));
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

// Pointers and sizes of one tile at iteration k.
struct TileCtx {
  const float* fk;   // f^k
  const float* fkm;  // f^{k-1}
  const float* pxk;  // p^k, x component
  const float* pyk;  // p^k, y component
  const float* g;
  float* fn;         // f^{k+1}
  float* pxn;        // p^{k+1}
  float* pyn;
  int ny, nx, pitch;
  int x0, y0, y1;    // strip start column, band rows [y0, y1)
  float lam, tau, sig, th;
};

// Ring slots of iteration k in a plane block laid out as
// [f slot 0..2][p slot 0 (x, y)][p slot 1 (x, y)][g].
__device__ __forceinline__ void ring2d(float* base, int64_t PL, int k,
                                       TileCtx& c) {
  const int s0 = k % 3, s1 = (k + 1) % 3, sm = (k + 2) % 3;
  const int q0 = k & 1, q1 = q0 ^ 1;
  c.fk = base + s0 * PL;
  c.fkm = base + sm * PL;
  c.fn = base + s1 * PL;
  c.pxk = base + (3 + 2 * q0) * PL;
  c.pyk = c.pxk + PL;
  c.pxn = base + (3 + 2 * q1) * PL;
  c.pyn = c.pxn + PL;
  c.g = base + 7 * PL;
}

template <bool GAP>
__device__ __forceinline__ void sweep_tile(const TileCtx& c, double& acc_gap,
                                           double& acc_P) {
  const int lane = threadIdx.x & (kWave - 1);
  const float* fk = c.fk;
  const float* fkm = c.fkm;
  const float* pxk = c.pxk;
  const float* pyk = c.pyk;
  const float* g = c.g;
  float* fn = c.fn;
  float* pxn = c.pxn;
  float* pyn = c.pyn;
  const int x0 = c.x0, y0 = c.y0, y1 = c.y1;
  const int nx = c.nx, ny = c.ny;
  const int64_t P = c.pitch;
  const int xc = x0 + kColsPerLane * lane;
  const bool lin = xc < c.pitch;
  const bool hl = (lane == 0) && (x0 > 0);
  const bool hr = (lane == kWave - 1) && (x0 + kStripCols < nx);
  const int xl = x0 - 1, xr = x0 + kStripCols;
  const float lam = c.lam, tau = c.tau, sig = c.sig, th = c.th;
  const float iopt = prox_factor(tau);
  const float lam2 = lam * lam;

  // Row data.  In the steady state every lane issues every load (padding
  // lanes and the edge columns read clamped, valid addresses; their values
  // are masked out below), so the loads prefetched for the next row stay
  // in flight while this row is computed.
  const int xcl = min(xc, c.pitch - kColsPerLane);
  const int xlc = max(xl, 0);
  const int xrc = min(xr, c.pitch - 1);
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
      cb.v[j] = extrap(cur.f.v[j], cur.m.v[j], th);
      nb4.v[j] = extrap(nxt.f.v[j], nxt.m.v[j], th);
    }
    const float lb = extrap(cur.lf, cur.lm, th);
    const float rb = extrap(cur.rf, cur.rm, th);
    const float lnb = extrap(nxt.lf, nxt.lm, th);
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
        project2(dual_arg(opx.v[j], sig, gx), dual_arg(opy.v[j], sig, gy), lam, lam2, npx.v[j],
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
        project2(dual_arg(pc.lpx, sig, gx), dual_arg(pc.lpy, sig, gy), lam, lam2, hx, hy);
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
        const float v = fmaf(tau, d, cf.v[j]);
        fnew.v[j] = fmaf(tau, gg.v[j], v) * iopt;
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

}  // namespace dev
}  // namespace tvpd
