// S iterations of the 2D sweep in one pass over a tile (temporal blocking
// of depth S), on overlapping strips.
//
// Stage s (1..S) performs iteration k+s-1 -> k+s.  The band walk advances
// one row per step; at step t stage 1 works on row t, stage s on row
// t-(s-1), so everything stage s needs from stage s-1 (f^{k+s-1} on its row
// and the row below, p^{k+s-1} on its row) was produced this step or the
// step before and is still in registers.  A pass reads f^k, f^{k-1}, p^k
// (2 planes) and g (20 bytes per pixel) and writes f^{k+S-1} (the next
// pass's f^{k-1}), f^{k+S} and p^{k+S} (16 bytes): 36 bytes per S
// pixel-iterations.
//
// Columns: a wave loads the 256 columns [x0-M, x0+256-M) and owns the
// 256-2M columns [x0, x0+256-2M), with a margin M >= S (a multiple of 4; the
// plain solver uses xs_margin(S), the batched solver 8 for every S).  Each stage's results are exact on a range that shrinks by
// one column per stage at each end (a lane's right neighbour of the strip's
// last column and left neighbour of its first are unknown), so after S stages
// the owned columns are still exact and no halo column has to be recomputed
// separately: every value is computed by the same code as the owner's.  Rows: stage s walks rows [y0-1-(S-s), y1+(S-s)); the first row
// of each stage only provides p_y for the row below.  Image borders are
// handled by masks on the global row and column (forward differences vanish
// at the last index, p at index -1 counts as 0), so values computed outside
// the image never reach a stored one.  Every load is clamped into the image.
// A pass equals S single-iteration sweeps bit for bit.
#pragma once

#include "tile2d.h"

namespace tvpd {
namespace dev {


struct TileCtxS {
  const float* F;   // f^k
  const float* M;   // f^{k-1}
  const float* PX;  // p^k
  const float* PY;
  const float* G;
  float* FL;        // f^{k+S-1} (not written when S = 1)
  float* FN;        // f^{k+S}
  float* QX;        // p^{k+S}
  float* QY;
  int ny, nx, pitch;
  int x0, y0, y1;   // owned columns [x0, x0+256-2M), rows [y0, y1)
  float lam, tau, sig, th;
};

// One row of the loaded inputs.
struct XsLoad {
  F4 f, m, px, py, g;
};

template <int S, int M, bool GAP>
__device__ __forceinline__ void sweep_tile_xs(const TileCtxS& c,
                                              double& acc_gap,
                                              double& acc_P) {
  static_assert(S >= 1 && M >= S && M % kColsPerLane == 0 && 2 * M < kStripCols,
                "overlap margins");
  constexpr int kLeft = M;                     // columns left of the owned range
  constexpr int kOwned = kStripCols - 2 * M;
  const int lane = threadIdx.x & (kWave - 1);
  const int nx = c.nx, ny = c.ny, x0 = c.x0, y0 = c.y0, y1 = c.y1;
  const int64_t P = c.pitch;
  const int xs = x0 - kLeft;
  const int xg = xs + kColsPerLane * lane;     // first global column of the lane
  const int xcl = min(max(xg, 0), c.pitch - kColsPerLane);
  const bool owned = xg >= x0 && xg < x0 + kOwned && xg < c.pitch;
  const float lam = c.lam, tau = c.tau, sig = c.sig, th = c.th;
  const float iopt = prox_factor(tau);
  const float lam2 = lam * lam;

  auto load = [&](int y, XsLoad& L) {
    const int64_t o = (int64_t)min(max(y, 0), ny - 1) * P + xcl;
    L.f = ld4(c.F + o);
    L.m = ld4(c.M + o);
    L.px = ld4(c.PX + o);
    L.py = ld4(c.PY + o);
    L.g = ld4(c.G + o);
  };

  // Histories.  Loads: f^k of rows t, t-1 (lf1, lf2), f^{k-1} of row t
  // (lm1), p^k of row t (lp1x, lp1y) and p_y^k of row t-1 (lp2y), g of rows
  // t .. t-S+1 (gh[0..S-1]).  Stage s < S: f^{k+s} of its previous two rows
  // (fo1, fo2) and p^{k+s} of its previous row (po1x, po1y).  Every stage:
  // p_y^{k+s} of its previous row (cy).
  F4 lf1 = zero4(), lf2 = zero4(), lm1 = zero4(), lp1x = zero4(),
     lp1y = zero4(), lp2y = zero4();
  F4 gh[S];
  F4 fo1[S], fo2[S], po1x[S], po1y[S], cy[S + 1];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    gh[s] = zero4();
    fo1[s] = fo2[s] = po1x[s] = po1y[s] = zero4();
  }
#pragma unroll
  for (int s = 0; s <= S; ++s) cy[s] = zero4();

  // One walk step: L holds the loads of row t+1.
  auto step = [&](int t, const XsLoad& L) {
    F4 fo[S + 1], pox[S + 1], poy[S + 1];
#pragma unroll
    for (int s = 1; s <= S; ++s) {
      const int r = t - (s - 1);           // row of stage s
      const bool dn = r + 1 < ny;
      // inputs of stage s (see the header)
      const F4& A = (s == 1) ? L.f : fo[s - 1];       // f^{k+s-1}, row r+1
      const F4& B = (s == 1) ? lf1 : fo1[s - 1];      // f^{k+s-1}, row r
      const F4& C = (s == 1) ? L.m : (s == 2 ? lf1 : fo1[s - 2]);  // f^{k+s-2}, r+1
      const F4& D = (s == 1) ? lm1 : (s == 2 ? lf2 : fo2[s - 2]);  // f^{k+s-2}, r
      const F4& EX = (s == 1) ? lp1x : po1x[s - 1];   // p^{k+s-1}, row r
      const F4& EY = (s == 1) ? lp1y : po1y[s - 1];
      const F4& Gv = gh[s - 1];                        // g, row r
      F4 cb, nb;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cb.v[j] = extrap(B.v[j], D.v[j], th);
        nb.v[j] = extrap(A.v[j], C.v[j], th);
      }
      const float nbr = from_right(cb.v[0]);
      F4 npx, npy;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float right = (j < 3) ? cb.v[j + 1] : nbr;
        const float gx = (xg + j < nx - 1) ? right - cb.v[j] : 0.0f;
        const float gy = dn ? nb.v[j] - cb.v[j] : 0.0f;
        project2(dual_arg(EX.v[j], sig, gx), dual_arg(EY.v[j], sig, gy), lam, lam2, npx.v[j],
                 npy.v[j]);
      }
      const float left = from_left(npx.v[3]);
      const bool up = r > 0;
      F4 fnew;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float lp = (j == 0) ? (xg > 0 ? left : 0.0f) : npx.v[j - 1];
        const float d = (npx.v[j] - lp) + (npy.v[j] - (up ? cy[s].v[j] : 0.0f));
        const float v = fmaf(tau, d, B.v[j]);
        fnew.v[j] = fmaf(tau, Gv.v[j], v) * iopt;
      }
      fo[s] = fnew;
      pox[s] = npx;
      poy[s] = npy;
      if constexpr (GAP) {
        // gap density and primal energy of (f^k, p^k) on row t
        // (the lane shuffles run on the whole wave: a row condition is the
        // same for every lane, the column condition is applied afterwards)
        if (s == 1 && r >= y0 && r < y1) {
          const float nfr = from_right(B.v[0]);
          const float lox = from_left(EX.v[3]);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (owned && xg + j < nx) {
              const float right = (j < 3) ? B.v[j + 1] : nfr;
              const double fv = B.v[j];
              const double gx =
                  (xg + j < nx - 1) ? (double)right - fv : 0.0;
              const double gy = dn ? (double)A.v[j] - fv : 0.0;
              const double lo =
                  (j == 0) ? (xg > 0 ? (double)lox : 0.0) : (double)EX.v[j - 1];
              const double uo = up ? (double)lp2y.v[j] : 0.0;
              const double d = ((double)EX.v[j] - lo) +
                               ((double)EY.v[j] - uo);
              const double e = fv - (double)Gv.v[j];
              const double res = e - d;
              const double nrm = sqrt(gx * gx + gy * gy);
              acc_gap += 0.5 * res * res + (double)lam * nrm -
                         (gx * (double)EX.v[j] + gy * (double)EY.v[j]);
              acc_P += 0.5 * e * e + (double)lam * nrm;
            }
          }
        }
      }
    }
    // stores: f^{k+S} and p^{k+S} of stage S's row, f^{k+S-1} of stage
    // S-1's row, each inside the band
    if (owned) {
      const int rS = t - (S - 1);
      if (rS >= y0 && rS < y1) {
        const int64_t o = (int64_t)rS * P + xg;
        st4(c.FN + o, fo[S]);
        st4(c.QX + o, pox[S]);
        st4(c.QY + o, poy[S]);
      }
      if constexpr (S > 1) {
        const int rL = rS + 1;
        if (rL >= y0 && rL < y1) st4(c.FL + (int64_t)rL * P + xg, fo[S - 1]);
      }
    }
    // shift the histories
    lf2 = lf1;
    lf1 = L.f;
    lm1 = L.m;
    lp2y = lp1y;
    lp1x = L.px;
    lp1y = L.py;
#pragma unroll
    for (int s = S - 1; s > 0; --s) gh[s] = gh[s - 1];
    gh[0] = L.g;
#pragma unroll
    for (int s = 1; s < S; ++s) {
      fo2[s] = fo1[s];
      fo1[s] = fo[s];
      po1x[s] = pox[s];
      po1y[s] = poy[s];
    }
#pragma unroll
    for (int s = 1; s <= S; ++s) cy[s] = poy[s];
  };

  // The walk: step t runs stage 1 on row t, from y0-S to y1+S-2.  The
  // histories start with row y0-S; rows are prefetched one step ahead into
  // two buffers used alternately.
  const int tb = y0 - S;
  const int te = y1 + S - 2;
  {
    XsLoad Z;
    load(tb, Z);
    lf1 = Z.f;
    lm1 = Z.m;
    lp1x = Z.px;
    lp1y = Z.py;
    gh[0] = Z.g;
  }
  XsLoad X, Y;
  load(tb + 1, X);
  int t = tb;
  for (; t + 1 <= te; t += 2) {
    load(t + 2, Y);
    step(t, X);
    load(t + 3, X);
    step(t + 1, Y);
  }
  if (t <= te) step(t, X);
}

}  // namespace dev
}  // namespace tvpd
