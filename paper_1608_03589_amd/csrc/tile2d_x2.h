// Two iterations of the 2D sweep in one pass over a tile (temporal blocking).
//
// Stage A performs iteration k on row r and stage B iteration k+1 on row
// r-1 of the same band walk, so everything iteration k produces is consumed
// from registers:
//   A:  p^{k+1} = P_lam(p^k + sigma grad fbar^k),  fbar^k = f^k + theta (f^k - f^{k-1})
//       f^{k+1} = (f^k + tau div p^{k+1} + tau g) / (1 + tau)
//   B:  p^{k+2} = P_lam(p^{k+1} + sigma grad fbar^{k+1}),
//       fbar^{k+1} = f^{k+1} + theta (f^{k+1} - f^k)
//       f^{k+2} = (f^{k+1} + tau div p^{k+2} + tau g) / (1 + tau)
// A pass reads f^k, f^{k-1}, p^k (2 planes) and g (20 bytes per pixel) and
// writes f^{k+1} (the next pass's f^{k-1}), f^{k+2} and p^{k+2} (16 bytes):
// 36 bytes per two pixel-iterations instead of 64.
//
// Neighbours: A needs fbar^k one column right and one row down, and p_x^{k+1}
// one column left / p_y^{k+1} one row up; B needs the same of fbar^{k+1} and
// p^{k+2}.  Hence the strip's left halo carries A at columns x0-2 (p_x only)
// and x0-1 (p^{k+1}, f^{k+1}) and B at x0-1 (p_x only); the right halo
// carries A at x0+256 (p^{k+1}, f^{k+1}, reading fbar^k at x0+257).  Every
// halo value is computed with the owner's arithmetic, so a pass equals two
// single-iteration sweeps bit for bit.  The band walk starts two rows above
// the band (A at y0-2 gives p_y^{k+1} for f^{k+1} at y0-1, B at y0-1 gives
// p_y^{k+2} for the band's first row) and ends one row below it (A at y1
// gives f^{k+1} for B's last downward difference).
//
// Every lane issues every load (clamped rows and columns, values of padding
// lanes and absent neighbours are masked out), and row data is prefetched one
// step ahead into two buffers used alternately, so the loads stay in flight
// while the previous row is computed.
#pragma once

#include "tile2d.h"

namespace tvpd {
namespace dev {

struct TileCtx2 {
  const float* F;   // f^k
  const float* M;   // f^{k-1}
  const float* PX;  // p^k
  const float* PY;
  const float* G;
  float* FA;        // f^{k+1}
  float* FB;        // f^{k+2}
  float* BX;        // p^{k+2}
  float* BY;
  int ny, nx, pitch;
  int x0, y0, y1;
  float lam, tau, sig, th;
};

// f^k, f^{k-1} of one row: the lane's four columns and the halo columns
// x0-2, x0-1 (l2, l1) and x0+256, x0+257 (r1, r2).
struct XRowF {
  F4 f, m;
  float l2f, l2m, l1f, l1m, r1f, r1m, r2f, r2m;
};
// p^k and g of one row, with p^k at x0-2, x0-1, x0+256 and g at x0-1, x0+256.
struct XRowP {
  F4 px, py, g;
  float l2x, l2y, l1x, l1y, l1g, r1x, r1y, r1g;
};

template <bool GAP>
__device__ __forceinline__ void sweep_tile_x2(const TileCtx2& c,
                                              double& acc_gap,
                                              double& acc_P) {
  const int lane = threadIdx.x & (kWave - 1);
  const int nx = c.nx, ny = c.ny, x0 = c.x0, y0 = c.y0, y1 = c.y1;
  const int64_t P = c.pitch;
  const int xc = x0 + kColsPerLane * lane;
  const bool lin = xc < c.pitch;
  const bool hasL = x0 > 0;                  // a strip to the left exists
  const int xR1 = x0 + kStripCols;           // right halo columns
  const int xL1 = x0 - 1, xL2 = x0 - 2;
  const float lam = c.lam, tau = c.tau, sig = c.sig, th = c.th;
  const float iopt = prox_factor(tau);
  const float lam2 = lam * lam;
  const bool last_lane = lane == kWave - 1;

  // clamped addresses: every load is valid, unused values are masked below
  const int xcl = min(xc, c.pitch - kColsPerLane);
  const int cl2 = max(xL2, 0), cl1 = max(xL1, 0);
  const int cr1 = min(xR1, c.pitch - 1), cr2 = min(xR1 + 1, c.pitch - 1);
  auto rowc = [&](int y) { return (int64_t)min(max(y, 0), ny - 1) * P; };
  auto loadF = [&](int y, XRowF& r) {
    const int64_t ro = rowc(y);
    r.f = ld4(c.F + ro + xcl);
    r.m = ld4(c.M + ro + xcl);
    r.l2f = c.F[ro + cl2];
    r.l2m = c.M[ro + cl2];
    r.l1f = c.F[ro + cl1];
    r.l1m = c.M[ro + cl1];
    r.r1f = c.F[ro + cr1];
    r.r1m = c.M[ro + cr1];
    r.r2f = c.F[ro + cr2];
    r.r2m = c.M[ro + cr2];
  };
  auto loadP = [&](int y, XRowP& r) {
    const int64_t ro = rowc(y);
    r.px = ld4(c.PX + ro + xcl);
    r.py = ld4(c.PY + ro + xcl);
    r.g = ld4(c.G + ro + xcl);
    r.l2x = c.PX[ro + cl2];
    r.l2y = c.PY[ro + cl2];
    r.l1x = c.PX[ro + cl1];
    r.l1y = c.PY[ro + cl1];
    r.l1g = c.G[ro + cl1];
    r.r1x = c.PX[ro + cr1];
    r.r1y = c.PY[ro + cr1];
    r.r1g = c.G[ro + cr1];
  };
  auto xb = [&](float f, float m) { return extrap(f, m, th); };

  // ---- state carried from row to row (values of row r-1, or of row r
  // for the extrapolation of the current row)
  F4 ab = zero4();                 // fbar^k of row r
  float abL2 = 0.f, abL1 = 0.f, abR1 = 0.f, abR2 = 0.f;
  F4 F0 = zero4();                 // f^k of row r
  float F0L1 = 0.f, F0R1 = 0.f;
  F4 Fm1 = zero4();                // f^k of row r-1
  float Fm1L1 = 0.f, Fm1R1 = 0.f;
  F4 FAm1 = zero4();               // f^{k+1} of row r-1
  float FAm1L1 = 0.f, FAm1R1 = 0.f;
  F4 AXm1 = zero4(), AYm1 = zero4();  // p^{k+1} of row r-1 (0 above row 0)
  float AXm1L1 = 0.f, AYm1L1 = 0.f, AYm1R1 = 0.f;
  F4 Gm1 = zero4();                // g of row r-1
  F4 BYm2 = zero4();               // p_y^{k+2} of row r-2
  F4 PYm1 = zero4();               // p_y^k of row r-1 (gap)

  const int rs = max(y0 - 2, 0);
  const int rb0 = max(y0 - 1, 0);

  // One step: stage A on row r (f of row r+1 in `nx_`, p and g of row r in
  // `pc`), stage B on row r-1, then the carried state moves down one row.
  auto step = [&](int r, const XRowF& nxr, const XRowP& pc) {
    const bool doA = r < ny;
    const bool dnA = r + 1 < ny;
    const bool doFA = doA && r >= y0 - 1;
    // fbar^k of row r+1
    F4 abn;
#pragma unroll
    for (int j = 0; j < 4; ++j) abn.v[j] = xb(nxr.f.v[j], nxr.m.v[j]);
    const float abnL2 = xb(nxr.l2f, nxr.l2m), abnL1 = xb(nxr.l1f, nxr.l1m);
    const float abnR1 = xb(nxr.r1f, nxr.r1m), abnR2 = xb(nxr.r2f, nxr.r2m);

    // ---- stage A: iteration k on row r
    F4 ax = zero4(), ay = zero4(), fa = zero4();
    float axL2 = 0.f, axL1 = 0.f, ayL1 = 0.f, axR1 = 0.f, ayR1 = 0.f;
    float faL1 = 0.f, faR1 = 0.f;
    if (doA) {
      const float abr = from_right(ab.v[0]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float right =
            (j < 3) ? ab.v[(j + 1) & 3] : (last_lane ? abR1 : abr);
        const float gx = (xc + j < nx - 1) ? right - ab.v[j] : 0.0f;
        const float gy = dnA ? abn.v[j] - ab.v[j] : 0.0f;
        project2(dual_arg(pc.px.v[j], sig, gx), dual_arg(pc.py.v[j], sig, gy), lam, lam2, ax.v[j],
                 ay.v[j]);
      }
      {  // halo x0-2 (p_x only), x0-1 and x0+256
        float dummy;
        const float gx2 = abL1 - abL2;
        const float gy2 = dnA ? abnL2 - abL2 : 0.0f;
        project2(dual_arg(pc.l2x, sig, gx2), dual_arg(pc.l2y, sig, gy2), lam, lam2, axL2, dummy);
        const float gx1 = ab.v[0] - abL1;
        const float gy1 = dnA ? abnL1 - abL1 : 0.0f;
        project2(dual_arg(pc.l1x, sig, gx1), dual_arg(pc.l1y, sig, gy1), lam, lam2, axL1, ayL1);
        const float gxr = (xR1 < nx - 1) ? abR2 - abR1 : 0.0f;
        const float gyr = dnA ? abnR1 - abR1 : 0.0f;
        project2(dual_arg(pc.r1x, sig, gxr), dual_arg(pc.r1y, sig, gyr), lam, lam2, axR1, ayR1);
      }
      if (doFA) {
        float lft = from_left(ax.v[3]);
        if (lane == 0) lft = hasL ? axL1 : 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float lp = (j == 0) ? lft : ax.v[(j + 3) & 3];
          const float d = (ax.v[j] - lp) + (ay.v[j] - AYm1.v[j]);
          const float v = fmaf(tau, d, F0.v[j]);
          fa.v[j] = fmaf(tau, pc.g.v[j], v) * iopt;
        }
        // x0-1 (its left neighbour x0-2 always exists when x0 > 0)
        const float dL = (axL1 - axL2) + (ayL1 - AYm1L1);
        faL1 = fmaf(tau, pc.l1g, fmaf(tau, dL, F0L1)) * iopt;
        // x0+256: its left neighbour is this lane's last column
        const float dR = (axR1 - ax.v[3]) + (ayR1 - AYm1R1);
        faR1 = fmaf(tau, pc.r1g, fmaf(tau, dR, F0R1)) * iopt;
        if (r >= y0 && r < y1 && lin) st4(c.FA + (int64_t)r * P + xc, fa);
      }
      if constexpr (GAP) {
        if (r >= y0 && r < y1) {
          const float nfr = from_right(F0.v[0]);
          float lo0 = from_left(pc.px.v[3]);
          if (lane == 0) lo0 = hasL ? pc.l1x : 0.0f;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float right =
                (j < 3) ? F0.v[(j + 1) & 3] : (last_lane ? F0R1 : nfr);
            if (xc + j < nx) {
              const double gx =
                  (xc + j < nx - 1) ? (double)right - (double)F0.v[j] : 0.0;
              const double gy =
                  dnA ? (double)nxr.f.v[j] - (double)F0.v[j] : 0.0;
              const double lo = (j == 0) ? lo0 : pc.px.v[(j + 3) & 3];
              const double d = ((double)pc.px.v[j] - lo) +
                               ((double)pc.py.v[j] - (double)PYm1.v[j]);
              const double e = (double)F0.v[j] - (double)pc.g.v[j];
              const double rr = e - d;
              const double nrm = sqrt(gx * gx + gy * gy);
              acc_gap += 0.5 * rr * rr + (double)lam * nrm -
                         (gx * (double)pc.px.v[j] + gy * (double)pc.py.v[j]);
              acc_P += 0.5 * e * e + (double)lam * nrm;
            }
          }
        }
      }
    }

    // ---- stage B: iteration k+1 on row rb = r-1
    const int rb = r - 1;
    if (rb >= rb0 && rb < y1) {
      const bool dnB = rb + 1 < ny;
      F4 bb0, bb1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bb0.v[j] = xb(FAm1.v[j], Fm1.v[j]);
        bb1.v[j] = xb(fa.v[j], F0.v[j]);
      }
      const float bbL1a = xb(FAm1L1, Fm1L1), bbL1b = xb(faL1, F0L1);
      const float bbR1a = xb(FAm1R1, Fm1R1);
      F4 bx, by;
      const float bbr = from_right(bb0.v[0]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float right =
            (j < 3) ? bb0.v[(j + 1) & 3] : (last_lane ? bbR1a : bbr);
        const float gx = (xc + j < nx - 1) ? right - bb0.v[j] : 0.0f;
        const float gy = dnB ? bb1.v[j] - bb0.v[j] : 0.0f;
        project2(dual_arg(AXm1.v[j], sig, gx), dual_arg(AYm1.v[j], sig, gy), lam, lam2, bx.v[j],
                 by.v[j]);
      }
      float bxL1, dummy;
      {
        const float gx = bb0.v[0] - bbL1a;
        const float gy = dnB ? bbL1b - bbL1a : 0.0f;
        project2(dual_arg(AXm1L1, sig, gx), dual_arg(AYm1L1, sig, gy), lam, lam2, bxL1, dummy);
      }
      if (rb >= y0) {
        float lft = from_left(bx.v[3]);
        if (lane == 0) lft = hasL ? bxL1 : 0.0f;
        F4 fb;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float lp = (j == 0) ? lft : bx.v[(j + 3) & 3];
          const float d = (bx.v[j] - lp) + (by.v[j] - BYm2.v[j]);
          const float v = fmaf(tau, d, FAm1.v[j]);
          fb.v[j] = fmaf(tau, Gm1.v[j], v) * iopt;
        }
        if (lin) {
          const int64_t o = (int64_t)rb * P + xc;
          st4(c.FB + o, fb);
          st4(c.BX + o, bx);
          st4(c.BY + o, by);
        }
      }
      BYm2 = by;
    }

    // ---- move down one row
    Fm1 = F0;
    Fm1L1 = F0L1;
    Fm1R1 = F0R1;
    FAm1 = fa;
    FAm1L1 = faL1;
    FAm1R1 = faR1;
    AXm1 = ax;
    AYm1 = ay;
    AXm1L1 = axL1;
    AYm1L1 = ayL1;
    AYm1R1 = ayR1;
    Gm1 = pc.g;
    PYm1 = pc.py;
    ab = abn;
    abL2 = abnL2;
    abL1 = abnL1;
    abR1 = abnR1;
    abR2 = abnR2;
    F0 = nxr.f;
    F0L1 = nxr.l1f;
    F0R1 = nxr.r1f;
  };

  // prime: f of row rs (current) and of row rs+1 (next), p and g of row rs
  XRowF X, Y;
  XRowP PA, PB;
  loadF(rs, X);
#pragma unroll
  for (int j = 0; j < 4; ++j) ab.v[j] = xb(X.f.v[j], X.m.v[j]);
  abL2 = xb(X.l2f, X.l2m);
  abL1 = xb(X.l1f, X.l1m);
  abR1 = xb(X.r1f, X.r1m);
  abR2 = xb(X.r2f, X.r2m);
  F0 = X.f;
  F0L1 = X.l1f;
  F0R1 = X.r1f;
  loadF(rs + 1, X);
  loadP(rs, PA);
  // steps r = rs .. y1, two per loop turn so that the two row buffers swap
  // roles by name
  int r = rs;
  for (; r + 1 <= y1; r += 2) {
    loadF(r + 2, Y);
    loadP(r + 1, PB);
    step(r, X, PA);
    loadF(r + 3, X);
    loadP(r + 2, PA);
    step(r + 1, Y, PB);
  }
  if (r <= y1) step(r, X, PA);
}

}  // namespace dev
}  // namespace tvpd
