// S iterations of the 2D sweep in one pass over a tile (temporal blocking
// of depth S), on overlapping strips.  Every pass of the plain and the
// batched 2D solvers runs here (S = 1 .. kMaxPass).
//
// Extrapolation from the current iterate.  The data prox gives
// f^k = (f^{k-1} + tau d^k + tau g) / (1 + tau), with d^k = div p^k and tau
// the step that produced f^k, so
//     fbar^k = f^k + theta (f^k - f^{k-1}) = f^k + theta tau (g + d^k - f^k),
// and fbar^0 = g (f^0 = g, p^0 = 0).  The stage that computes f^{k+s} forms
// fbar^{k+s} from its own divergence; the first stage of a pass forms fbar^k
// from the stored p^k with the same operations in the same order, so a pass
// of S iterations equals S passes of one bit for bit.  A pass reads f^k,
// p^k (2 planes) and g (16 bytes per pixel) and writes f^{k+S} and p^{k+S}
// (12 bytes): f^{k-1} is neither stored nor read.
//
// Stage s (1..S) performs iteration k+s-1 -> k+s.  The band walk advances
// one row per step; at step t stage 1 works on row t, stage s on row
// t-(s-1), so everything stage s needs from stage s-1 (fbar^{k+s-1} on its
// row and the row below, f^{k+s-1} and p^{k+s-1} on its row) was produced
// this step or the step before and is still in registers.
//
// Columns: a wave loads the 256 columns [x0-M, x0+256-M) and owns the
// 256-2M columns [x0, x0+256-2M).  Values are exact on a column range that
// shrinks at the left by one for fbar^k (its divergence needs the left
// neighbour's p_x) and at both ends by one per stage (a lane's right
// neighbour of the strip's last column and left neighbour of its first are
// unknown), so a margin M >= S + 1 (a multiple of 4; the plain solver uses
// xs_margin(S), the batched solver 8 for every S) keeps the owned columns
// exact with no halo computed separately: every value is computed by the
// same code as the owner's.  Rows: the walk starts S + 1 rows above the
// band, and f^{k+s} is exact from row y0-S+s on.  Image borders are handled
// by masks on the global row and column (forward differences vanish at the
// last index, p at index -1 counts as 0), so values computed outside the
// image never reach a stored one; with SPLIT, tiles where no mask can fire
// walk a second copy of the loop without them.  Every load is clamped into
// the image.
//
// The unrolled solver's forward passes use the same walk with three
// differences: the extrapolation as defined (PROX = false: f^{k-1} is read
// once per pass and each stage forms fbar from its new and its input iterate,
// the values its adjoint recomputes from the stored iterates), coefficients
// per stage, and every stage storing its iterate (ALL).
#pragma once

#include <type_traits>

#include "tile2d.h"

namespace tvpd {
namespace dev {

struct TileCtxS {
  const float* F;   // f^k
  const float* PX;  // p^k
  const float* PY;
  const float* G;
  float* FN;        // f^{k+S}
  float* QX;        // p^{k+S}
  float* QY;
  int ny, nx, pitch;
  int x0, y0, y1;   // owned columns [x0, x0+256-2M), rows [y0, y1)
  float lam, tau, sig, th;
  float tau_prev;   // the step that produced f^k (any value at k = 0)
  // PROX = false: f^{k-1}
  const float* MF;
  // ALL: stage s's coefficients and outputs f^{k+s}, p^{k+s} at index s-1
  float slam[kMaxPass], stau[kMaxPass], ssig[kMaxPass];
  float* SF[kMaxPass];
  float* SQX[kMaxPass];
  float* SQY[kMaxPass];
};

// One row of the loaded inputs (m: f^{k-1}, loaded with PROX = false only).
struct XsLoad {
  F4 f, px, py, g, m;
};

template <int S, int M, bool GAP, bool SPLIT = true, bool PROX = true,
          bool ALL = false>
__device__ __forceinline__ void sweep_tile_xs(const TileCtxS& c,
                                              double& acc_gap,
                                              double& acc_P) {
  static_assert(S >= 1 && M >= S + 1 && M % kColsPerLane == 0 &&
                    2 * M < kStripCols,
                "overlap margins");
  static_assert(!(ALL && GAP), "the per-stage variant has no gap");
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
  const float thtau = th * tau;            // fbar of the iterates this pass makes
  const float thtau0 = th * c.tau_prev;    // fbar^k

  auto load = [&](int y, XsLoad& L) {
    const int64_t o = (int64_t)min(max(y, 0), ny - 1) * P + xcl;
    L.f = ld4(c.F + o);
    L.px = ld4(c.PX + o);
    L.py = ld4(c.PY + o);
    L.g = ld4(c.G + o);
    if constexpr (!PROX) L.m = ld4(c.MF + o);
  };

  // fbar^k on row y from its loads L and p_y^k of the row above (pya).
  auto fbar_loaded = [&](auto edge_tag, int y, const XsLoad& L, const F4& pya,
                         F4& out) {
    constexpr bool kEdge = decltype(edge_tag)::value;
    if constexpr (!PROX) {
#pragma unroll
      for (int j = 0; j < 4; ++j) out.v[j] = extrap(L.f.v[j], L.m.v[j], th);
      return;
    }
    const bool up = !kEdge || y > 0;
    const float pl = from_left(L.px.v[3]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float lp = (j == 0) ? ((!kEdge || xg > 0) ? pl : 0.0f) : L.px.v[j - 1];
      const float d = (L.px.v[j] - lp) + (L.py.v[j] - (up ? pya.v[j] : 0.0f));
      out.v[j] = extrap_prox(L.f.v[j], L.g.v[j], d, thtau0);
    }
  };

  // The walk: step t runs stage 1 on row t, from y0-S-1 to y1+S-2.
  const int tb = y0 - S - 1;
  const int te = y1 + S - 2;

  // Interior tiles: every row a stage visits, [y0-2S, y1+S-2], has a row
  // above and a row below in the image, and every loaded column has both
  // neighbours in the image, so no border mask can fire.
  const bool interior =
      xs >= 1 && xs + kStripCols < nx && y0 >= 2 * S + 1 && y1 + S <= ny;

  // Histories.  Loads: f^k of row t (lf1), p^k of row t (lp1x, lp1y) and
  // p_y^k of row t-1 (lp2y), g of rows t .. t-S+1 (gh[0..S-1]).  fbar^k of
  // row t and, for stage s < S, fbar^{k+s} of its previous row (fbh[s]).
  // Stage s < S: f^{k+s} and p^{k+s} of its previous row (fo1, po1x, po1y).
  // Every stage: p_y^{k+s} of its previous row (cy).
  // (Index S of fbh, fo1, po1x, po1y is never written: it stands for the
  // outputs of a stage S that the ramp-up below skips.)
  F4 lf1 = zero4(), lp1x = zero4(), lp1y = zero4(), lp2y = zero4();
  F4 gh[S], fbh[S + 1];
  F4 fo1[S + 1], po1x[S + 1], po1y[S + 1], cy[S + 1];
#pragma unroll
  for (int s = 0; s < S; ++s) gh[s] = zero4();
#pragma unroll
  for (int s = 0; s <= S; ++s) {
    fbh[s] = fo1[s] = po1x[s] = po1y[s] = cy[s] = zero4();
  }

  // Ramp-up.  Stage s is needed on rows [y0-S+s-1, y1+S-s-1]: f^{k+s} on
  // [y0-(S-s), y1+(S-s)) and p^{k+s} one row further up, for the divergence
  // of the row below.  It reaches the first of them at step tb + 2s - 1, so
  // during the first 2S - 1 steps only the stages s <= (t - tb + 1) / 2 run;
  // the others would compute rows that nothing reads (S^2 stage-rows per
  // band).  A skipped stage leaves its histories as they are.
  auto ramp = [&](int t) { return min(S, (t - tb + 1) >> 1); };

  // One walk step: L holds the loads of row t+1; stages 1..m run.
  auto step = [&](auto edge_tag, int t, const XsLoad& L, auto m) {
    constexpr bool kEdge = decltype(edge_tag)::value;
    // fb[s]: fbar^{k+s} on row t-s+1 (stage s+1's next row); fb[0] from the
    // loads of row t+1
    F4 fo[S + 1], fb[S + 1], pox[S + 1], poy[S + 1];
    fbar_loaded(edge_tag, t + 1, L, lp1y, fb[0]);
#pragma unroll
    for (int s = 1; s <= S; ++s) {
      if (s > m) {
        fo[s] = fo1[s];
        fb[s] = fbh[s];
        pox[s] = po1x[s];
        poy[s] = cy[s];
        continue;
      }
      const int r = t - (s - 1);           // row of stage s
      const bool dn = !kEdge || r + 1 < ny;
      // inputs of stage s (see the header)
      const F4& cb = fbh[s - 1];                      // fbar^{k+s-1}, row r
      const F4& nb = fb[s - 1];                       // fbar^{k+s-1}, row r+1
      const F4& B = (s == 1) ? lf1 : fo1[s - 1];      // f^{k+s-1}, row r
      const F4& EX = (s == 1) ? lp1x : po1x[s - 1];   // p^{k+s-1}, row r
      const F4& EY = (s == 1) ? lp1y : po1y[s - 1];
      const F4& Gv = gh[s - 1];                        // g, row r
      // the stage's coefficients
      const float lam_s = ALL ? c.slam[s - 1] : lam;
      const float tau_s = ALL ? c.stau[s - 1] : tau;
      const float sig_s = ALL ? c.ssig[s - 1] : sig;
      const float iopt_s = ALL ? prox_factor(tau_s) : iopt;
      const float thtau_s = ALL ? th * tau_s : thtau;
      const float nbr = from_right(cb.v[0]);
      F4 npx, npy;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float right = (j < 3) ? cb.v[j + 1] : nbr;
        const float gx = (!kEdge || xg + j < nx - 1) ? right - cb.v[j] : 0.0f;
        const float gy = dn ? nb.v[j] - cb.v[j] : 0.0f;
        project2(dual_arg(EX.v[j], sig_s, gx), dual_arg(EY.v[j], sig_s, gy), lam_s,
                 npx.v[j], npy.v[j]);
      }
      const float left = from_left(npx.v[3]);
      const bool up = !kEdge || r > 0;
      F4 fnew, fbnew;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float lp = (j == 0) ? ((!kEdge || xg > 0) ? left : 0.0f) : npx.v[j - 1];
        const float d = (npx.v[j] - lp) + (npy.v[j] - (up ? cy[s].v[j] : 0.0f));
        fnew.v[j] = data_prox(B.v[j], Gv.v[j], d, tau_s, iopt_s);
        fbnew.v[j] = PROX ? extrap_prox(fnew.v[j], Gv.v[j], d, thtau_s)
                          : extrap(fnew.v[j], B.v[j], th);
      }
      fo[s] = fnew;
      fb[s] = fbnew;
      pox[s] = npx;
      poy[s] = npy;
      if constexpr (ALL) {
        if (owned && r >= y0 && r < y1) {
          const int64_t o = (int64_t)r * P + xg;
          st4(c.SF[s - 1] + o, fnew);
          st4(c.SQX[s - 1] + o, npx);
          st4(c.SQY[s - 1] + o, npy);
        }
      }
      if constexpr (GAP) {
        // gap density and primal energy of (f^k, p^k) on row t
        // (the lane shuffles run on the whole wave: a row condition is the
        // same for every lane, the column condition is applied afterwards).
        // Each pixel's terms are formed in float32 and summed in float64:
        // rounding errors of a few units in the last place per term, of
        // either sign, bound the sum's error by 5e-7 P and leave it near 1e-9
        // P in practice, far below any stopping tolerance; the float64 terms
        // cost a third more instructions in this launch.
        // lambda |grad f| - <grad f, p> is subtracted in float64 (exactly).
        if (s == 1 && r >= y0 && r < y1) {
          const F4& A = L.f;                          // f^k, row r+1
          const float nfr = from_right(B.v[0]);
          const float lox = from_left(EX.v[3]);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (owned && (!kEdge || xg + j < nx)) {
              const float right = (j < 3) ? B.v[j + 1] : nfr;
              const float fv = B.v[j];
              const float gx = (!kEdge || xg + j < nx - 1) ? right - fv : 0.0f;
              const float gy = dn ? A.v[j] - fv : 0.0f;
              const float lo = (j == 0) ? ((!kEdge || xg > 0) ? lox : 0.0f) : EX.v[j - 1];
              const float uo = up ? lp2y.v[j] : 0.0f;
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
      }
    }
    // stores: f^{k+S} and p^{k+S} of stage S's row, inside the band
    if (!ALL && owned) {
      const int rS = t - (S - 1);
      if (rS >= y0 && rS < y1) {
        const int64_t o = (int64_t)rS * P + xg;
        st4(c.FN + o, fo[S]);
        st4(c.QX + o, pox[S]);
        st4(c.QY + o, poy[S]);
      }
    }
    // shift the histories
    lf1 = L.f;
    lp2y = lp1y;
    lp1x = L.px;
    lp1y = L.py;
#pragma unroll
    for (int s = S - 1; s > 0; --s) gh[s] = gh[s - 1];
    gh[0] = L.g;
#pragma unroll
    for (int s = 0; s < S; ++s) fbh[s] = fb[s];
#pragma unroll
    for (int s = 1; s < S; ++s) {
      fo1[s] = fo[s];
      po1x[s] = pox[s];
      po1y[s] = poy[s];
    }
#pragma unroll
    for (int s = 1; s <= S; ++s) cy[s] = poy[s];
  };

  // The histories start with row tb (its fbar^k lacks p_y of the row above:
  // such first-row values only feed rows outside the band); rows are
  // prefetched two steps ahead into three buffers used in turn.
  {
    XsLoad Z;
    load(tb, Z);
    lf1 = Z.f;
    lp1x = Z.px;
    lp1y = Z.py;
    gh[0] = Z.g;
    fbar_loaded(std::true_type{}, tb, Z, zero4(), fbh[0]);
  }
  XsLoad X, Y, Z;
  load(tb + 1, X);
  load(tb + 2, Y);
  constexpr std::integral_constant<int, S> kAll{};
  auto run = [&](auto edge) {
    int t = tb;
    for (; t + 2 <= te && t < tb + 2 * S - 1; t += 3) {
      load(t + 3, Z);
      step(edge, t, X, ramp(t));
      load(t + 4, X);
      step(edge, t + 1, Y, ramp(t + 1));
      load(t + 5, Y);
      step(edge, t + 2, Z, ramp(t + 2));
    }
    for (; t + 2 <= te; t += 3) {
      load(t + 3, Z);
      step(edge, t, X, kAll);
      load(t + 4, X);
      step(edge, t + 1, Y, kAll);
      load(t + 5, Y);
      step(edge, t + 2, Z, kAll);
    }
    // (a walk shorter than the ramp-up runs every stage on its last steps)
    if (t <= te) step(edge, t, X, kAll);
    if (t + 1 <= te) step(edge, t + 1, Y, kAll);
  };
  if constexpr (SPLIT) {
    if (interior)
      run(std::false_type{});
    else
      run(std::true_type{});
  } else {
    // the same loops written out: inside a lambda they cost registers
    constexpr std::true_type kE{};
    int t = tb;
    for (; t + 2 <= te && t < tb + 2 * S - 1; t += 3) {
      load(t + 3, Z);
      step(kE, t, X, ramp(t));
      load(t + 4, X);
      step(kE, t + 1, Y, ramp(t + 1));
      load(t + 5, Y);
      step(kE, t + 2, Z, ramp(t + 2));
    }
    for (; t + 2 <= te; t += 3) {
      load(t + 3, Z);
      step(kE, t, X, kAll);
      load(t + 4, X);
      step(kE, t + 1, Y, kAll);
      load(t + 5, Y);
      step(kE, t + 2, Z, kAll);
    }
    if (t <= te) step(kE, t, X, kAll);
    if (t + 1 <= te) step(kE, t + 1, Y, kAll);
  }
}

}  // namespace dev
}  // namespace tvpd
