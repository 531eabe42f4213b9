// Device code of the fused 2D adjoint sweep: one adjoint step of the
// unrolled solver over one tile (a 256-column strip by a band of rows), in a
// single pass over the data.
//
// Step k of the forward map is
//     fbar = f^k + theta (f^k - f^{k-1});  q = p^k + sigma grad fbar;
//     p^{k+1} = P_lam(q);  d = div p^{k+1};
//     f^{k+1} = (f^k + tau d + tau g) * (1 / (1 + tau)).
// Given a = dL/df^{k+1}, b (the share of dL/df^k collected from step k+1's
// extrapolation) and r = dL/dp^{k+1}, its reverse-mode derivative is
//     alpha = a / (1 + tau);  s = r - grad(tau alpha)          (forward diffs)
//     t = s inside the ball, else (lam/|q|)(s - n (n.s)), n = q/|q|
//     w = -sigma div t;  a' = alpha + b + (1 + theta) w;  b' = -theta w;
//     r' = t;  gbar += tau alpha;                              (backward diffs)
//     lambar += sum n.s (outside);  sigmabar += sum t.grad fbar;
//     taubar += sum alpha (d + g - f^{k+1}).
// The forward quantities are recomputed with the forward sweep's arithmetic
// (pointwise.h), so the projection takes the forward's branch.
//
// Layout of the walk: a wave owns a 256-column strip (one float4 per lane),
// walks a band of rows top to bottom carrying the previous row's p_y^{k+1}
// and t_y, takes x-neighbours from adjacent lanes, reads the strip's outer
// columns (x0-1, x0+256) at one shared address per row, and recomputes the
// values owned by other tiles (column x0-1, row y0-1) with the owner's
// arithmetic, so the result does not depend on the tiling.  Per pixel it reads f^k,
// f^{k-1}, p^k (2), g, a, b, r (2) and gbar, and writes a', b', r' (2) and
// gbar: 60 bytes, against 92 for a forward-difference pass followed by a
// backward-difference pass that hands p^{k+1} and t over through memory.
#pragma once

#include "pointwise.h"
#include "tile2d.h"

namespace tvpd {
namespace dev {

struct AdjCtx2D {
  const float* fk;
  const float* fkm;
  const float* px;   // p^k
  const float* py;
  const float* g;
  const float* a;    // a, b, r of step k+1
  const float* b;
  const float* rx;
  const float* ry;
  float* ao;         // a', b', r' = t
  float* bo;
  float* tx;
  float* ty;
  float* gbar;       // read and updated in place
  int ny, nx, pitch;
  int x0, y0, y1;
  float lam, tau, sig, th;
};

// Row data that is needed for the row itself and for the row above it.
struct AdjRowA {
  F4 f, m, a;
  float lf, lm, la;  // column x0-1
  float rf, rm, ra;  // column x0+256
};
// Row data needed for the row itself only.
struct AdjRowB {
  F4 px, py, rx, ry, b, g, gb;
  float lpx, lpy, lrx, lry;  // column x0-1
};

// t from s for a pixel with dual argument q (same branch as the forward).
__device__ __forceinline__ void adj_project2(float qx, float qy, float sx,
                                             float sy, float lam,
                                             float& tx, float& ty,
                                             float& ns_out, bool& outside) {
  const float n2 = sq2(qx, qy);
  const float rn = inv_norm(n2);
  outside = ball_scale_r(rn, lam) < 1.0f;
  const float nx = qx * rn, ny = qy * rn;
  float ns = nx * sx;
  ns = ns + ny * sy;
  const float sc = lam * rn;
  tx = outside ? sc * (sx - nx * ns) : sx;
  ty = outside ? sc * (sy - ny * ns) : sy;
  ns_out = ns;
}

__device__ __forceinline__ void adj_tile2d(const AdjCtx2D& c, double& acc_l,
                                           double& acc_s, double& acc_t) {
  const int lane = threadIdx.x & (kWave - 1);
  const int x0 = c.x0, y0 = c.y0, y1 = c.y1;
  const int nx = c.nx, ny = c.ny;
  const int64_t P = c.pitch;
  const int xc = x0 + kColsPerLane * lane;
  const bool lin = xc < c.pitch;
  const bool hl = (lane == 0) && (x0 > 0);
  const float lam = c.lam, tau = c.tau, sig = c.sig, th = c.th;
  const float iopt = prox_factor(tau);
  const float opth = 1.0f + th;
  const int xcl = min(xc, c.pitch - kColsPerLane);
  const int xlc = max(x0 - 1, 0);
  const int xrc = min(x0 + kStripCols, c.pitch - 1);

  auto loadA = [&](int y, AdjRowA& r) {
    const int64_t ro = (int64_t)min(max(y, 0), ny - 1) * P;
    r.f = ld4(c.fk + ro + xcl);
    r.m = ld4(c.fkm + ro + xcl);
    r.a = ld4(c.a + ro + xcl);
    r.lf = c.fk[ro + xlc];
    r.lm = c.fkm[ro + xlc];
    r.la = c.a[ro + xlc];
    r.rf = c.fk[ro + xrc];
    r.rm = c.fkm[ro + xrc];
    r.ra = c.a[ro + xrc];
  };
  auto loadB = [&](int y, AdjRowB& r) {
    const int64_t ro = (int64_t)min(max(y, 0), ny - 1) * P;
    r.px = ld4(c.px + ro + xcl);
    r.py = ld4(c.py + ro + xcl);
    r.rx = ld4(c.rx + ro + xcl);
    r.ry = ld4(c.ry + ro + xcl);
    r.b = ld4(c.b + ro + xcl);
    r.g = ld4(c.g + ro + xcl);
    r.gb = ld4(c.gbar + ro + xcl);
    r.lpx = c.px[ro + xlc];
    r.lpy = c.py[ro + xlc];
    r.lrx = c.rx[ro + xlc];
    r.lry = c.ry[ro + xlc];
  };

  F4 up_pn = zero4();  // p_y^{k+1} of the row above (0 above row 0)
  F4 up_t = zero4();   // t_y of the row above

  auto compute = [&](int y, const AdjRowA& cur, const AdjRowA& nxt,
                     const AdjRowB& pc) {
    const bool dn = y + 1 < ny;
    const bool own = y >= y0;
    // forward-difference part: p^{k+1} and t of every column of the strip
    F4 cb, nb, ta, tan;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      cb.v[j] = extrap(cur.f.v[j], cur.m.v[j], th);
      nb.v[j] = extrap(nxt.f.v[j], nxt.m.v[j], th);
      ta.v[j] = tau * (cur.a.v[j] * iopt);
      tan.v[j] = tau * (nxt.a.v[j] * iopt);
    }
    const float rb = extrap(cur.rf, cur.rm, th);
    const float rta = tau * (cur.ra * iopt);
    const float nbr = from_right(cb.v[0]);
    const float ntr = from_right(ta.v[0]);
    F4 pnx, pny, tx, ty;
    double lsum = 0.0, ssum = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool xf = xc + j < nx - 1;
      const float rgt =
          (j < 3) ? cb.v[(j + 1) & 3] : (lane == kWave - 1 ? rb : nbr);
      const float rgta =
          (j < 3) ? ta.v[(j + 1) & 3] : (lane == kWave - 1 ? rta : ntr);
      const float gx = xf ? rgt - cb.v[j] : 0.0f;
      const float gy = dn ? nb.v[j] - cb.v[j] : 0.0f;
      const float qx = dual_arg(pc.px.v[j], sig, gx);
      const float qy = dual_arg(pc.py.v[j], sig, gy);
      project2(qx, qy, lam, pnx.v[j], pny.v[j]);
      const float sx = pc.rx.v[j] - (xf ? rgta - ta.v[j] : 0.0f);
      const float sy = pc.ry.v[j] - (dn ? tan.v[j] - ta.v[j] : 0.0f);
      float ns;
      bool out;
      adj_project2(qx, qy, sx, sy, lam, tx.v[j], ty.v[j], ns, out);
      if (own && xc + j < nx) {
        if (out) lsum += ns;
        ssum += (double)tx.v[j] * (double)gx;
        ssum += (double)ty.v[j] * (double)gy;
      }
    }
    // p_x^{k+1} and t_x of the column to the left
    float l_pn = from_left(pnx.v[3]);
    float l_t = from_left(tx.v[3]);
    if (lane == 0) {
      l_pn = 0.0f;
      l_t = 0.0f;
      if (hl) {
        const float lb = extrap(cur.lf, cur.lm, th);
        const float lnb = extrap(nxt.lf, nxt.lm, th);
        const float lta = tau * (cur.la * iopt);
        const float ltan = tau * (nxt.la * iopt);
        const float gx = cb.v[0] - lb;
        const float gy = dn ? lnb - lb : 0.0f;
        const float qx = dual_arg(pc.lpx, sig, gx);
        const float qy = dual_arg(pc.lpy, sig, gy);
        float hx, hy;
        project2(qx, qy, lam, hx, hy);
        const float sx = pc.lrx - (ta.v[0] - lta);
        const float sy = pc.lry - (dn ? ltan - lta : 0.0f);
        float htx, hty, ns;
        bool out;
        adj_project2(qx, qy, sx, sy, lam, htx, hty, ns, out);
        l_pn = hx;
        l_t = htx;
      }
    }
    // backward-difference part on the band's own rows
    if (own) {
      F4 ao, bo, gbo;
      double tsum = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float lpn = (j == 0) ? l_pn : pnx.v[(j + 3) & 3];
        const float lt = (j == 0) ? l_t : tx.v[(j + 3) & 3];
        float d = pnx.v[j] - lpn;
        d = d + (pny.v[j] - up_pn.v[j]);
        const float fnew = data_prox(cur.f.v[j], pc.g.v[j], d, tau, iopt);
        const float alpha = cur.a.v[j] * iopt;
        gbo.v[j] = pc.gb.v[j] + tau * alpha;
        if (xc + j < nx)
          tsum += (double)alpha *
                  (((double)d + (double)pc.g.v[j]) - (double)fnew);
        float dt = tx.v[j] - lt;
        dt = dt + (ty.v[j] - up_t.v[j]);
        const float w = -sig * dt;
        ao.v[j] = (alpha + pc.b.v[j]) + opth * w;
        bo.v[j] = -th * w;
      }
      if (lin) {
        const int64_t o = (int64_t)y * P + xc;
        st4(c.ao + o, ao);
        st4(c.bo + o, bo);
        st4(c.tx + o, tx);
        st4(c.ty + o, ty);
        st4(c.gbar + o, gbo);
      }
      acc_l += lsum;
      acc_s += ssum;
      acc_t += tsum;
    }
    up_pn = pny;
    up_t = ty;
  };

  const int ys = y0 > 0 ? y0 - 1 : 0;
  const int ymain = min(y1 - 1, ny - 2);
  AdjRowA A0, A1, A2;
  AdjRowB B0, B1, B2;
  loadA(ys, A0);
  loadA(ys + 1, A1);
  loadB(ys, B0);
  int y = ys;
  const int ngroups = ymain > ys ? (ymain - ys) / 3 : 0;
  for (int grp = 0; grp < ngroups; ++grp, y += 3) {
    loadA(y + 2, A2);
    loadB(y + 1, B1);
    compute(y, A0, A1, B0);
    loadA(y + 3, A0);
    loadB(y + 2, B2);
    compute(y + 1, A1, A2, B1);
    loadA(y + 4, A1);
    loadB(y + 3, B0);
    compute(y + 2, A2, A0, B2);
  }
  AdjRowA cur = A0, nxt = A1;
  AdjRowB pc = B0;
  for (; y < y1; ++y) {
    AdjRowA nn;
    AdjRowB pn;
    loadA(y + 2, nn);
    loadB(y + 1, pn);
    compute(y, cur, nxt, pc);
    cur = nxt;
    nxt = nn;
    pc = pn;
  }
}

}  // namespace dev
}  // namespace tvpd
