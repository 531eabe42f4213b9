// Device code of the fused 3D adjoint sweep: one adjoint step of the
// unrolled solver (the recursion of adj2d.h with the z axis added) over one
// tile -- a 256-column strip, a band of TH rows and a segment of planes
// [z0, z1) -- in a single pass.
//
// The walk is that of the forward 3D tile (tile3d.h): the wave marches down
// the segment holding f^k, f^{k-1} and a of planes z and z+1 and the dual,
// r, b, g and gbar of plane z, carries p_z^{k+1} and t_z of plane z-1, and
// recomputes what other tiles own (column x0-1, row y0-1, and plane z0-1 in
// a prologue step that stores nothing).  Finished rows are refilled with the
// next planes' rows at once (rolling prefetch).  Per voxel it reads f^k,
// f^{k-1}, p^k (3), g, a, b, r (3), gbar and writes a', b', r' (3), gbar:
// 72 bytes, against 116 for the two-pass form.
#pragma once

#include "adj2d.h"
#include "tile3d.h"

namespace tvpd {
namespace dev {

struct AdjCtx3D {
  const float* fk;
  const float* fkm;
  const float* pk;   // x; y at +cs, z at +2 cs
  const float* g;
  const float* a;
  const float* b;
  const float* r;    // x; y at +cs, z at +2 cs
  float* ao;
  float* bo;
  float* t;          // x; y at +cs, z at +2 cs
  float* gbar;
  int64_t cs;
  int nz, ny, nx, pitch;
  int x0, y0, z0, z1;
  float lam, tau, sig, th;
};

template <int TH>
struct AdjPlaneF {
  F4 f[TH + 2], m[TH + 2], a[TH + 2];  // rows y0-1 .. y0+TH
  float lf[TH + 2], lm[TH + 2], la[TH + 2];  // column x0-1
  float rf[TH + 2], rm[TH + 2], ra[TH + 2];  // column x0+256
};

template <int TH>
struct AdjPlaneP {
  F4 px[TH + 1], py[TH + 1], pz[TH + 1];  // rows y0-1 .. y0+TH-1
  F4 rx[TH + 1], ry[TH + 1], rz[TH + 1];
  float lpx[TH], lpy[TH], lpz[TH];        // column x0-1, rows y0 ..
  float lrx[TH], lry[TH], lrz[TH];
  F4 b[TH], g[TH], gb[TH];                // rows y0 .. y0+TH-1
};

// t from s for a voxel with dual argument q (same branch as the forward).
__device__ __forceinline__ void adj_project3(float qx, float qy, float qz,
                                             float sx, float sy, float sz,
                                             float lam, float& tx,
                                             float& ty, float& tz,
                                             float& ns_out, bool& outside) {
  const float n2 = sq3(qx, qy, qz);
  const float rn = inv_norm(n2);
  outside = ball_scale_r(rn, lam) < 1.0f;
  const float ux = qx * rn, uy = qy * rn, uz = qz * rn;
  float ns = ux * sx;
  ns = ns + uy * sy;
  ns = ns + uz * sz;
  const float sc = lam * rn;
  tx = outside ? sc * (sx - ux * ns) : sx;
  ty = outside ? sc * (sy - uy * ns) : sy;
  tz = outside ? sc * (sz - uz * ns) : sz;
  ns_out = ns;
}

template <int TH>
__device__ __forceinline__ void adj_tile3d(const AdjCtx3D& c, double& acc_l,
                                           double& acc_s, double& acc_t) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t cs = c.cs;
  const int nz = c.nz, ny = c.ny, nx = c.nx;
  const int64_t P = c.pitch;
  const int64_t SZ = (int64_t)ny * P;
  const int x0 = c.x0, y0 = c.y0, z0 = c.z0, z1 = c.z1;
  const int xc = x0 + kColsPerLane * lane;
  const bool lin = xc < c.pitch;
  const bool hl = x0 > 0;
  const float lam = c.lam, tau = c.tau, sig = c.sig, th = c.th;
  const float iopt = prox_factor(tau);
  const float opth = 1.0f + th;
  const int xcl = min(xc, c.pitch - kColsPerLane);
  const int xlc = max(x0 - 1, 0);
  const int xrc = min(x0 + kStripCols, c.pitch - 1);

  auto rowc = [&](int y) { return min(max(y, 0), ny - 1); };

  auto loadFrow = [&](int z, AdjPlaneF<TH>& b, int r) {
    const int64_t o =
        (int64_t)min(z, nz - 1) * SZ + (int64_t)rowc(y0 - 1 + r) * P;
    b.f[r] = ld4(c.fk + o + xcl);
    b.m[r] = ld4(c.fkm + o + xcl);
    b.a[r] = ld4(c.a + o + xcl);
    if (r >= 1) {
      b.lf[r] = c.fk[o + xlc];
      b.lm[r] = c.fkm[o + xlc];
      b.la[r] = c.a[o + xlc];
    } else {
      b.lf[r] = b.lm[r] = b.la[r] = 0.0f;
    }
    if (r <= TH) {
      b.rf[r] = c.fk[o + xrc];
      b.rm[r] = c.fkm[o + xrc];
      b.ra[r] = c.a[o + xrc];
    } else {
      b.rf[r] = b.rm[r] = b.ra[r] = 0.0f;
    }
  };
  auto loadProw = [&](int z, AdjPlaneP<TH>& b, int i) {
    const int64_t zo = (int64_t)z * SZ;
    const int64_t o = zo + (int64_t)rowc(y0 - 1 + i) * P + xcl;
    b.px[i] = ld4(c.pk + o);
    b.py[i] = ld4(c.pk + cs + o);
    b.pz[i] = ld4(c.pk + 2 * cs + o);
    b.rx[i] = ld4(c.r + o);
    b.ry[i] = ld4(c.r + cs + o);
    b.rz[i] = ld4(c.r + 2 * cs + o);
    if (i < TH) {
      const int64_t q = zo + (int64_t)rowc(y0 + i) * P;
      b.lpx[i] = c.pk[q + xlc];
      b.lpy[i] = c.pk[cs + q + xlc];
      b.lpz[i] = c.pk[2 * cs + q + xlc];
      b.lrx[i] = c.r[q + xlc];
      b.lry[i] = c.r[cs + q + xlc];
      b.lrz[i] = c.r[2 * cs + q + xlc];
      b.b[i] = ld4(c.b + q + xcl);
      b.g[i] = ld4(c.g + q + xcl);
      b.gb[i] = ld4(c.gbar + q + xcl);
    }
  };

  F4 pzn[TH], tzc[TH];  // p_z^{k+1} and t_z of plane z-1 (0 before z = 0)
#pragma unroll
  for (int r = 0; r < TH; ++r) {
    pzn[r] = zero4();
    tzc[r] = zero4();
  }

  auto step = [&](int z, AdjPlaneF<TH>& cur, const AdjPlaneF<TH>& nxt,
                  AdjPlaneP<TH>& pc) {
    const bool own = z >= z0;
    const bool zf = z + 1 < nz;
    const int64_t zo = (int64_t)z * SZ;
    const int zF = min(z + 2, z1);
    const int zP = min(z + 1, z1 - 1);
    F4 up_pn = zero4(), up_t = zero4();
#pragma unroll
    for (int r = 0; r < TH + 1; ++r) {
      const int y = y0 - 1 + r;
      const bool active = (r == 0) ? (own && y0 > 0) : (y < ny);
      if (active) {
        const bool dn = y + 1 < ny;
        F4 cb, db, zb, ta, tad, taz;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cb.v[j] = extrap(cur.f[r].v[j], cur.m[r].v[j], th);
          db.v[j] = extrap(cur.f[r + 1].v[j], cur.m[r + 1].v[j], th);
          zb.v[j] = extrap(nxt.f[r].v[j], nxt.m[r].v[j], th);
          ta.v[j] = tau * (cur.a[r].v[j] * iopt);
          tad.v[j] = tau * (cur.a[r + 1].v[j] * iopt);
          taz.v[j] = tau * (nxt.a[r].v[j] * iopt);
        }
        const float rb = extrap(cur.rf[r], cur.rm[r], th);
        const float rta = tau * (cur.ra[r] * iopt);
        const float nbr = from_right(cb.v[0]);
        const float ntr = from_right(ta.v[0]);
        F4 pnx, pny, pnz, tx, ty, tz;
        double lsum = 0.0, ssum = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool xf = xc + j < nx - 1;
          const float rgt =
              (j < 3) ? cb.v[(j + 1) & 3] : (lane == kWave - 1 ? rb : nbr);
          const float rgta =
              (j < 3) ? ta.v[(j + 1) & 3] : (lane == kWave - 1 ? rta : ntr);
          const float gx = xf ? rgt - cb.v[j] : 0.0f;
          const float gy = dn ? db.v[j] - cb.v[j] : 0.0f;
          const float gz = zf ? zb.v[j] - cb.v[j] : 0.0f;
          const float qx = dual_arg(pc.px[r].v[j], sig, gx);
          const float qy = dual_arg(pc.py[r].v[j], sig, gy);
          const float qz = dual_arg(pc.pz[r].v[j], sig, gz);
          project3(qx, qy, qz, lam, pnx.v[j], pny.v[j], pnz.v[j]);
          const float sx = pc.rx[r].v[j] - (xf ? rgta - ta.v[j] : 0.0f);
          const float sy = pc.ry[r].v[j] - (dn ? tad.v[j] - ta.v[j] : 0.0f);
          const float sz = pc.rz[r].v[j] - (zf ? taz.v[j] - ta.v[j] : 0.0f);
          float ns;
          bool out;
          adj_project3(qx, qy, qz, sx, sy, sz, lam, tx.v[j], ty.v[j],
                       tz.v[j], ns, out);
          if (xc + j < nx) {
            if (out) lsum += ns;
            ssum += (double)tx.v[j] * (double)gx;
            ssum += (double)ty.v[j] * (double)gy;
            ssum += (double)tz.v[j] * (double)gz;
          }
        }
        if (r > 0) {
          const int ri = r - 1;
          if (own) {
            // p_x^{k+1} and t_x of the column to the left
            float l_pn = from_left(pnx.v[3]);
            float l_t = from_left(tx.v[3]);
            if (hl) {
              const float lb = extrap(cur.lf[r], cur.lm[r], th);
              const float ldb =
                  extrap(cur.lf[r + 1], cur.lm[r + 1], th);
              const float lzb = extrap(nxt.lf[r], nxt.lm[r], th);
              const float lta = tau * (cur.la[r] * iopt);
              const float ltad = tau * (cur.la[r + 1] * iopt);
              const float ltaz = tau * (nxt.la[r] * iopt);
              const float gx = cb.v[0] - lb;
              const float gy = dn ? ldb - lb : 0.0f;
              const float gz = zf ? lzb - lb : 0.0f;
              const float qx = dual_arg(pc.lpx[ri], sig, gx);
              const float qy = dual_arg(pc.lpy[ri], sig, gy);
              const float qz = dual_arg(pc.lpz[ri], sig, gz);
              float hx, hy, hz;
              project3(qx, qy, qz, lam, hx, hy, hz);
              const float sx = pc.lrx[ri] - (ta.v[0] - lta);
              const float sy = pc.lry[ri] - (dn ? ltad - lta : 0.0f);
              const float sz = pc.lrz[ri] - (zf ? ltaz - lta : 0.0f);
              float htx, hty, htz, ns;
              bool out;
              adj_project3(qx, qy, qz, sx, sy, sz, lam, htx, hty, htz,
                           ns, out);
              if (lane == 0) {
                l_pn = hx;
                l_t = htx;
              }
            } else if (lane == 0) {
              l_pn = 0.0f;
              l_t = 0.0f;
            }
            F4 ao, bo, gbo;
            double tsum = 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const float lpn = (j == 0) ? l_pn : pnx.v[(j + 3) & 3];
              const float lt = (j == 0) ? l_t : tx.v[(j + 3) & 3];
              float d = pnx.v[j] - lpn;
              d = d + (pny.v[j] - up_pn.v[j]);
              d = d + (pnz.v[j] - pzn[ri].v[j]);
              const float fnew = data_prox(cur.f[r].v[j], pc.g[ri].v[j], d, tau, iopt);
              const float alpha = cur.a[r].v[j] * iopt;
              gbo.v[j] = pc.gb[ri].v[j] + tau * alpha;
              if (xc + j < nx)
                tsum += (double)alpha *
                        (((double)d + (double)pc.g[ri].v[j]) - (double)fnew);
              float dt = tx.v[j] - lt;
              dt = dt + (ty.v[j] - up_t.v[j]);
              dt = dt + (tz.v[j] - tzc[ri].v[j]);
              const float w = -sig * dt;
              ao.v[j] = (alpha + pc.b[ri].v[j]) + opth * w;
              bo.v[j] = -th * w;
            }
            if (lin) {
              const int64_t o = zo + (int64_t)y * P + xc;
              st4(c.ao + o, ao);
              st4(c.bo + o, bo);
              st4(c.t + o, tx);
              st4(c.t + cs + o, ty);
              st4(c.t + 2 * cs + o, tz);
              st4(c.gbar + o, gbo);
            }
            acc_l += lsum;
            acc_s += ssum;
            acc_t += tsum;
          }
          pzn[ri] = pnz;
          tzc[ri] = tz;
        }
        up_pn = pny;
        up_t = ty;
      }
      if (r >= 1) loadProw(zP, pc, r - 1);
      loadFrow(zF, cur, r);
    }
    loadProw(zP, pc, TH);
    loadFrow(zF, cur, TH + 1);
  };

  const int zs = z0 > 0 ? z0 - 1 : 0;
  AdjPlaneF<TH> A, B;
  AdjPlaneP<TH> Q;
#pragma unroll
  for (int r = 0; r < TH + 2; ++r) {
    loadFrow(zs, A, r);
    loadFrow(zs + 1, B, r);
  }
#pragma unroll
  for (int i = 0; i < TH + 1; ++i) loadProw(zs, Q, i);
  int z = zs;
  for (; z + 1 < z1; z += 2) {
    step(z, A, B, Q);
    step(z + 1, B, A, Q);
  }
  if (z < z1) step(z, A, B, Q);
}

}  // namespace dev
}  // namespace tvpd
