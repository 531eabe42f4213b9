// Device code of the fused 3D sweep over one tile: a 256-column strip, a band
// of TH rows and a segment of planes [z0, z1).  Shared by the plain 3D solver
// and the unrolled 3D forward, so both perform bit-identical arithmetic.
//
// One call performs iteration k -> k+1 of the primal-dual method on the
// tile's voxels (the same update as the 2D tile, with the z axis added):
//     fbar    = f^k + theta (f^k - f^{k-1})
//     p^{k+1} = P_lam(p^k + sigma grad fbar)          (3-vector projection)
//     f^{k+1} = (f^k + tau div p^{k+1} + tau g) / (1 + tau)
// and, with GAP, accumulates the gap density and primal energy of
// (f^k, p^k) in float64.
//
// A wave owns the strip (one float4 per lane) for TH rows and marches down
// the segment plane by plane.  At plane z it holds f^k, f^{k-1} of planes z
// and z+1 (rows y0-1 .. y0+TH) and p^k, g of plane z; it carries p_z^{k+1}
// (and, for the gap, p_z^k) of plane z-1 from the previous step.  As soon as
// a row of plane z is finished, its registers are refilled with the same row
// of plane z+2 (f) and z+1 (p, g), so every load has a whole plane step of
// time to arrive and the march never waits on a fresh load.  Values
// owned by other tiles are recomputed here with the owner's arithmetic:
// p_y^{k+1} of row y0-1 (for div at row y0), p_x^{k+1} of column x0-1 (for
// div at column x0) and, on the segment's first plane, p_z^{k+1} of plane
// z0-1 (a prologue step that stores nothing).  The iterates therefore do not
// depend on the tiling.  Every load address is clamped into the volume;
// values read at clamped addresses are masked out.
#pragma once

#include "tile2d.h"

namespace tvpd {
namespace dev {

// Pointers and sizes of one 3D tile at iteration k.
struct Tile3DCtx {
  const float* fk;   // f^k
  const float* fkm;  // f^{k-1}
  const float* pk;   // p^k: x component; y at +cs, z at +2 cs
  const float* g;
  float* fn;         // f^{k+1}
  float* pn;         // p^{k+1}: x; y at +cs, z at +2 cs
  int64_t cs;        // floats between dual components
  int nz, ny, nx, pitch;
  int x0, y0, z0, z1;  // strip start, band rows [y0, y0+TH), planes [z0, z1)
  float lam, tau, sig, th;
};

// Projection of q onto the ball of radius lam.
__device__ __forceinline__ void project3(float qx, float qy, float qz,
                                         float lam, float& px,
                                         float& py, float& pz) {
  const float c = ball_scale(sq3(qx, qy, qz), lam);
  px = qx * c;
  py = qy * c;
  pz = qz * c;
}

// f^k and f^{k-1} of one plane of the tile: rows y0-1 .. y0+TH (index r is
// row y0-1+r), with the strip's outer columns.
template <int TH>
struct Plane3F {
  F4 f[TH + 2], m[TH + 2];
  float lf[TH + 2], lm[TH + 2];  // column x0-1 (rows y0 .. y0+TH used)
  float rf[TH + 2], rm[TH + 2];  // column x0+256 (rows y0-1 .. y0+TH-1 used)
};

// p^k and g of one plane: dual rows y0-1 .. y0+TH-1 (index r is row y0-1+r),
// the dual at column x0-1 and g for the band's rows (index r is row y0+r).
template <int TH>
struct Plane3P {
  F4 px[TH + 1], py[TH + 1], pz[TH + 1];
  float lx[TH], ly[TH], lz[TH];
  F4 g[TH];
};

template <int TH, bool GAP>
__device__ __forceinline__ void sweep_tile3d(const Tile3DCtx& c,
                                             double& acc_gap, double& acc_P) {
  const int lane = threadIdx.x & (kWave - 1);
  const float* __restrict__ fk = c.fk;
  const float* __restrict__ fkm = c.fkm;
  const float* __restrict__ pk = c.pk;
  const float* __restrict__ gp = c.g;
  float* __restrict__ fn = c.fn;
  float* __restrict__ pn = c.pn;
  const int64_t cs = c.cs;
  const int nz = c.nz, ny = c.ny, nx = c.nx;
  const int64_t P = c.pitch;
  const int64_t SZ = (int64_t)ny * P;
  const int x0 = c.x0, y0 = c.y0, z0 = c.z0, z1 = c.z1;
  const int xc = x0 + kColsPerLane * lane;
  const bool lin = xc < c.pitch;
  const bool hl = x0 > 0;                       // a column x0-1 exists
  const float lam = c.lam, tau = c.tau, sig = c.sig, th = c.th;
  const float iopt = prox_factor(tau);
  const int xcl = min(xc, c.pitch - kColsPerLane);
  const int xlc = max(x0 - 1, 0);
  const int xrc = min(x0 + kStripCols, c.pitch - 1);

  auto rowc = [&](int y) { return min(max(y, 0), ny - 1); };

  // Row r (row y0-1+r) of plane z of f^k, f^{k-1}.
  auto loadFrow = [&](int z, Plane3F<TH>& b, int r) {
    const int64_t o =
        (int64_t)min(z, nz - 1) * SZ + (int64_t)rowc(y0 - 1 + r) * P;
    b.f[r] = ld4(fk + o + xcl);
    b.m[r] = ld4(fkm + o + xcl);
    if (r >= 1) {
      b.lf[r] = fk[o + xlc];
      b.lm[r] = fkm[o + xlc];
    } else {
      b.lf[r] = b.lm[r] = 0.0f;
    }
    if (r <= TH) {
      b.rf[r] = fk[o + xrc];
      b.rm[r] = fkm[o + xrc];
    } else {
      b.rf[r] = b.rm[r] = 0.0f;
    }
  };
  // Dual row i (row y0-1+i) of plane z and, for i < TH, the column-x0-1
  // dual and g of row y0+i.
  auto loadProw = [&](int z, Plane3P<TH>& b, int i) {
    const int64_t zo = (int64_t)z * SZ;
    const int64_t o = zo + (int64_t)rowc(y0 - 1 + i) * P + xcl;
    b.px[i] = ld4(pk + o);
    b.py[i] = ld4(pk + cs + o);
    b.pz[i] = ld4(pk + 2 * cs + o);
    if (i < TH) {
      const int64_t q = zo + (int64_t)rowc(y0 + i) * P;
      b.lx[i] = pk[q + xlc];
      b.ly[i] = pk[cs + q + xlc];
      b.lz[i] = pk[2 * cs + q + xlc];
      b.g[i] = ld4(gp + q + xcl);
    }
  };

  F4 pzn[TH], pzo[TH];  // p_z^{k+1} and p_z^k of plane z-1 (0 before z = 0)
#pragma unroll
  for (int r = 0; r < TH; ++r) {
    pzn[r] = zero4();
    pzo[r] = zero4();
  }

  // One plane z: cur = plane z, nxt = plane z+1, pc = p^k and g of plane z.
  // Finished rows of cur are refilled from plane min(z+2, z1) and those of
  // pc from plane min(z+1, z1-1) (planes past the segment are not needed;
  // the clamped re-reads hit the cache).
  auto step = [&](int z, Plane3F<TH>& cur, const Plane3F<TH>& nxt,
                  Plane3P<TH>& pc) {
    const bool own = z >= z0;
    const bool zf = z + 1 < nz;
    const int64_t zo = (int64_t)z * SZ;
    const int zF = min(z + 2, z1);
    const int zP = min(z + 1, z1 - 1);
    F4 up = zero4();  // p_y^{k+1} of the row above
#pragma unroll
    for (int r = 0; r < TH + 1; ++r) {
      const int y = y0 - 1 + r;
      // row y0-1 is needed only for div at row y0, and only inside the image
      const bool active = (r == 0) ? (own && y0 > 0) : (y < ny);
      if (active) {
        const bool dn = y + 1 < ny;
        F4 cb, db, zb;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cb.v[j] = extrap(cur.f[r].v[j], cur.m[r].v[j], th);
          db.v[j] = extrap(cur.f[r + 1].v[j], cur.m[r + 1].v[j], th);
          zb.v[j] = extrap(nxt.f[r].v[j], nxt.m[r].v[j], th);
        }
        const float rb = extrap(cur.rf[r], cur.rm[r], th);
        const float nbr = from_right(cb.v[0]);
        F4 npx, npy, npz;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float right =
              (j < 3) ? cb.v[(j + 1) & 3] : (lane == kWave - 1 ? rb : nbr);
          const float gx = (xc + j < nx - 1) ? right - cb.v[j] : 0.0f;
          const float gy = dn ? db.v[j] - cb.v[j] : 0.0f;
          const float gz = zf ? zb.v[j] - cb.v[j] : 0.0f;
          project3(dual_arg(pc.px[r].v[j], sig, gx), dual_arg(pc.py[r].v[j], sig, gy),
                   dual_arg(pc.pz[r].v[j], sig, gz), lam, npx.v[j], npy.v[j],
                   npz.v[j]);
        }
        if (r > 0) {
          const int ri = r - 1;  // index among the band's rows
          if (own) {
            // p_x^{k+1} of the column to the left (0 left of the image):
            // every lane evaluates it from the shared column values, lane 0
            // uses it; hl is the same for the whole wave
            float left_n = from_left(npx.v[3]);
            if (hl) {
              const float lb = extrap(cur.lf[r], cur.lm[r], th);
              const float ldb =
                  extrap(cur.lf[r + 1], cur.lm[r + 1], th);
              const float lzb = extrap(nxt.lf[r], nxt.lm[r], th);
              const float gx = cb.v[0] - lb;
              const float gy = dn ? ldb - lb : 0.0f;
              const float gz = zf ? lzb - lb : 0.0f;
              float hx, hy, hz;
              project3(dual_arg(pc.lx[ri], sig, gx), dual_arg(pc.ly[ri], sig, gy),
                       dual_arg(pc.lz[ri], sig, gz), lam, hx, hy, hz);
              if (lane == 0) left_n = hx;
            } else if (lane == 0) {
              left_n = 0.0f;
            }
            F4 fnew;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const float lp = (j == 0) ? left_n : npx.v[(j + 3) & 3];
              float d = (npx.v[j] - lp) + (npy.v[j] - up.v[j]);
              d = d + (npz.v[j] - pzn[ri].v[j]);
              fnew.v[j] = data_prox(cur.f[r].v[j], pc.g[ri].v[j], d, tau, iopt);
            }
            if (lin) {
              const int64_t o = zo + (int64_t)y * P + xc;
              st4(fn + o, fnew);
              st4(pn + o, npx);
              st4(pn + cs + o, npy);
              st4(pn + 2 * cs + o, npz);
            }
            if constexpr (GAP) {
              const F4& cf = cur.f[r];
              const float nfr = from_right(cf.v[0]);
              float left_o = from_left(pc.px[r].v[3]);
              if (lane == 0) left_o = hl ? pc.lx[ri] : 0.0f;
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (xc + j < nx) {
                  const float right =
                      (j < 3) ? cf.v[(j + 1) & 3]
                              : (lane == kWave - 1 ? cur.rf[r] : nfr);
                  const double fv = cf.v[j];
                  const double gx =
                      (xc + j < nx - 1) ? (double)right - fv : 0.0;
                  const double gy =
                      dn ? (double)cur.f[r + 1].v[j] - fv : 0.0;
                  const double gz = zf ? (double)nxt.f[r].v[j] - fv : 0.0;
                  const double lo =
                      (j == 0) ? left_o : pc.px[r].v[(j + 3) & 3];
                  const double uo =
                      (y > 0) ? (double)pc.py[r - 1].v[j] : 0.0;
                  double d = ((double)pc.px[r].v[j] - lo) +
                             ((double)pc.py[r].v[j] - uo);
                  d = d + ((double)pc.pz[r].v[j] - (double)pzo[ri].v[j]);
                  const double e = fv - (double)pc.g[ri].v[j];
                  const double res = e - d;
                  const double nrm = sqrt(gx * gx + gy * gy + gz * gz);
                  acc_gap += 0.5 * res * res + (double)lam * nrm -
                             (gx * (double)pc.px[r].v[j] +
                              gy * (double)pc.py[r].v[j] +
                              gz * (double)pc.pz[r].v[j]);
                  acc_P += 0.5 * e * e + (double)lam * nrm;
                }
              }
            }
          }
          pzn[ri] = npz;
          if constexpr (GAP) pzo[ri] = pc.pz[r];
        }
        up = npy;
      }
      // refill what no later row of this plane reads
      if (r >= 1) loadProw(zP, pc, r - 1);
      loadFrow(zF, cur, r);
    }
    loadProw(zP, pc, TH);
    loadFrow(zF, cur, TH + 1);
  };

  const int zs = z0 > 0 ? z0 - 1 : 0;
  Plane3F<TH> A, B;
  Plane3P<TH> Q;
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
