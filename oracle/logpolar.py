"""FP64 oracle for the log-polar backprojection (test infrastructure only).

Andersson's formula (Section 2.1, eq. and_approach and and_kernel; the change
of variables of eq. andersson): in log-polar coordinates x = R e^rho xi_theta
the backprojection is a two-dimensional convolution,

    [B g]_L(rho, theta) = int int [g]_L(mu, phi) K(rho - mu, theta - phi) dmu dphi,
    K(a, b) = delta(1 - e^a cos b),

where [g]_L(mu, phi) = g_P(R e^mu, phi) is the sinogram on the semi-polar mesh
(a ray of angle phi in [0, 2 pi) carries g(s, phi) for phi < pi and g(-s,
phi - pi) beyond).  The delta has a unit derivative at its root a = -ln cos b,
so the formula sums, over the rays through x, the sinogram at the foot of the
perpendicular: the circle through the origin and x.

Geometry: the tomography oracle's (``oracle.tomo``): pixel units, detector
bins t_i = i + 1/2 - n_det/2, angles theta_k = k pi / n_angles, B = dtheta A^T
for sampled data.  The paper's unit disc is the detector's: R = n_det / 2.

The algorithm of Section 5 ("Algorithm for log-polar backprojection") in its
four steps, with the mesh of the table of symbols and the adaptive rho_0 of
"Problem near the origin":

  Step 1. [g]_s -> [g]_L: every ray of the semi-polar mesh (2 n_angles angles
          phi_j = j pi / n_angles) is the sinogram row of angle phi_j mod pi,
          read at t = +-s; linear interpolation along it at the log-polar
          radii R e^{rho_i} (zero beyond the detector's ends, as in A^T).
  Step 2. The kernel on the lag mesh a_m = m drho: height 1/drho at the
          root of e^a cos phi_j = 1, falling linearly in a to 0 one step
          away; nonzero on the band where e^{a_m} cos phi_j lies within a
          factor e^{+-drho} of 1, which is the paper's band |e^{a_m} cos phi_j
          - 1| <= drho (eq. calc_and_kernel) to first order (reading below).
  Step 3. The convolution by FFTs: periodic in the angle (2 pi), linear in
          rho (zero-padded to at least 2 N_rho - 1), with the quadrature
          weights drho dphi.
  Step 4. Bilinear interpolation of the log-polar result at every pixel
          centre (rho = ln(r / R), theta = atan2(y, x) in [0, 2 pi)).

Readings where the paper is silent, ambiguous or at odds with itself:
  * The mesh (table of symbols and eq. N_rho): rho_0 = ln(min(dx, dy) / 2)
    with the pixel size dx = dy = 1 / R, i.e. the second form of eq. N_rho,
    ln(min(1/N_x, 1/N_y)) on the paper's [-1, 1] square: the innermost ring
    lies half a pixel from the origin (the first form, rho_0 < ln(min(dx,
    dy)), would leave the four pixels around the centre of an even grid
    below the mesh).  The step follows eq. N_rho with ds = 2 / N_t:
    N_rho = ceil((rho_top - rho_0) / -ln(1 - ds)), drho = (rho_top - rho_0) /
    N_rho, nodes rho_i = rho_0 + (i + 1) drho, i = 0 .. N_rho - 1, so that
    the top node is rho_top and the largest radial step is at most one bin
    (the table's rho mesh ends at ln 1 with the first node one step above
    rho_0).  rho_top = 0 (r = R), raised to ln(r_max / R) when the image's
    corners lie outside the detector's disc, so that every pixel centre is
    inside the mesh (beyond the detector the sinogram is zero).
  * The kernel's argument: the convolution's lag rho - mu is >= 0 on the
    kernel's support, so the kernel is sampled on the lag mesh a_m = m drho,
    m >= 0 (on the image mesh rho <= 0 the printed condition only holds at
    the origin).
  * The kernel's values: taken literally, height 1/drho on the band
    |e^a cos b - 1| <= drho puts 2 or 3 lag nodes on every angle, a discrete
    mass of 2 to 3 where the delta has mass 1.  The hat
    (1/drho) max(0, 1 - |a + ln cos b| / drho) has the same peak and, to
    first order, the same band; its lag samples sum to exactly 1 (a partition
    of unity), so that the sum over lags is the linear interpolation of [g]_L
    at the foot point mu = rho + ln cos b.  It is the linear-interpolation
    form of a delta on a level set, the kind of improvement the paper points
    to after eq. calc_and_kernel.
  * Pixels nearer the origin than the first node (the centre pixel of an odd
    grid) take the first node's value; the angle is periodic.

Plain NumPy in float64; the FFTs are numpy's.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Mesh:
    R: float          # detector half-width in pixels (the unit of the paper's disc)
    rho0: float       # the mesh's lower end (the first node is rho0 + drho)
    drho: float
    n_rho: int
    n_phi: int        # 2 n_angles rays over [0, 2 pi)
    dphi: float       # pi / n_angles

    def rho(self) -> np.ndarray:
        return self.rho0 + (np.arange(self.n_rho) + 1.0) * self.drho

    def phi(self) -> np.ndarray:
        return np.arange(self.n_phi) * self.dphi


def mesh(H: int, W: int, n_angles: int, n_det: int) -> Mesh:
    """The log-polar mesh of the readings above."""
    if n_det < 4:
        raise ValueError("n_det >= 4")
    R = n_det / 2.0
    ds = 2.0 / n_det
    rho0 = math.log(0.5 / R)
    r_max = math.hypot(W / 2.0 - 0.5, H / 2.0 - 0.5)
    rho_top = max(0.0, math.log(r_max / R)) if r_max > 0 else 0.0
    n_rho = int(math.ceil((rho_top - rho0) / -math.log(1.0 - ds)))
    drho = (rho_top - rho0) / n_rho
    return Mesh(R, rho0, drho, n_rho, 2 * n_angles, math.pi / n_angles)


def conv_length(m: Mesh) -> int:
    """Length of the zero-padded rho axis: the smallest power of two >=
    2 n_rho - 1 (the linear convolution of two n_rho-long sequences)."""
    L = 1
    while L < 2 * m.n_rho - 1:
        L *= 2
    return L


def to_logpolar(s: np.ndarray, m: Mesh) -> np.ndarray:
    """Step 1: [g]_L[j, i] = sinogram row (j mod n_angles) at t = +-R e^{rho_i}
    (+ for j < n_angles), linear in t.  Shape (n_phi, n_rho)."""
    s = np.asarray(s, dtype=np.float64)
    n_angles, n_det = s.shape
    r = m.R * np.exp(m.rho())
    out = np.empty((m.n_phi, m.n_rho))
    for j in range(m.n_phi):
        k, sign = (j, 1.0) if j < n_angles else (j - n_angles, -1.0)
        ext = np.concatenate(([0.0], s[k], [0.0]))   # ext[i + 1] = s[k, i]
        v = sign * r + n_det / 2.0 - 0.5               # bin index of t
        i0 = np.floor(v).astype(np.int64)
        w = v - i0
        lo = np.clip(i0, -1, n_det) + 1
        hi = np.clip(i0 + 1, -1, n_det) + 1
        out[j] = (1.0 - w) * ext[lo] + w * ext[hi]
    return out


def kernel(m: Mesh, n_lags: int | None = None) -> np.ndarray:
    """Step 2: k[j, l] at angle offset phi_j and lag a_l = l drho (eq.
    calc_and_kernel, hat reading).  Shape (n_phi, n_lags), n_lags = n_rho.
    Zero where cos phi_j <= 0 (no root)."""
    n_lags = m.n_rho if n_lags is None else n_lags
    a = np.arange(n_lags) * m.drho
    c = np.cos(m.phi())
    out = np.zeros((m.n_phi, n_lags))
    pos = c > 0.0
    root = -np.log(c[pos])                     # e^a cos phi = 1
    out[pos] = np.maximum(0.0, 1.0 - np.abs(a[None, :] - root[:, None]) / m.drho)
    return out / m.drho


def convolve(gL: np.ndarray, k: np.ndarray, m: Mesh) -> np.ndarray:
    """Step 3: out[j, i] = drho dphi sum_{j', l <= i} k[j', l] gL[(j - j') mod
    n_phi, i - l], by FFTs (angle periodic, rho zero-padded)."""
    L = conv_length(m)
    G = np.fft.fft2(gL, s=(m.n_phi, L))
    Kf = np.fft.fft2(k, s=(m.n_phi, L))
    out = np.real(np.fft.ifft2(G * Kf))[:, :m.n_rho]
    return m.drho * m.dphi * out


def to_cartesian(bL: np.ndarray, m: Mesh, H: int, W: int) -> np.ndarray:
    """Step 4: bilinear in (rho, theta) at the pixel centres."""
    x = np.arange(W) + 0.5 - W / 2.0
    y = np.arange(H) + 0.5 - H / 2.0
    X, Y = np.meshgrid(x, y)
    r = np.hypot(X, Y)
    with np.errstate(divide="ignore"):
        rho = np.log(r / m.R)
    u = np.clip((rho - (m.rho0 + m.drho)) / m.drho, 0.0, m.n_rho - 1.0)
    th = np.mod(np.arctan2(Y, X), 2.0 * math.pi)
    v = th / m.dphi
    i0 = np.minimum(np.floor(u).astype(np.int64), m.n_rho - 2)
    wu = u - i0
    j0 = np.floor(v).astype(np.int64)
    wv = v - j0
    j0 %= m.n_phi
    j1 = (j0 + 1) % m.n_phi
    return ((1 - wv) * ((1 - wu) * bL[j0, i0] + wu * bL[j0, i0 + 1])
            + wv * ((1 - wu) * bL[j1, i0] + wu * bL[j1, i0 + 1]))


def backproject_logpolar(s: np.ndarray, H: int, W: int) -> np.ndarray:
    """B s by the log-polar algorithm (Steps 1-4)."""
    n_angles, n_det = np.shape(s)
    m = mesh(H, W, n_angles, n_det)
    bL = convolve(to_logpolar(s, m), kernel(m), m)
    return to_cartesian(bL, m, H, W)


def logpolar_result(s: np.ndarray, H: int, W: int) -> np.ndarray:
    """[B s]_L on the mesh (Steps 1-3), shape (n_phi, n_rho)."""
    n_angles, n_det = np.shape(s)
    m = mesh(H, W, n_angles, n_det)
    return convolve(to_logpolar(s, m), kernel(m), m)
