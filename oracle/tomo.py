"""FP64 oracle for the tomographic data term (test infrastructure only).

Problem: the paper's regularised reconstruction (Section 6, eq. opt) with its
Radon transform as forward operator,

    minimise_f  1/2 ||A f - g||^2 + lam * TV(f)          (reg = "tv")
    minimise_f  1/2 ||A f - g||^2 + lam/2 * ||f||^2      (reg = "tikhonov")

where the Tikhonov case is half of eq. opt, so that its optimality condition is
the paper's normal equation (Section 6, eq. neq2) (A^T A + lam I) f = A^T g.

Discretisation (pixel units, detector spacing 1):
  * image f of shape (H, W); pixel (a, b) has centre
        X_ab = (b + 1/2 - W/2,  a + 1/2 - H/2)
    relative to the rotation centre (x along columns, y along rows);
  * angles theta_k = k pi / n_angles, k = 0 .. n_angles-1 (the angle mesh of
    the paper's table of symbols, Section 5), xi_k = (cos theta_k, sin theta_k)
    as in Section 1 eq. L;
  * detector bins t_i = i + 1/2 - n_det / 2, i = 0 .. n_det-1.

Projection, the discrete Radon transform (Section 1 eq. P_theta, with the
line's delta function replaced by the unit hat Lambda(s) = max(0, 1 - |s|)):
    (A f)[k, i] = sum_ab f[a, b] Lambda(X_ab . xi_k - t_i).
Backprojection, its exact transpose: linear interpolation of each projection
at X_ab . xi_k, summed over the angles (Section 2 eq. bp_app without the factor
dtheta; the sinogram counts as zero beyond the detector's ends):
    (A^T s)[a, b] = sum_k interp(s[k, :], X_ab . xi_k).
The pair satisfies the discrete form of Section 1 eq. adjoint,
<A f, s> = <f, A^T s>.

Sinograms are arrays of shape (n_angles, n_det): angle-major, t fastest.

Iteration (Chambolle & Pock 2011, Algorithm 1, theta = 1, with the operator
(A, grad) and one dual step size per block, sigma_r for the sinogram dual r and
sigma_p for the gradient dual p):
    fbar    = f^k + theta (f^k - f^{k-1})
    r^{k+1} = (r^k + sigma_r (A fbar - g)) / (1 + sigma_r)
    p^{k+1} = P_lam(p^k + sigma_p grad fbar)                       (tv)
    f^{k+1} = f^k - tau A^T r^{k+1} + tau div p^{k+1}               (tv)
    f^{k+1} = (f^k - tau A^T r^{k+1}) / (1 + tau lam)               (tikhonov)
from f^0 = f^{-1} = 0 (or a given f^0), r^0 = 0, p^0 = 0.  Convergence needs
tau (sigma_r ||A||^2 + sigma_p ||grad||^2) <= 1 (tv) or tau sigma_r ||A||^2
<= 1 (tikhonov); ||A||^2 comes from :func:`opnorm_sq`.

Plain NumPy in float64; nothing is blocked, fused or reordered.
"""
from __future__ import annotations

import math

import numpy as np

from .pdhg import div, grad, project_ball

REGS = ("tv", "tikhonov")


# --------------------------------------------------------------------------
# Geometry.
# --------------------------------------------------------------------------

def angles(n_angles: int) -> np.ndarray:
    """theta_k = k pi / n_angles (Section 5, table of symbols)."""
    return np.arange(n_angles, dtype=np.float64) * (math.pi / n_angles)


def pixel_centres(H: int, W: int):
    """(x, y) of every pixel centre, each of shape (H, W)."""
    x = np.arange(W, dtype=np.float64) + 0.5 - W / 2.0
    y = np.arange(H, dtype=np.float64) + 0.5 - H / 2.0
    return np.broadcast_to(x[None, :], (H, W)), np.broadcast_to(y[:, None], (H, W))


def detector(n_det: int) -> np.ndarray:
    """t_i = i + 1/2 - n_det / 2."""
    return np.arange(n_det, dtype=np.float64) + 0.5 - n_det / 2.0


# --------------------------------------------------------------------------
# The operator pair.  project() scatters every pixel onto the two bins its
# hat overlaps; backproject() gathers by linear interpolation.  They are
# written independently, so their adjointness is a check, not a tautology.
# --------------------------------------------------------------------------

def project(f: np.ndarray, n_angles: int, n_det: int) -> np.ndarray:
    """A f: shape (n_angles, n_det)."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    x, y = pixel_centres(H, W)
    t0 = 0.5 - n_det / 2.0
    out = np.zeros((n_angles, n_det), dtype=np.float64)
    fv = f.ravel()
    for k, th in enumerate(angles(n_angles)):
        u = (x * math.cos(th) + y * math.sin(th)).ravel()
        v = u - t0                      # position in bin units: bin i at v = i
        i0 = np.floor(v).astype(np.int64)
        w = v - i0                      # weight of bin i0 + 1
        for idx, wt in ((i0, 1.0 - w), (i0 + 1, w)):
            ok = (idx >= 0) & (idx < n_det)
            np.add.at(out[k], idx[ok], fv[ok] * wt[ok])
    return out


def backproject(s: np.ndarray, H: int, W: int) -> np.ndarray:
    """A^T s: shape (H, W)."""
    s = np.asarray(s, dtype=np.float64)
    n_angles, n_det = s.shape
    x, y = pixel_centres(H, W)
    t0 = 0.5 - n_det / 2.0
    out = np.zeros((H, W), dtype=np.float64)
    for k, th in enumerate(angles(n_angles)):
        ext = np.concatenate(([0.0], s[k], [0.0]))   # ext[i + 1] = s[k, i]
        v = x * math.cos(th) + y * math.sin(th) - t0
        i0 = np.floor(v).astype(np.int64)
        w = v - i0
        lo = np.clip(i0, -1, n_det) + 1
        hi = np.clip(i0 + 1, -1, n_det) + 1
        out += (1.0 - w) * ext[lo] + w * ext[hi]
    return out


def opnorm_sq(H: int, W: int, n_angles: int, n_det: int, iters: int = 50):
    """Power iteration for ||A||^2 = largest eigenvalue of A^T A, from the
    all-ones image.  Returns the Rayleigh quotient after ``iters`` steps."""
    v = np.ones((H, W), dtype=np.float64)
    v /= np.linalg.norm(v)
    est = 0.0
    for _ in range(iters):
        w = backproject(project(v, n_angles, n_det), H, W)
        est = float(np.sum(v * w))
        nrm = np.linalg.norm(w)
        if nrm == 0.0:
            return 0.0
        v = w / nrm
    return est


# --------------------------------------------------------------------------
# Energy and iteration.
# --------------------------------------------------------------------------

def energy(f: np.ndarray, g: np.ndarray, lam: float, reg: str = "tv"):
    """(data term, regulariser term, total) of the problem above."""
    f = np.asarray(f, dtype=np.float64)
    res = project(f, *np.shape(g)) - np.asarray(g, dtype=np.float64)
    data = 0.5 * float(np.sum(res * res))
    if reg == "tv":
        gr = grad(f)
        regv = lam * float(np.sum(np.sqrt(np.sum(gr * gr, axis=0))))
    elif reg == "tikhonov":
        regv = 0.5 * lam * float(np.sum(f * f))
    else:
        raise ValueError(reg)
    return data, regv, data + regv


def init_state(H: int, W: int, n_angles: int, n_det: int, f0=None):
    f = np.zeros((H, W)) if f0 is None else np.array(f0, dtype=np.float64)
    return dict(f=f, f_prev=f.copy(), r=np.zeros((n_angles, n_det)),
                p=np.zeros((2, H, W)))


def iteration(state, g, lam, tau, sigma_r, sigma_p, reg="tv", theta=1.0):
    """One iteration; returns the new state (the input is not modified)."""
    f, fp, r, p = state["f"], state["f_prev"], state["r"], state["p"]
    H, W = f.shape
    fbar = f + theta * (f - fp)
    r_new = (r + sigma_r * (project(fbar, *r.shape) - g)) / (1.0 + sigma_r)
    bp = backproject(r_new, H, W)
    if reg == "tv":
        p_new = project_ball(p + sigma_p * grad(fbar), lam)
        f_new = f - tau * bp + tau * div(p_new)
    elif reg == "tikhonov":
        p_new = p
        f_new = (f - tau * bp) / (1.0 + tau * lam)
    else:
        raise ValueError(reg)
    return dict(f=f_new, f_prev=f, r=r_new, p=p_new)


def run(g, H, W, lam, tau, sigma_r, sigma_p, n_iter, reg="tv", f0=None,
        theta=1.0):
    """``n_iter`` iterations from the initial state; returns the state."""
    g = np.asarray(g, dtype=np.float64)
    st = init_state(H, W, g.shape[0], g.shape[1], f0)
    for _ in range(n_iter):
        st = iteration(st, g, lam, tau, sigma_r, sigma_p, reg, theta)
    return st


# --------------------------------------------------------------------------
# Single entries, for sampled checks of large problems: the definitions of
# the two operators evaluated at chosen outputs only.
# --------------------------------------------------------------------------

def project_at(f: np.ndarray, n_angles: int, n_det: int, ks, iis) -> np.ndarray:
    """(A f)[k, i] for the pairs (ks[j], iis[j])."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    x, y = pixel_centres(H, W)
    th = angles(n_angles)
    t = detector(n_det)
    out = np.empty(len(ks), dtype=np.float64)
    for j, (k, i) in enumerate(zip(ks, iis)):
        u = x * math.cos(th[k]) + y * math.sin(th[k])
        out[j] = float(np.sum(f * np.maximum(0.0, 1.0 - np.abs(u - t[i]))))
    return out


def backproject_at(s: np.ndarray, H: int, W: int, rows, cols) -> np.ndarray:
    """(A^T s)[a, b] for the pixels (rows[j], cols[j])."""
    s = np.asarray(s, dtype=np.float64)
    n_angles, n_det = s.shape
    th = angles(n_angles)
    t = detector(n_det)
    out = np.empty(len(rows), dtype=np.float64)
    for j, (a, b) in enumerate(zip(rows, cols)):
        x = b + 0.5 - W / 2.0
        y = a + 0.5 - H / 2.0
        u = x * np.cos(th) + y * np.sin(th)                 # one per angle
        w = np.maximum(0.0, 1.0 - np.abs(u[:, None] - t[None, :]))
        out[j] = float(np.sum(w * s))
    return out


# --------------------------------------------------------------------------
# Regularised filtered backprojection (Section 6, eq. reg_sol and the filter
# after it): f_lam = B F_lam g, each projection filtered in t by the
# frequency response |nu| / (1 + lam |nu|) and backprojected with the factor
# dtheta = pi / n_angles (B = dtheta A^T).  nu is in cycles per pixel (for
# lam = 0 this is the ramp filter of the standard inversion formula); lam is
# in pixels.  The filter acts on each projection zero-padded to
# fbp_length(n_det), the smallest power of two >= 2 n_det, so that the
# circular convolution equals the linear one on the detector.
# --------------------------------------------------------------------------

def fbp_length(n_det: int) -> int:
    L = 1
    while L < 2 * n_det:
        L *= 2
    return L


def fbp_response(n_det: int, lam: float) -> np.ndarray:
    """The filter's DFT samples H[m] at nu_m = fftfreq(L)[m]."""
    nu = np.abs(np.fft.fftfreq(fbp_length(n_det)))
    return nu / (1.0 + lam * nu)


def fbp_filter(s: np.ndarray, lam: float) -> np.ndarray:
    """F_lam applied to every projection (row) of s."""
    s = np.asarray(s, dtype=np.float64)
    n_angles, n_det = s.shape
    L = fbp_length(n_det)
    spec = np.fft.fft(s, n=L, axis=1) * fbp_response(n_det, lam)[None, :]
    return np.real(np.fft.ifft(spec, axis=1))[:, :n_det]


def fbp(s: np.ndarray, H: int, W: int, lam: float) -> np.ndarray:
    """f_lam = (pi / n_angles) A^T F_lam s."""
    n_angles = np.shape(s)[0]
    return (math.pi / n_angles) * backproject(fbp_filter(s, lam), H, W)


# --------------------------------------------------------------------------
# Backprojection slice theorem (BST, Section 3, eq. bst, and the algorithm of
# Section 5): the 2D Fourier transform of B g on the line through the origin
# at angle theta equals the 1D Fourier transform of the projection at theta,
# divided by |nu|.  In the cycles convention (transforms with exp(-2 pi i nu x))
# F[B g](nu xi_theta) = G(nu, theta) / |nu| exactly, with B = dtheta A^T for
# sampled data.  Steps, on a detector of spacing 1:
#   1. G_k(nu_j) = sum_i g_k[i] exp(-2 pi i nu_j t_i), nu_j = j / M on the
#      zero-padded grid of length M = bst_lengths()[0];
#   2. times K(nu) = 1 / |nu|, and 1 / dnu = M at nu = 0 (the origin rule of
#      the kernel K^sigma in Section 5);
#   3. bilinear interpolation of these polar samples (theta_k, nu_j) at the
#      Cartesian frequencies (p / Q, q / Q) of a Q x Q grid, zero beyond
#      |nu| = 1/2; theta in [0, pi) with signed nu covers the plane;
#   4. 2D inverse DFT, evaluated at the pixel centres.
# No window is applied: with full projections (t over the whole detector)
# the data already vanish at both ends.
# --------------------------------------------------------------------------

def bst_lengths(H: int, W: int, n_det: int):
    """(M, Q): 1D transform length (power of two >= 2 n_det) and the side of
    the Cartesian frequency grid (power of two >= 2 max(H, W))."""
    M = fbp_length(n_det)
    Q = 1
    while Q < 2 * max(H, W):
        Q *= 2
    return M, Q


def bst_spectra(s: np.ndarray, M: int, lam: float | None = None) -> np.ndarray:
    """Steps 1-2: K(nu_j) G_k(nu_j) for j = -M/2 .. M/2-1 (row k, column
    j + M/2), complex128.  K = 1/|nu| with the origin rule, or with lam the
    kernel 1/(1 + lam |nu|) of the regularised Fourier slice theorem
    (Section 6, eq. reg_fst): the ramp of the filter F_lam cancels 1/|nu|, so
    the BST of these spectra is B F_lam g, the regularised FBP (eq. reg_sol)."""
    s = np.asarray(s, dtype=np.float64)
    n_angles, n_det = s.shape
    t = detector(n_det)
    nu = (np.arange(M) - M // 2) / M
    G = s @ np.exp(-2j * np.pi * np.outer(t, nu))          # plain DFT
    if lam is None:
        K = np.where(nu == 0.0, float(M), 1.0 / np.where(nu == 0.0, 1.0, np.abs(nu)))
    else:
        K = 1.0 / (1.0 + lam * np.abs(nu))
    return G * K[None, :]


def bst_cartesian(P: np.ndarray, Q: int) -> np.ndarray:
    """Step 3: the Q x Q grid of frequencies (u_p, v_q) = (p, q) / Q for
    p, q = -Q/2 .. Q/2-1 (array index [q + Q/2, p + Q/2]), bilinear in
    (theta, nu) from the polar samples P."""
    n_angles, M = P.shape
    f = (np.arange(Q) - Q // 2) / Q
    u, v = np.meshgrid(f, f)                  # u along columns (x), v along rows (y)
    rho = np.hypot(u, v)
    phi = np.arctan2(v, u)                     # (-pi, pi]
    neg = phi < 0.0
    theta = np.where(neg, phi + np.pi, phi)
    nu = np.where(neg, -rho, rho)
    top = theta >= np.pi                       # phi = pi: theta pi == 0 with -nu
    theta = np.where(top, theta - np.pi, theta)
    nu = np.where(top, -nu, nu)
    a = theta / (np.pi / n_angles)             # angle index, in [0, n_angles)
    k0 = np.floor(a).astype(np.int64)
    wa = a - k0
    k1 = k0 + 1                                # k1 == n_angles: theta = pi, nu -> -nu
    flip = k1 >= n_angles
    k1 = np.where(flip, 0, k1)

    def radial(k, nuv):
        x = nuv * M + M // 2                   # radial index
        j0 = np.floor(x).astype(np.int64)
        wr = x - j0
        ok0 = (j0 >= 0) & (j0 < M)
        ok1 = (j0 + 1 >= 0) & (j0 + 1 < M)
        p0 = np.where(ok0, P[k, np.clip(j0, 0, M - 1)], 0.0)
        p1 = np.where(ok1, P[k, np.clip(j0 + 1, 0, M - 1)], 0.0)
        return (1.0 - wr) * p0 + wr * p1

    F = (1.0 - wa) * radial(k0, nu) + wa * radial(k1, np.where(flip, -nu, nu))
    return np.where(rho <= 0.5, F, 0.0)


def bst(s: np.ndarray, H: int, W: int, lam: float | None = None) -> np.ndarray:
    """B s (= dtheta A^T s up to the method's interpolation) by the BST; with
    lam the regularised FBP B F_lam s through the same steps (fbp_bst)."""
    s = np.asarray(s, dtype=np.float64)
    M, Q = bst_lengths(H, W, s.shape[1])
    F = bst_cartesian(bst_spectra(s, M, lam), Q)
    f = (np.arange(Q) - Q // 2) / Q
    x = np.arange(W) + 0.5 - W / 2.0
    y = np.arange(H) + 0.5 - H / 2.0
    # b(x, y) = sum_{p,q} F[q, p] exp(2 pi i (u_p x + v_q y)) / Q^2
    Ex = np.exp(2j * np.pi * np.outer(f, x))   # [p, x]
    Ey = np.exp(2j * np.pi * np.outer(y, f))   # [y, q]
    return np.real(Ey @ F @ Ex) / (Q * Q)


def bst_at(s: np.ndarray, H: int, W: int, rows, cols, lam: float | None = None) -> np.ndarray:
    """bst(s, H, W, lam)[rows[j], cols[j]]: the same grid F, with the inverse
    DFT evaluated at the listed pixels only (for images too large for the
    dense transform matrices of bst())."""
    s = np.asarray(s, dtype=np.float64)
    M, Q = bst_lengths(H, W, s.shape[1])
    F = bst_cartesian(bst_spectra(s, M, lam), Q)
    f = (np.arange(Q) - Q // 2) / Q
    x = np.asarray(cols, dtype=np.float64) + 0.5 - W / 2.0
    y = np.asarray(rows, dtype=np.float64) + 0.5 - H / 2.0
    Fx = F @ np.exp(2j * np.pi * np.outer(f, x))            # [q, j]: sum over p
    Ey = np.exp(2j * np.pi * np.outer(y, f))                # [j, q]
    return np.real(np.sum(Ey * Fx.T, axis=1)) / (Q * Q)


def fbp_bst(s: np.ndarray, H: int, W: int, lam: float) -> np.ndarray:
    """The regularised FBP f_lam = B F_lam s (Section 6, eq. reg_sol) with B
    computed by the BST: the spectra times 1/(1 + lam |nu|) (eq. reg_fst),
    gridded and inverted as in bst().  Equals fbp() up to the interpolation
    of the polar samples."""
    if not lam >= 0.0:
        raise ValueError("lam must be >= 0")
    return bst(s, H, W, float(lam))
