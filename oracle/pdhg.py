"""FP64 oracle: operators, one primal-dual iteration, energies, stopping.

Test infrastructure only (see the package docstring).  Plain NumPy in float64;
nothing here is blocked, fused or reordered.

Notation follows the paper's regularised problem (Section 6, eq. opt): ``f`` is
the image (the paper's feature function), ``g`` the data, ``lam`` the weight on
the regulariser.  With the identity as forward operator and the isotropic total
variation as regulariser the problem reads

    min_f  1/2 ||f - g||^2 + lam * TV(f),   TV(f) = sum_i |(grad f)_i|_2.

The factor 1/2 on the data term is a reading: the paper writes the data term
without it; with it, lam = 0.1 and tau = sigma = 1/sqrt(8) are the usual
settings for images with values in [0, 1].
"""
from __future__ import annotations

import math

import numpy as np


# --------------------------------------------------------------------------
# Operators.  grad and -div form an adjoint pair, the same relation the paper
# states for the Radon transform and the backprojection (Section 1, eq.
# adjoint): <grad f, p> = -<f, div p>.
# --------------------------------------------------------------------------

def grad(f: np.ndarray) -> np.ndarray:
    """Forward differences with Neumann boundary, grid spacing 1.

    Returns an array of shape (f.ndim, *f.shape).  Component c differentiates
    along array axis f.ndim - 1 - c (c = 0 is x, the last axis).  The
    difference at the last index of each axis is 0.
    """
    f = np.asarray(f, dtype=np.float64)
    nd = f.ndim
    out = np.zeros((nd,) + f.shape, dtype=np.float64)
    for c in range(nd):
        ax = nd - 1 - c
        n = f.shape[ax]
        if n < 2:
            continue
        lo = [slice(None)] * nd
        hi = [slice(None)] * nd
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        out[c][tuple(lo)] = f[tuple(hi)] - f[tuple(lo)]
    return out


def div(p: np.ndarray) -> np.ndarray:
    """Discrete divergence, defined as minus the adjoint of :func:`grad`.

    Along an axis of length n (index i), for the matching component p_c:
        i = 0:          p_c[0]
        0 < i < n - 1:  p_c[i] - p_c[i-1]
        i = n - 1:      -p_c[n-2]
    (for n = 1 the contribution is 0).
    """
    p = np.asarray(p, dtype=np.float64)
    nd = p.shape[0]
    shape = p.shape[1:]
    assert len(shape) == nd
    out = np.zeros(shape, dtype=np.float64)
    for c in range(nd):
        ax = nd - 1 - c
        n = shape[ax]
        if n < 2:
            continue
        pc = p[c]

        def sl(a, b):
            s = [slice(None)] * nd
            s[ax] = slice(a, b)
            return tuple(s)

        out[sl(0, 1)] += pc[sl(0, 1)]
        if n > 2:
            out[sl(1, n - 1)] += pc[sl(1, n - 1)] - pc[sl(0, n - 2)]
        out[sl(n - 1, n)] -= pc[sl(n - 2, n - 1)]
    return out


def step_bound(shape) -> float:
    """Largest eigenvalue of -div grad (the Neumann Laplacian), i.e. ||grad||^2.

    The Neumann Laplacian is diagonalised by the type-II DCT; along an axis of
    length n its eigenvalues are 4 sin^2(pi k / (2 n)), k = 0..n-1, and the
    multi-axis operator adds them.
    """
    return float(sum(4.0 * math.sin(math.pi * (n - 1) / (2.0 * n)) ** 2
                     for n in shape))


# --------------------------------------------------------------------------
# Proximal maps.
# --------------------------------------------------------------------------

def project_ball(q: np.ndarray, lam: float) -> np.ndarray:
    """Pointwise projection of the vector field q onto {|p_i|_2 <= lam}.

    This is the proximal map of the convex conjugate of lam * TV (for any
    step sigma).  Tie rule: |q_i| <= lam keeps q_i unchanged, so lam = 0
    gives p = 0.
    """
    q = np.asarray(q, dtype=np.float64)
    nrm = np.sqrt(np.sum(q * q, axis=0))
    inside = nrm <= lam
    safe = np.where(inside, 1.0, nrm)
    scale = np.where(inside, 1.0, lam / safe)
    return q * scale[None]


def prox_data(v: np.ndarray, g: np.ndarray, tau: float) -> np.ndarray:
    """Proximal map of tau * 1/2 ||. - g||^2: (v + tau g) / (1 + tau)."""
    return (v + tau * g) / (1.0 + tau)


# --------------------------------------------------------------------------
# One iteration (Chambolle-Pock Algorithm 1 with K = grad, K* = -div).
# --------------------------------------------------------------------------

def init_state(g: np.ndarray):
    """Initial state: f^0 = g, f^{-1} = f^0 (so the first extrapolation is g),
    p^0 = 0."""
    g = np.asarray(g, dtype=np.float64)
    return g.copy(), g.copy(), np.zeros((g.ndim,) + g.shape)


def pdhg_iteration(f, f_prev, p, g, lam, tau, sigma, theta=1.0):
    """One iteration k -> k+1.  Returns (f^{k+1}, p^{k+1}).

    1. extrapolation  fbar = f^k + theta (f^k - f^{k-1})
    2. dual ascent     q = p^k + sigma grad fbar
    3. dual prox       p^{k+1} = projection of q onto the lam-ball
    4. primal descent  v = f^k + tau div p^{k+1}
    5. data prox       f^{k+1} = (v + tau g) / (1 + tau)
    """
    fbar = f + theta * (f - f_prev)
    q = p + sigma * grad(fbar)
    p_new = project_ball(q, lam)
    v = f + tau * div(p_new)
    f_new = prox_data(v, g, tau)
    return f_new, p_new


def quadratic_iteration(f, f_prev, p, g, lam, tau, sigma, theta=1.0):
    """Same iteration for the quadratic regulariser (lam/2) ||grad f||^2.

    Only the dual prox changes: the conjugate is ||p||^2 / (2 lam), whose prox
    is q / (1 + sigma / lam).  The minimiser solves (I - lam div grad) f = g,
    the gradient-penalty analogue of the paper's normal equations (Section 6,
    eq. neq), and has a closed-form Fourier (cosine) filter solution like
    eq. quaseo.
    """
    fbar = f + theta * (f - f_prev)
    q = p + sigma * grad(fbar)
    p_new = q / (1.0 + sigma / lam)
    v = f + tau * div(p_new)
    f_new = prox_data(v, g, tau)
    return f_new, p_new


# --------------------------------------------------------------------------
# Energies and duality gap.
# --------------------------------------------------------------------------

def primal_energy(f, g, lam) -> float:
    """P(f) = 1/2 ||f - g||^2 + lam sum_i |(grad f)_i|_2."""
    gf = grad(f)
    return float(0.5 * np.sum((f - g) ** 2)
                 + lam * np.sum(np.sqrt(np.sum(gf * gf, axis=0))))


def dual_energy(p, g) -> float:
    """D(p) = -1/2 ||div p||^2 - <g, div p>, valid for |p_i| <= lam.

    It comes from eliminating f in the saddle form
    1/2 ||f - g||^2 - <f, div p>, whose minimiser is f = g + div p.
    """
    d = div(p)
    return float(-0.5 * np.sum(d * d) - np.sum(g * d))


def gap_density(f, p, g, lam) -> np.ndarray:
    """Per-pixel duality gap
        gamma_i = 1/2 (f_i - g_i - (div p)_i)^2 + lam |(grad f)_i| - <(grad f)_i, p_i>.

    sum_i gamma_i = P(f) - D(p) exactly, and each gamma_i >= 0 when
    |p_i| <= lam (Cauchy-Schwarz).
    """
    gf = grad(f)
    d = div(p)
    r = f - g - d
    return (0.5 * r * r + lam * np.sqrt(np.sum(gf * gf, axis=0))
            - np.sum(gf * p, axis=0))


def energy_gap(f, p, g, lam):
    """Return (P, D, gap) with gap = sum of the gap density."""
    P = primal_energy(f, g, lam)
    D = dual_energy(p, g)
    gap = float(np.sum(gap_density(f, p, g, lam)))
    return P, D, gap


# --------------------------------------------------------------------------
# Solvers.
# --------------------------------------------------------------------------

def solve(g, lam, tau=None, sigma=None, theta=1.0, max_iter=1000,
          check_every=10, gap_tol=-1.0, return_history=False):
    """Plain solve with the stopping rule.

    For k = 0, 1, ..., max_iter - 1: when check_every > 0 and
    k % check_every == 0, evaluate (P, D, gap) at the pair (f^k, p^k); if
    gap <= gap_tol * P the solve stops and returns f^k with iters = k,
    converged = True.  Otherwise iterate k -> k + 1.  If no check passes the
    result is f^{max_iter}, iters = max_iter, converged = False, with (P, D,
    gap) evaluated at that final pair.  gap_tol < 0 never stops.

    tau and sigma default to 1 / sqrt(4 ndim), for which
    tau sigma ||grad||^2 < 1 holds on every grid (step_bound < 4 ndim).
    """
    g = np.asarray(g, dtype=np.float64)
    if tau is None:
        tau = 1.0 / math.sqrt(4.0 * g.ndim)
    if sigma is None:
        sigma = 1.0 / math.sqrt(4.0 * g.ndim)
    f, f_prev, p = init_state(g)
    hist = []
    for k in range(max_iter):
        if check_every > 0 and k % check_every == 0:
            P, D, gp = energy_gap(f, p, g, lam)
            hist.append((k, P, D, gp))
            if gp <= gap_tol * P:
                out = dict(f=f, p=p, iters=k, converged=True, P=P, D=D, gap=gp)
                if return_history:
                    out["history"] = hist
                return out
        f_new, p = pdhg_iteration(f, f_prev, p, g, lam, tau, sigma, theta)
        f_prev, f = f, f_new
    P, D, gp = energy_gap(f, p, g, lam)
    out = dict(f=f, p=p, iters=max_iter, converged=False, P=P, D=D, gap=gp)
    if return_history:
        out["history"] = hist
    return out


def run_fixed(g, lam, tau, sigma, n_iter, theta=1.0):
    """n_iter iterations from the initial state; returns (f^n, f^{n-1}, p^n)."""
    f, f_prev, p = init_state(g)
    for _ in range(n_iter):
        f_new, p = pdhg_iteration(f, f_prev, p, g, lam, tau, sigma, theta)
        f_prev, f = f, f_new
    return f, f_prev, p
