"""FP64 oracle for the unrolled (differentiable) solver.  Test infrastructure.

K iterations of the primal-dual method (the iteration in ``pdhg``), each with its
own coefficients c_k = (lam_k, tau_k, sigma_k), theta fixed.  The output is
f^K.  Gradients of a scalar loss L(f^K) with respect to the data g and to every
c_k are obtained by plain reverse-mode differentiation of the iteration.

Forward, k = 0..K-1 (with f^{-1} = f^0 = g, p^0 = 0):
    fbar    = (1 + theta) f^k - theta f^{k-1}
    q       = p^k + sigma_k grad fbar
    p^{k+1} = projection of q onto the lam_k-ball (pointwise)
    d       = div p^{k+1}
    f^{k+1} = (f^k + tau_k (d + g)) / (1 + tau_k)

Reverse: carry a = dL/df^{k+1}, b = the part of dL/df^k already collected
from the extrapolation of iteration k+1, r = dL/dp^{k+1} from iteration k+1.
    alpha   = a / (1 + tau_k)
    gbar   += tau_k alpha;           taubar_k = sum alpha (d + g - f^{k+1})
    s       = r - grad(tau_k alpha)          (div is minus the adjoint of grad)
    t       = s                       where |q| <= lam_k
            = (lam_k/|q|)(s - n (n.s)) with n = q/|q|   elsewhere
    lambar_k = sum over the projected pixels of n.s
    sigmabar_k = sum t . grad fbar
    w       = -sigma_k div t                  (dL/dfbar)
    a <- alpha + b + (1 + theta) w;  b <- -theta w;  r <- t
and finally gbar += a + b because f^0 = f^{-1} = g.
The derivative of the projection at |q| = lam_k uses the identity branch.
"""
from __future__ import annotations

import numpy as np

from .pdhg import grad, div, project_ball, init_state, pdhg_iteration


def _forward_states(g, coeffs, theta):
    f, f_prev, p = init_state(g)
    fs = [f_prev, f]          # fs[k + 1] = f^k, k = -1..K
    ps = [p]                  # ps[k] = p^k
    for lam, tau, sigma in coeffs:
        f_new, p = pdhg_iteration(f, f_prev, p, g, lam, tau, sigma, theta)
        f_prev, f = f, f_new
        fs.append(f)
        ps.append(p)
    return fs, ps


def unrolled_forward(g, coeffs, theta=1.0):
    """f^K for one image g (any ndim) and coeffs of shape (K, 3)."""
    g = np.asarray(g, dtype=np.float64)
    coeffs = np.asarray(coeffs, dtype=np.float64).reshape(-1, 3)
    fs, _ = _forward_states(g, coeffs, theta)
    return fs[-1]


def unrolled_backward(g, coeffs, grad_f, theta=1.0):
    """Return (grad_g, grad_coeffs[K, 3]) for dL/df^K = grad_f."""
    g = np.asarray(g, dtype=np.float64)
    coeffs = np.asarray(coeffs, dtype=np.float64).reshape(-1, 3)
    K = coeffs.shape[0]
    fs, ps = _forward_states(g, coeffs, theta)
    a = np.asarray(grad_f, dtype=np.float64).copy()
    b = np.zeros_like(g)
    r = np.zeros((g.ndim,) + g.shape)
    gbar = np.zeros_like(g)
    cbar = np.zeros((K, 3))
    for k in range(K - 1, -1, -1):
        lam, tau, sigma = coeffs[k]
        fk, fkm1, pk, fn = fs[k + 1], fs[k], ps[k], fs[k + 2]
        fbar = fk + theta * (fk - fkm1)
        gfb = grad(fbar)
        q = pk + sigma * gfb
        p_new = project_ball(q, lam)
        d = div(p_new)
        alpha = a / (1.0 + tau)
        gbar += tau * alpha
        cbar[k, 1] = np.sum(alpha * (d + g - fn))
        s = r - grad(tau * alpha)
        nrm = np.sqrt(np.sum(q * q, axis=0))
        inside = nrm <= lam
        safe = np.where(inside, 1.0, nrm)
        n = q / safe[None]
        ns = np.sum(n * s, axis=0)
        t_out = (lam / safe)[None] * (s - n * ns[None])
        t = np.where(inside[None], s, t_out)
        cbar[k, 0] = np.sum(np.where(inside, 0.0, ns))
        cbar[k, 2] = np.sum(t * gfb)
        w = -sigma * div(t)
        a, b = alpha + b + (1.0 + theta) * w, -theta * w
        r = t
    gbar += a + b
    return gbar, cbar


def unrolled_forward_batch(gs, coeffs, theta=1.0):
    return np.stack([unrolled_forward(g, coeffs, theta) for g in gs])


def unrolled_backward_batch(gs, coeffs, grad_fs, theta=1.0):
    """Coefficients are shared by the batch: their gradients add up."""
    gg, cc = [], 0.0
    for g, gf in zip(gs, grad_fs):
        a, c = unrolled_backward(g, coeffs, gf, theta)
        gg.append(a)
        cc = cc + c
    return np.stack(gg), cc
