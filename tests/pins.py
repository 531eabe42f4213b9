"""Independent reference solutions used to pin the FP64 oracle.

None of this shares code with the oracle: operators are built here as explicit
sparse matrices, and the 1D problem is solved by an exact finite algorithm.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from scipy.optimize import minimize


# --------------------------------------------------------------------------
# Explicit difference matrices.
# --------------------------------------------------------------------------

def diff_matrix(n: int) -> sp.csr_matrix:
    """n x n forward difference, last row zero (Neumann)."""
    if n < 2:
        return sp.csr_matrix((n, n))
    main = -np.ones(n)
    main[-1] = 0.0
    up = np.ones(n - 1)
    return sp.diags([main, up], [0, 1], shape=(n, n), format="csr")


def grad_matrix(shape) -> sp.csr_matrix:
    """Stacked gradient matrix; block c differentiates axis ndim-1-c (x first)
    on row-major flattened arrays."""
    nd = len(shape)
    blocks = []
    for c in range(nd):
        ax = nd - 1 - c
        mats = [sp.identity(n, format="csr") for n in shape]
        mats[ax] = diff_matrix(shape[ax])
        M = mats[0]
        for m in mats[1:]:
            M = sp.kron(M, m, format="csr")
        blocks.append(M)
    return sp.vstack(blocks, format="csr")


# --------------------------------------------------------------------------
# Exact 1D total-variation denoising by following the solution path in lam
# (the fused-lasso signal approximator path: adjacent groups fuse as lam
# grows and never split in 1D; Friedman, Hastie, Hoefling & Tibshirani 2007,
# Hoefling 2010).  Within a group G with outer neighbours L, R:
#   v_G(lam) = (sum_{i in G} g_i - lam (s_L + s_R)) / |G|,
#   s_L = sign(v_G - v_L), s_R = sign(v_G - v_R)  (0 if no neighbour).
# --------------------------------------------------------------------------

def tv1d_exact(g, lam: float) -> np.ndarray:
    g = np.asarray(g, dtype=np.float64)
    n = g.size
    # groups: [start, end (exclusive)]; their values at the current lam in vals
    groups, vals = [], []
    for i in range(n):
        if groups and g[i] == vals[-1]:
            groups[-1][1] += 1
        else:
            groups.append([i, i + 1])
            vals.append(float(g[i]))
    cur = 0.0
    while True:
        m = len(groups)
        slopes = []
        for j in range(m):
            sL = 0.0 if j == 0 else math.copysign(1.0, vals[j] - vals[j - 1])
            sR = 0.0 if j == m - 1 else math.copysign(1.0, vals[j] - vals[j + 1])
            slopes.append(-(sL + sR) / (groups[j][1] - groups[j][0]))
        # next fusion of two adjacent groups
        best, bj = None, -1
        for j in range(m - 1):
            ds = slopes[j] - slopes[j + 1]
            if ds == 0.0:
                continue
            t = (vals[j + 1] - vals[j]) / ds
            if t >= 0.0 and (best is None or t < best):
                best, bj = t, j
        if best is None or cur + best >= lam:
            out = np.empty(n)
            for G, v, s in zip(groups, vals, slopes):
                out[G[0]:G[1]] = v + (lam - cur) * s
            return out
        vals = [v + best * s for v, s in zip(vals, slopes)]
        cur += best
        A, B = groups[bj], groups[bj + 1]
        na, nb = A[1] - A[0], B[1] - B[0]
        vals[bj] = (na * vals[bj] + nb * vals[bj + 1]) / (na + nb)
        groups[bj] = [A[0], B[1]]
        del groups[bj + 1]
        del vals[bj + 1]


def tv1d_certificate(u, g, lam, tol=1e-10):
    """Optimality certificate for 1D TV denoising with forward differences.

    u - g + D^T z = 0 forces z_j = sum_{i<=j} (u_i - g_i); optimality needs
    |z_j| <= lam and z_j = lam sign(u_{j+1} - u_j) wherever u_{j+1} != u_j,
    plus sum(u - g) = 0.  Returns the largest violation.
    """
    u = np.asarray(u, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    z = np.cumsum(u - g)
    viol = abs(z[-1])
    z = z[:-1]
    du = np.diff(u)
    viol = max(viol, float(np.max(np.abs(z)) - lam) if z.size else 0.0)
    jump = np.abs(du) > tol
    if np.any(jump):
        viol = max(viol, float(np.max(np.abs(z[jump] - lam * np.sign(du[jump])))))
    return viol


# --------------------------------------------------------------------------
# Brute-force 2D TV on tiny images through the dual problem
#   min_p 1/2 ||g - G^T p||^2   s.t.  |p_i|_2 <= lam,   f = g - G^T p,
# with G the explicit gradient matrix (so -G^T is the divergence).
# --------------------------------------------------------------------------

def tv2d_bruteforce(g, lam):
    g = np.asarray(g, dtype=np.float64)
    shape = g.shape
    N = g.size
    nd = g.ndim
    G = grad_matrix(shape).toarray()
    gv = g.ravel()

    def obj(pv):
        r = gv - G.T @ pv
        return 0.5 * r @ r

    def jac(pv):
        r = gv - G.T @ pv
        return -(G @ r)

    def cons(pv):
        P = pv.reshape(nd, N)
        return lam * lam - np.sum(P * P, axis=0)

    def cons_jac(pv):
        P = pv.reshape(nd, N)
        J = np.zeros((N, nd * N))
        for c in range(nd):
            J[np.arange(N), c * N + np.arange(N)] = -2.0 * P[c]
        return J

    res = minimize(obj, np.zeros(nd * N), jac=jac, method="SLSQP",
                   constraints=[dict(type="ineq", fun=cons, jac=cons_jac)],
                   options=dict(ftol=1e-16, maxiter=2000))
    f = (gv - G.T @ res.x).reshape(shape)
    return f, res


# --------------------------------------------------------------------------
# Reference solver of the tomographic TV problem
#   min_f 1/2 ||A f - g||^2 + lam sum_i |(G f)_i|_2
# by ADMM on the split z = G f with exact dense f-solves (Boyd et al. 2011,
# Section 6.4.1): a different algorithm from the primal-dual iteration, with
# A given as a dense matrix and G the explicit gradient matrix above.
# --------------------------------------------------------------------------

def tomo_tv_admm(A, g, lam, shape, rho=10.0, iters=20000):
    N = int(np.prod(shape))
    G = grad_matrix(shape).toarray()
    Minv = np.linalg.inv(A.T @ A + rho * G.T @ G)
    Atg = A.T @ np.asarray(g, dtype=np.float64).ravel()
    z = np.zeros(2 * N)
    u = np.zeros(2 * N)
    f = np.zeros(N)
    for _ in range(iters):
        f = Minv @ (Atg + rho * G.T @ (z - u))
        v = (G @ f + u).reshape(2, N)
        nv = np.sqrt(np.sum(v * v, axis=0))
        shrink = np.maximum(0.0, 1.0 - (lam / rho) / np.maximum(nv, 1e-300))
        z = (v * shrink).ravel()
        u = u + G @ f - z
    return f.reshape(shape)
