"""Pins of the oracle's unrolled solver and its reverse-mode adjoint (CPU)."""
import math

import numpy as np

import oracle
from oracle.unrolled import unrolled_backward_batch, unrolled_forward_batch
from scenes import scene2d, scene3d


def _mse_loss(fK, c):
    return float(np.mean((fK - c) ** 2))


def _crop_pair(seed=4000, n=16):
    clean, noisy = scene2d(512, 512, 20, 0.1, seed)
    return clean[:n, :n].copy(), noisy.astype(np.float32).astype(np.float64)[:n, :n].copy()


def _coeffs(K, lam=0.1, ndim=2, rng=None):
    s = 1.0 / math.sqrt(4.0 * ndim)
    c = np.tile([lam, s, s], (K, 1)).astype(np.float64)
    if rng is not None:
        c *= rng.uniform(0.8, 1.2, size=c.shape)
    return c


def test_forward_equals_plain_iteration():
    _, g = _crop_pair()
    K = 20
    c = _coeffs(K)
    fK = oracle.unrolled_forward(g, c)
    f, _, _ = oracle.run_fixed(g, 0.1, c[0, 1], c[0, 2], K)
    assert np.array_equal(fK, f)


def test_finite_differences_16x16():
    """Central differences of the MSE to the clean crop, over all 3K
    coefficients and 32 random data pixels, against the adjoint.  The step is
    1e-7: with 1e-6 the difference for lam_14 straddles a pixel where the
    projection switches branch (|q| = lam) and is off by 2e-3."""
    clean, g = _crop_pair()
    K = 20
    rng = np.random.default_rng(40)
    c = _coeffs(K, rng=rng)
    fK = oracle.unrolled_forward(g, c)
    grad_f = 2.0 * (fK - clean) / fK.size
    gg, gc = oracle.unrolled_backward(g, c, grad_f)
    h = 1e-7
    num_c = np.zeros_like(c)
    for k in range(K):
        for j in range(3):
            cp, cm = c.copy(), c.copy()
            cp[k, j] += h
            cm[k, j] -= h
            num_c[k, j] = (_mse_loss(oracle.unrolled_forward(g, cp), clean)
                           - _mse_loss(oracle.unrolled_forward(g, cm), clean)) / (2 * h)
    err_c = np.linalg.norm(num_c - gc) / np.linalg.norm(num_c)
    assert err_c < 1e-6, err_c
    idx = rng.choice(g.size, size=32, replace=False)
    num_g, ana_g = [], []
    for i in idx:
        gp, gm = g.copy().ravel(), g.copy().ravel()
        gp[i] += h
        gm[i] -= h
        num_g.append((_mse_loss(oracle.unrolled_forward(gp.reshape(g.shape), c), clean)
                      - _mse_loss(oracle.unrolled_forward(gm.reshape(g.shape), c), clean))
                     / (2 * h))
        ana_g.append(gg.ravel()[i])
    num_g, ana_g = np.array(num_g), np.array(ana_g)
    assert np.linalg.norm(num_g - ana_g) / np.linalg.norm(num_g) < 1e-6


def test_finite_differences_3d():
    clean, noisy = scene3d(10, 9, 8, 5, 0.1, 50)
    g = noisy
    K = 6
    rng = np.random.default_rng(41)
    c = _coeffs(K, ndim=3, rng=rng)
    fK = oracle.unrolled_forward(g, c)
    grad_f = 2.0 * (fK - clean) / fK.size
    _, gc = oracle.unrolled_backward(g, c, grad_f)
    h = 1e-6
    num = np.zeros_like(c)
    for k in range(K):
        for j in range(3):
            cp, cm = c.copy(), c.copy()
            cp[k, j] += h
            cm[k, j] -= h
            num[k, j] = (_mse_loss(oracle.unrolled_forward(g, cp), clean)
                         - _mse_loss(oracle.unrolled_forward(g, cm), clean)) / (2 * h)
    assert np.linalg.norm(num - gc) / np.linalg.norm(num) < 1e-6


def test_one_iteration_closed_form():
    """K = 1 with the projection inactive everywhere (sigma |grad g| <= lam):
    f^1 = g + s L g with s = tau sigma / (1 + tau) and L = div grad, so for
    L(f) = 1/2 |f^1 - c|^2 and e = f^1 - c:
        dL/dg = e + s L e,  dL/dlam = 0,
        dL/dsigma = tau/(1+tau) <e, L g>,  dL/dtau = sigma/(1+tau)^2 <e, L g>.
    """
    rng = np.random.default_rng(42)
    g = rng.normal(scale=0.05, size=(7, 9))
    c_img = rng.normal(size=(7, 9))
    lam, tau, sigma = 10.0, 0.3, 0.4
    coeffs = np.array([[lam, tau, sigma]])
    Lg = oracle.div(oracle.grad(g))
    s = tau * sigma / (1 + tau)
    f1 = oracle.unrolled_forward(g, coeffs)
    np.testing.assert_allclose(f1, g + s * Lg, atol=1e-14)
    e = f1 - c_img
    gg, gc = oracle.unrolled_backward(g, coeffs, e)
    np.testing.assert_allclose(gg, e + s * oracle.div(oracle.grad(e)), atol=1e-13)
    assert gc[0, 0] == 0.0
    assert math.isclose(gc[0, 2], tau / (1 + tau) * np.sum(e * Lg), rel_tol=1e-12)
    assert math.isclose(gc[0, 1], sigma / (1 + tau) ** 2 * np.sum(e * Lg),
                        rel_tol=1e-12)


def test_one_iteration_projection_active_lambda_gradient():
    """K = 1, all pixels projected (lam tiny): p^1 = lam n with n = grad g /
    |grad g|, so dL/dlam = <e, tau/(1+tau) div n>."""
    rng = np.random.default_rng(43)
    g = rng.normal(size=(6, 8))
    c_img = rng.normal(size=(6, 8))
    lam, tau, sigma = 1e-3, 0.3, 0.4
    coeffs = np.array([[lam, tau, sigma]])
    gr = oracle.grad(g)
    nrm = np.sqrt(np.sum(gr * gr, axis=0))
    # Neumann edges have a zero gradient component; the corner pixel has no
    # gradient at all and stays at p = 0 (identity branch).
    n = np.where(nrm > 0, gr / np.where(nrm > 0, nrm, 1.0), 0.0)
    f1 = oracle.unrolled_forward(g, coeffs)
    e = f1 - c_img
    _, gc = oracle.unrolled_backward(g, coeffs, e)
    expect = tau / (1 + tau) * np.sum(e * oracle.div(n))
    assert math.isclose(gc[0, 0], expect, rel_tol=1e-10)
    assert abs(gc[0, 2]) < 1e-12 * abs(expect) + 1e-15  # sigma drops out


def test_batch_shares_coefficients():
    rng = np.random.default_rng(44)
    gs = rng.normal(size=(3, 6, 7))
    K = 4
    c = _coeffs(K, rng=rng)
    fs = unrolled_forward_batch(gs, c)
    gfs = rng.normal(size=fs.shape)
    gg, gc = unrolled_backward_batch(gs, c, gfs)
    tot = sum(oracle.unrolled_backward(gs[i], c, gfs[i])[1] for i in range(3))
    np.testing.assert_allclose(gc, tot, atol=1e-13)
    assert gg.shape == gs.shape
