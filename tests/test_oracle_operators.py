"""Pins of the oracle's operators and proximal maps (CPU only).

Each test checks the oracle against something it does not compute itself:
explicit sparse matrices, the cosine-transform spectrum of the Neumann
Laplacian, dense eigenvalues, or a second formula for the same proximal map.
"""
import math

import numpy as np
import pytest
import scipy.fft as sfft

import oracle
import pins

SHAPES_2D = [(1, 1), (1, 7), (2, 2), (5, 3), (37, 53), (16, 16)]
SHAPES_3D = [(1, 4, 5), (3, 4, 5), (6, 2, 7), (8, 8, 8)]


@pytest.mark.parametrize("shape", SHAPES_2D + SHAPES_3D)
def test_adjointness(shape):
    """<grad f, p> = -<f, div p> (the adjoint-pair relation, cf. the paper's
    eq. adjoint for R and B), to round-off."""
    rng = np.random.default_rng(1)
    f = rng.normal(size=shape)
    p = rng.normal(size=(len(shape),) + shape)
    lhs = np.sum(oracle.grad(f) * p)
    rhs = -np.sum(f * oracle.div(p))
    scale = np.linalg.norm(oracle.grad(f)) * np.linalg.norm(p) + 1e-300
    assert abs(lhs - rhs) <= 1e-13 * scale


@pytest.mark.parametrize("shape", SHAPES_2D + SHAPES_3D)
def test_grad_matches_explicit_matrix(shape):
    rng = np.random.default_rng(2)
    f = rng.normal(size=shape)
    G = pins.grad_matrix(shape)
    ref = (G @ f.ravel()).reshape((len(shape),) + shape)
    assert np.array_equal(oracle.grad(f), ref)
    p = rng.normal(size=(len(shape),) + shape)
    ref_div = -(G.T @ p.ravel()).reshape(shape)
    np.testing.assert_allclose(oracle.div(p), ref_div, rtol=0, atol=1e-13)


def test_component_convention():
    """p[0] differentiates along x (last axis), p[1] along y, p[2] along z."""
    z, y, x = np.meshgrid(np.arange(3.0), np.arange(4.0), np.arange(5.0),
                          indexing="ij")
    gx = oracle.grad(x)
    assert np.all(gx[0][:, :, :-1] == 1) and np.all(gx[0][:, :, -1] == 0)
    assert np.all(gx[1] == 0) and np.all(gx[2] == 0)
    gy = oracle.grad(y)
    assert np.all(gy[1][:, :-1, :] == 1) and np.all(gy[1][:, -1, :] == 0)
    gz = oracle.grad(z)
    assert np.all(gz[2][:-1] == 1) and np.all(gz[2][-1] == 0)


@pytest.mark.parametrize("shape", [(9, 14), (32, 32), (5, 6, 7)])
def test_laplacian_cosine_spectrum(shape):
    """-div grad is the Neumann Laplacian: diagonal in the type-II DCT with
    eigenvalues sum_axes 4 sin^2(pi k / 2n)."""
    rng = np.random.default_rng(3)
    f = rng.normal(size=shape)
    lap = -oracle.div(oracle.grad(f))
    mu = np.zeros(shape)
    for ax, n in enumerate(shape):
        k = np.arange(n)
        s = [1] * len(shape)
        s[ax] = n
        mu = mu + (4.0 * np.sin(np.pi * k / (2.0 * n)) ** 2).reshape(s)
    ref = sfft.idctn(mu * sfft.dctn(f, type=2, norm="ortho"), type=2,
                     norm="ortho")
    np.testing.assert_allclose(lap, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("shape", [(2, 2), (3, 5), (8, 8), (4, 3, 5)])
def test_step_bound_dense_eigs(shape):
    G = pins.grad_matrix(shape).toarray()
    lmax = np.linalg.eigvalsh(G.T @ G).max()
    assert abs(oracle.step_bound(shape) - lmax) <= 1e-12 * max(lmax, 1)
    assert oracle.step_bound(shape) < 4 * len(shape)


def test_step_bound_power_iteration():
    shape = (64, 48)
    rng = np.random.default_rng(4)
    v = rng.normal(size=shape)
    for _ in range(3000):
        v = -oracle.div(oracle.grad(v))
        v /= np.linalg.norm(v)
    lam = np.sum(v * -oracle.div(oracle.grad(v)))
    assert abs(lam - oracle.step_bound(shape)) < 1e-4


def test_divergence_sums_to_zero():
    rng = np.random.default_rng(5)
    for shape in SHAPES_2D + SHAPES_3D:
        p = rng.normal(size=(len(shape),) + shape)
        assert abs(np.sum(oracle.div(p))) < 1e-12 * p.size


def _soft_vec(v, t):
    n = np.sqrt(np.sum(v * v, axis=0))
    scale = np.maximum(0.0, 1.0 - t / np.maximum(n, 1e-300))
    return v * scale[None]


@pytest.mark.parametrize("lam,sigma", [(0.1, 0.35), (1.0, 1.0), (0.0, 0.5)])
def test_projection_moreau(lam, sigma):
    """Moreau: q = prox_{sigma F*}(q) + sigma prox_{F/sigma}(q / sigma) for
    F = lam |.|_2 per pixel; prox_{F/sigma} is vector soft-thresholding."""
    rng = np.random.default_rng(6)
    q = rng.normal(scale=0.3, size=(2, 17, 19))
    p = oracle.project_ball(q, lam)
    np.testing.assert_allclose(p + sigma * _soft_vec(q / sigma, lam / sigma), q,
                               rtol=0, atol=1e-14)
    assert np.all(np.sqrt(np.sum(p * p, axis=0)) <= lam * (1 + 1e-15))


def test_projection_is_nearest_point():
    rng = np.random.default_rng(7)
    lam = 0.4
    q = rng.normal(size=(2, 200))
    p = oracle.project_ball(q, lam)
    d_p = np.sqrt(np.sum((q - p) ** 2, axis=0))
    for _ in range(200):
        ang = rng.uniform(0, 2 * np.pi, size=200)
        rad = lam * np.sqrt(rng.uniform(0, 1, size=200))
        z = np.stack([rad * np.cos(ang), rad * np.sin(ang)])
        assert np.all(d_p <= np.sqrt(np.sum((q - z) ** 2, axis=0)) + 1e-15)


def test_projection_ties_and_zero_weight():
    q = np.array([[0.3, 0.0, 0.6], [0.4, 0.0, 0.8]])
    p = oracle.project_ball(q, 0.5)       # |q| = 0.5, 0, 1.0
    np.testing.assert_array_equal(p[:, 0], q[:, 0])   # tie keeps q
    np.testing.assert_array_equal(p[:, 1], 0.0)
    np.testing.assert_allclose(p[:, 2], [0.3, 0.4], atol=1e-16)
    assert np.all(oracle.project_ball(q, 0.0) == 0.0)


def test_data_prox_minimises():
    """(v + tau g)/(1 + tau) minimises 1/2 |x - v|^2 + tau/2 |x - g|^2."""
    rng = np.random.default_rng(8)
    v, g = rng.normal(size=50), rng.normal(size=50)
    tau = 0.37
    x = oracle.prox_data(v, g, tau)
    np.testing.assert_allclose((x - v) + tau * (x - g), 0.0, atol=1e-15)


def test_gap_density_identity():
    """sum of the gap density equals P - D, and every term is >= 0 for a
    feasible dual."""
    rng = np.random.default_rng(9)
    for shape in [(23, 31), (6, 7, 8)]:
        g = rng.normal(size=shape)
        f = rng.normal(size=shape)
        lam = 0.3
        p = oracle.project_ball(rng.normal(size=(len(shape),) + shape), lam)
        P, D, gap = oracle.energy_gap(f, p, g, lam)
        assert abs(gap - (P - D)) <= 1e-10 * abs(P)
        assert np.all(oracle.gap_density(f, p, g, lam) >= -1e-14)


def test_step_sizes_default():
    assert math.isclose(1.0 / math.sqrt(8.0) ** 2 * oracle.step_bound((256, 256)),
                        oracle.step_bound((256, 256)) / 8.0)
    assert (1.0 / 8.0) * oracle.step_bound((4096, 4096)) < 1.0
    assert (1.0 / 12.0) * oracle.step_bound((256, 256, 256)) < 1.0
