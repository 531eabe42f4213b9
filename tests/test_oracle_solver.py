"""Pins of the oracle's iteration and solution (CPU only)."""
import math

import numpy as np
import pytest
import scipy.fft as sfft

import oracle
import pins
from scenes import scene2d, scene3d

TAU2 = SIG2 = 1.0 / math.sqrt(8.0)


def test_quadratic_variant_matches_cosine_filter():
    """With the quadratic regulariser (lam/2)|grad f|^2 the iteration must
    converge to the closed-form filter solution DCT^{-1}[DCT(g)/(1 + lam mu)]
    (the cosine-transform analogue of the paper's Fourier filter, Section 6,
    eq. quaseo / eq. reg_fst).  This pins the order of the updates, both
    proximal maps and the operators together."""
    rng = np.random.default_rng(11)
    H, W = 12, 17
    g = rng.normal(size=(H, W))
    lam = 0.7
    mu = (4 * np.sin(np.pi * np.arange(H) / (2 * H)) ** 2)[:, None] + \
         (4 * np.sin(np.pi * np.arange(W) / (2 * W)) ** 2)[None, :]
    exact = sfft.idctn(sfft.dctn(g, norm="ortho") / (1 + lam * mu), norm="ortho")
    f, f_prev, p = oracle.init_state(g)
    for _ in range(3000):
        f_new, p = oracle.quadratic_iteration(f, f_prev, p, g, lam, TAU2, SIG2)
        f_prev, f = f, f_new
    np.testing.assert_allclose(f, exact, rtol=0, atol=1e-12)
    # dual optimum: p = lam grad f
    np.testing.assert_allclose(p, lam * oracle.grad(exact), rtol=0, atol=1e-12)


def test_quadratic_variant_3d():
    rng = np.random.default_rng(12)
    shape = (5, 6, 7)
    g = rng.normal(size=shape)
    lam = 0.5
    mu = sum((4 * np.sin(np.pi * np.arange(n) / (2 * n)) ** 2).reshape(
        [n if a == ax else 1 for a in range(3)]) for ax, n in enumerate(shape))
    exact = sfft.idctn(sfft.dctn(g, norm="ortho") / (1 + lam * mu), norm="ortho")
    t = s = 1.0 / math.sqrt(12.0)
    f, f_prev, p = oracle.init_state(g)
    for _ in range(3000):
        f_new, p = oracle.quadratic_iteration(f, f_prev, p, g, lam, t, s)
        f_prev, f = f, f_new
    np.testing.assert_allclose(f, exact, rtol=0, atol=1e-12)


@pytest.mark.parametrize("lam", [0.05, 0.3])
def test_one_dimensional_reduction(lam):
    """g constant along y: every iterate stays constant along y, and the
    solution's rows equal the exact 1D total-variation solution."""
    rng = np.random.default_rng(13)
    row = np.cumsum(rng.normal(scale=0.3, size=24)) * 0.2 + \
        (np.arange(24) > 11) * 1.0
    g = np.tile(row, (6, 1))
    r = oracle.solve(g, lam, TAU2, SIG2, max_iter=200000, check_every=50,
                     gap_tol=1e-15)
    assert np.max(np.abs(r["f"] - r["f"][0:1])) == 0.0
    # the 2D energy of a y-constant image is H times the 1D energy
    exact = pins.tv1d_exact(row, lam)
    assert pins.tv1d_certificate(exact, row, lam) < 1e-12
    np.testing.assert_allclose(r["f"][0], exact, rtol=0, atol=1e-6)
    bound = math.sqrt(2 * r["gap"])
    assert np.linalg.norm(r["f"] - np.tile(exact, (6, 1))) <= bound + 1e-9


def test_large_weight_gives_mean():
    rng = np.random.default_rng(14)
    g = rng.normal(size=(16, 16))
    r = oracle.solve(g, 50.0, TAU2, SIG2, max_iter=20000, check_every=10,
                     gap_tol=1e-14)
    np.testing.assert_allclose(r["f"], g.mean(), rtol=0, atol=1e-7)


@pytest.mark.parametrize("seed,lam", [(15, 0.3), (16, 0.1)])
def test_bruteforce_8x8(seed, lam):
    """8x8 images: the iteration's limit equals the minimiser found by a
    generic constrained optimiser on the dual problem built from explicit
    matrices."""
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(8, 8))
    f_bf, res = pins.tv2d_bruteforce(g, lam)
    r = oracle.solve(g, lam, TAU2, SIG2, max_iter=400000, check_every=100,
                     gap_tol=1e-13)
    assert r["converged"]
    np.testing.assert_allclose(r["f"], f_bf, rtol=0, atol=2e-6)
    # primal energies agree and the oracle's is not higher
    P_or = oracle.primal_energy(r["f"], g, lam)
    P_bf = oracle.primal_energy(f_bf, g, lam)
    assert P_or <= P_bf + 1e-12
    assert P_bf - P_or < 1e-6   # the optimiser stops on its objective change


def test_kkt_at_solution():
    """Optimality (the pattern of the paper's normal equations, Section 6,
    eq. neq): f = g + div p with p_i = lam grad f_i / |grad f_i| where the
    gradient is non-zero and |p_i| <= lam everywhere."""
    rng = np.random.default_rng(17)
    g = rng.normal(size=(10, 12))
    lam = 0.2
    r = oracle.solve(g, lam, TAU2, SIG2, max_iter=400000, check_every=100,
                     gap_tol=1e-14)
    f, p = r["f"], r["p"]
    np.testing.assert_allclose(f, g + oracle.div(p), atol=1e-6)
    gf = oracle.grad(f)
    n = np.sqrt(np.sum(gf * gf, axis=0))
    big = n > 1e-3
    np.testing.assert_allclose(p[:, big], lam * gf[:, big] / n[big], atol=1e-4)
    assert np.all(np.sqrt(np.sum(p * p, axis=0)) <= lam * (1 + 1e-12))


def test_transpose_equivariance():
    """Solving the transposed image gives the transposed iterates exactly
    (catches an x/y mix-up on non-square images)."""
    _, g = scene2d(20, 33, 6, 0.1, 21)
    lam = 0.1
    f1, _, p1 = oracle.run_fixed(g, lam, TAU2, SIG2, 37)
    f2, _, p2 = oracle.run_fixed(g.T.copy(), lam, TAU2, SIG2, 37)
    assert np.array_equal(f1.T, f2)
    assert np.array_equal(p1[0].T, p2[1]) and np.array_equal(p1[1].T, p2[0])


def test_invariances():
    _, g = scene2d(24, 19, 6, 0.1, 22)
    lam = 0.1
    f, _, p = oracle.run_fixed(g, lam, TAU2, SIG2, 25)
    # shift: f -> f + c, p unchanged
    fs, _, ps = oracle.run_fixed(g + 0.75, lam, TAU2, SIG2, 25)
    np.testing.assert_allclose(fs, f + 0.75, atol=1e-12)
    np.testing.assert_allclose(ps, p, atol=1e-12)
    # scale: g -> a g and lam -> a lam give f -> a f, p -> a p
    a = 3.0
    fa, _, pa = oracle.run_fixed(a * g, a * lam, TAU2, SIG2, 25)
    np.testing.assert_allclose(fa, a * f, atol=1e-12)
    np.testing.assert_allclose(pa, a * p, atol=1e-12)
    # lam = 0: the dual stays 0 and f stays g
    f0, _, p0 = oracle.run_fixed(g, 0.0, TAU2, SIG2, 25)
    assert np.all(p0 == 0.0)
    np.testing.assert_allclose(f0, g, atol=1e-15)
    # constant image: solved at k = 0 with zero gap
    r = oracle.solve(np.full((9, 9), 0.3), lam, TAU2, SIG2, max_iter=100,
                     check_every=10, gap_tol=1e-4)
    assert r["converged"] and r["iters"] == 0 and r["gap"] == 0.0


def test_mass_conservation():
    _, g = scene2d(31, 29, 8, 0.1, 23)
    f, _, _ = oracle.run_fixed(g, 0.1, TAU2, SIG2, 50)
    assert abs(f.sum() - g.sum()) < 1e-10 * g.size


def test_gap_nonnegative_and_monotone_on_scene():
    """Gap >= 0 at every check (weak duality) and, observed on this scene,
    non-increasing from check to check; it reaches a relative 1e-4 within the
    1000-iteration budget."""
    _, g = scene2d(256, 256, 20, 0.1, 1000)
    g = g.astype(np.float32).astype(np.float64)
    r = oracle.solve(g, 0.1, TAU2, SIG2, max_iter=1000, check_every=10,
                     gap_tol=1e-4, return_history=True)
    gaps = np.array([h[3] for h in r["history"]])
    Ps = np.array([h[1] for h in r["history"]])
    Ds = np.array([h[2] for h in r["history"]])
    assert np.all(gaps >= 0)
    assert np.all(np.diff(gaps) <= 1e-12 * gaps[:-1])
    np.testing.assert_allclose(gaps, Ps - Ds, rtol=1e-8)
    assert r["converged"] and r["iters"] < 1000


def test_single_disc_plateau():
    """Continuum ROF solution for g = c 1_{disc of radius R}: (c - 2 lam / R)
    inside.  On the grid only the centre value is checked, to within 15% of
    the predicted loss 2 lam / R (discrete perimeter error).  This fixes the
    1/2 on the data term: without it the loss would halve."""
    H = W = 112
    R, c, lam = 32.0, 1.0, 0.4
    yy, xx = np.mgrid[0:H, 0:W] + 0.5
    g = c * (((yy - H / 2) ** 2 + (xx - W / 2) ** 2) <= R * R)
    r = oracle.solve(g, lam, TAU2, SIG2, max_iter=20000, check_every=100,
                     gap_tol=1e-9)
    centre = r["f"][H // 2, W // 2]
    loss = 2 * lam / R
    assert abs((c - centre) - loss) <= 0.15 * loss
    # On a bounded grid with Neumann boundary the mass taken from the disc
    # (loss times area) lifts the background by lam * perimeter / outer area.
    lift = lam * 2 * math.pi * R / (H * W - math.pi * R * R)
    assert abs(r["f"][2, 2] - lift) <= 0.15 * lift


def test_3d_scene_runs_and_gap_decreases():
    _, g = scene3d(12, 14, 16, 6, 0.1, 31)
    r = oracle.solve(g, 0.1, max_iter=300, check_every=10, gap_tol=-1.0,
                     return_history=True)
    gaps = np.array([h[3] for h in r["history"]])
    assert np.all(gaps >= 0) and gaps[-1] < 0.05 * gaps[0]


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_trajectory_in_the_cosine_basis(theta):
    """The iterates themselves, not only their limit.  With lam so large that
    the projection never acts, the dual stays a gradient, p^k = grad psi^k,
    and -div grad is diagonal in the orthonormal type-II DCT (eigenvalue mu
    per mode), so every mode of (f, psi) follows the scalar form of the
    iteration from f^0 = f^{-1} = g, psi^0 = 0:
        psi' = psi + sigma (f + theta (f - f_prev)),
        f'   = (f - tau mu psi' + tau g) / (1 + tau).
    This fixes the extrapolation, the order of the two updates and where each
    step size enters, none of which the limit depends on."""
    rng = np.random.default_rng(18)
    H, W = 9, 13
    g = rng.normal(size=(H, W))
    tau, sigma = 0.3, 0.25
    mu = (4 * np.sin(np.pi * np.arange(H) / (2 * H)) ** 2)[:, None] + \
         (4 * np.sin(np.pi * np.arange(W) / (2 * W)) ** 2)[None, :]
    G = pins.grad_matrix((H, W))
    gh = sfft.dctn(g, norm="ortho")
    fh, fh_prev, psih = gh.copy(), gh.copy(), np.zeros_like(gh)
    f, f_prev, p = oracle.init_state(g)
    for _ in range(10):
        psih = psih + sigma * (fh + theta * (fh - fh_prev))
        fh_prev, fh = fh, (fh - tau * mu * psih + tau * gh) / (1 + tau)
        f_new, p = oracle.pdhg_iteration(f, f_prev, p, g, 1e30, tau, sigma, theta)
        f_prev, f = f, f_new
        np.testing.assert_allclose(f, sfft.idctn(fh, norm="ortho"), rtol=0, atol=1e-12)
        psi = sfft.idctn(psih, norm="ortho")
        np.testing.assert_allclose(p, (G @ psi.ravel()).reshape(2, H, W),
                                   rtol=0, atol=1e-12)
