"""Pins of the FP64 tomography oracle (no GPU).

The projection and the backprojection are pinned by what the geometry fixes
exactly (adjointness, mass and first moment of every projection, line sums at
0 and 90 degrees, the half-turn and transpose symmetries), against the
independent line integrals of an ellipse phantom (Section 1 eq. P_theta), and
against the backprojection of a point source (Section 4, Example I: 1/|x - a|
once the printed form's sine and cosine are put back in place).  The
iteration is pinned by its first step in closed form, by the normal equation
of the Tikhonov problem (Section 6, eq. neq2), by the constant solution for a
large TV weight and by the TV solution of an independent solver (ADMM).
"""
import math

import numpy as np
import pytest

import scenes
from oracle import tomo
from pins import tomo_tv_admm


def rng(seed):
    return np.random.default_rng(seed)


def dense_A(H, W, na, nd):
    cols = []
    for j in range(H * W):
        e = np.zeros(H * W)
        e[j] = 1.0
        cols.append(tomo.project(e.reshape(H, W), na, nd).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("H,W,na,nd", [(37, 53, 30, 41), (16, 16, 7, 40),
                                       (5, 9, 1, 3), (20, 11, 64, 80)])
def test_adjoint_pair(H, W, na, nd):
    f = rng(1).normal(size=(H, W))
    s = rng(2).normal(size=(na, nd))
    lhs = float(np.sum(tomo.project(f, na, nd) * s))
    rhs = float(np.sum(f * tomo.backproject(s, H, W)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(f).sum() * np.abs(s).sum() * 1e-3)


@pytest.mark.parametrize("H,W,na", [(37, 53, 30), (64, 64, 48), (9, 4, 13)])
def test_mass_and_first_moment_of_every_projection(H, W, na):
    nd = int(math.ceil(math.hypot(H, W))) + 3
    f = rng(3).uniform(-1, 2, size=(H, W))
    s = tomo.project(f, na, nd)
    t = tomo.detector(nd)
    x, y = tomo.pixel_centres(H, W)
    for k, th in enumerate(tomo.angles(na)):
        assert s[k].sum() == pytest.approx(f.sum(), rel=1e-12, abs=1e-12)
        mom = float(np.sum(f * (x * math.cos(th) + y * math.sin(th))))
        assert float(np.sum(t * s[k])) == pytest.approx(mom, rel=1e-11, abs=1e-10)


def test_line_sums_at_0_and_90_degrees():
    H, W, na = 14, 22, 8
    nd = 30                       # nd - W and nd - H even: bins on pixel centres
    f = rng(4).normal(size=(H, W))
    s = tomo.project(f, na, nd)
    ox, oy = (nd - W) // 2, (nd - H) // 2
    np.testing.assert_allclose(s[0, ox:ox + W], f.sum(axis=0), rtol=0, atol=1e-12)
    assert np.all(s[0, :ox] == 0) and np.all(s[0, ox + W:] == 0)
    np.testing.assert_allclose(s[na // 2, oy:oy + H], f.sum(axis=1), rtol=0, atol=1e-12)


def test_half_turn_and_transpose_symmetries():
    N, na, nd = 24, 12, 37
    f = rng(5).normal(size=(N, N))
    s = tomo.project(f, na, nd)
    np.testing.assert_allclose(tomo.project(f[::-1, ::-1], na, nd), s[:, ::-1],
                               rtol=0, atol=1e-12)
    sT = tomo.project(f.T, na, nd)
    for k in range(na):
        ref = s[na // 2 - k] if k <= na // 2 else s[3 * na // 2 - k, ::-1]
        np.testing.assert_allclose(sT[k], ref, rtol=0, atol=1e-12)


def test_projection_of_ellipse_phantom_matches_line_integrals():
    # pixel sampling of the phantom costs a few percent; a wrong scale, axis
    # or sign costs far more
    img, clean, _ = scenes.tomo_scene(128, 128, 60, 184, n_ellipses=12, seed=7)
    s = tomo.project(img, 60, 184)
    err = np.linalg.norm(s - clean) / np.linalg.norm(clean)
    assert err < 0.03
    wrong = tomo.project(img[::-1, :], 60, 184)   # y axis flipped
    assert np.linalg.norm(wrong - clean) / np.linalg.norm(clean) > 0.3


def test_point_source_backprojection():
    # dtheta * A^T A e_a approximates the backprojection of a point source's
    # sinogram, 1/|x - a| (unit-integral hat kernels in t).  Pixel by pixel
    # the discrete kernel aliases (about +-30 %), so the check is on annulus
    # means and on 7 x 7 local means.
    from scipy.ndimage import uniform_filter
    N, na = 96, 1440
    nd = 140
    f = np.zeros((N, N))
    a, b = 40, 51
    f[a, b] = 1.0
    bimg = (math.pi / na) * tomo.backproject(tomo.project(f, na, nd), N, N)
    x, y = tomo.pixel_centres(N, N)
    r = np.hypot(x - x[a, b], y - y[a, b])
    for lo, hi in ((15, 25), (25, 35)):
        ring = (r >= lo) & (r <= hi)
        assert abs(float(np.mean(bimg[ring] * r[ring])) - 1.0) < 0.003
    ring = (r >= 15) & (r <= 35)
    local = uniform_filter(bimg, 7) / uniform_filter(1.0 / np.maximum(r, 1e-9), 7)
    assert float(np.max(np.abs(local[ring] - 1.0))) < 0.05


def test_opnorm_is_largest_eigenvalue():
    H, W, na, nd = 10, 12, 16, 20
    A = dense_A(H, W, na, nd)
    lmax = float(np.linalg.eigvalsh(A.T @ A)[-1])
    assert tomo.opnorm_sq(H, W, na, nd, 400) == pytest.approx(lmax, rel=1e-9)


def test_first_iteration_closed_form():
    H, W, na, nd = 12, 15, 9, 21
    g = rng(6).normal(size=(na, nd))
    tau, sr, sp = 0.02, 0.03, 0.5
    for reg, lam in (("tv", 0.7), ("tikhonov", 0.7)):
        st = tomo.iteration(tomo.init_state(H, W, na, nd), g, lam, tau, sr, sp, reg)
        r1 = -sr * g / (1 + sr)
        np.testing.assert_allclose(st["r"], r1, rtol=1e-14, atol=1e-15)
        f1 = -tau * tomo.backproject(r1, H, W)
        if reg == "tikhonov":
            f1 = f1 / (1 + tau * lam)
        np.testing.assert_allclose(st["f"], f1, rtol=1e-13, atol=1e-15)
        assert np.all(st["p"] == 0)


@pytest.mark.parametrize("reg,theta", [("tv", 1.0), ("tv", 0.5),
                                       ("tikhonov", 1.0), ("tikhonov", 0.5)])
def test_trajectory_with_two_orthogonal_projections(reg, theta):
    """The iterates themselves, not only their limit.  With the angles 0 and
    90 degrees and the bins on the pixel centres (n_det = H = W = N), A f is
    the column sums and the row sums of f.  In orthonormal DCT bases (2D for
    the image, 1D along each projection) A has only the entries sqrt(N), from
    image mode (0, k) to mode k of projection 0 and from (k, 0) to mode k of
    projection 1, and -div grad is diagonal (eigenvalue mu).  With lam so
    large that the TV projection never acts, p = grad psi, and the iteration
    runs mode by mode from a warm start f^0 = f^{-1}, r^0 = 0, psi^0 = 0:
        fbar = f + theta (f - f_prev)
        r'   = (r + sigma_r (C fbar - g)) / (1 + sigma_r)
        psi' = psi + sigma_p fbar,  f' = f - tau (C^T r' + mu psi')   (TV)
        f'   = (f - tau C^T r') / (1 + tau lam)                       (Tikhonov)
    """
    import scipy.fft as sfft
    from pins import grad_matrix
    N = 8
    f0 = rng(30).normal(size=(N, N))
    g = rng(31).normal(size=(2, N))
    tau, sr, sp = 0.2, 0.3, 0.4
    lam = 1e30 if reg == "tv" else 0.7
    k = np.arange(N)
    lap1 = 4 * np.sin(np.pi * k / (2 * N)) ** 2
    mu = lap1[:, None] + lap1[None, :]
    c = math.sqrt(N)

    def C(fh):
        return np.stack([c * fh[0, :], c * fh[:, 0]])

    def Ct(rh):
        out = np.zeros((N, N))
        out[0, :] += c * rh[0]
        out[:, 0] += c * rh[1]
        return out

    gh = sfft.dct(g, norm="ortho", axis=1)
    fh = sfft.dctn(f0, norm="ortho")
    fh_prev, rh, psih = fh.copy(), np.zeros((2, N)), np.zeros((N, N))
    st = tomo.init_state(N, N, 2, N, f0)
    G = grad_matrix((N, N))
    for _ in range(8):
        fbar = fh + theta * (fh - fh_prev)
        rh = (rh + sr * (C(fbar) - gh)) / (1 + sr)
        if reg == "tv":
            psih = psih + sp * fbar
            fnew = fh - tau * (Ct(rh) + mu * psih)
        else:
            fnew = (fh - tau * Ct(rh)) / (1 + tau * lam)
        fh_prev, fh = fh, fnew
        st = tomo.iteration(st, g, lam, tau, sr, sp, reg, theta)
        np.testing.assert_allclose(st["f"], sfft.idctn(fh, norm="ortho"),
                                   rtol=0, atol=1e-12)
        np.testing.assert_allclose(st["r"], sfft.idct(rh, norm="ortho", axis=1),
                                   rtol=0, atol=1e-12)
        psi = sfft.idctn(psih, norm="ortho")
        np.testing.assert_allclose(st["p"], (G @ psi.ravel()).reshape(2, N, N),
                                   rtol=0, atol=1e-12)


def test_tikhonov_limit_solves_the_normal_equation():
    H, W, na, nd = 10, 8, 12, 16
    img, _, g = scenes.tomo_scene(H, W, na, nd, n_ellipses=4, noise=0.05, seed=8)
    lam = 3.0
    L2 = tomo.opnorm_sq(H, W, na, nd, 200)
    tau = sr = 0.99 / math.sqrt(L2)
    st = tomo.run(g, H, W, lam, tau, sr, 0.0, 3000, reg="tikhonov")
    A = dense_A(H, W, na, nd)
    ref = np.linalg.solve(A.T @ A + lam * np.eye(H * W), A.T @ g.ravel())
    err = np.linalg.norm(st["f"].ravel() - ref) / np.linalg.norm(ref)
    assert err < 1e-9


def test_tv_large_weight_gives_the_best_constant():
    H, W, na, nd = 8, 9, 10, 16
    _, _, g = scenes.tomo_scene(H, W, na, nd, n_ellipses=3, noise=0.05, seed=9)
    L2 = tomo.opnorm_sq(H, W, na, nd, 200)
    tau = 1.0 / math.sqrt(L2)
    sr, sp = 0.5 / math.sqrt(L2), math.sqrt(L2) / 16
    st = tomo.run(g, H, W, 1e4, tau, sr, sp, 7000, reg="tv")
    a1 = tomo.project(np.ones((H, W)), na, nd)
    c = float(np.sum(a1 * g) / np.sum(a1 * a1))
    np.testing.assert_allclose(st["f"], c, rtol=1e-6, atol=0)


def test_tv_limit_matches_an_independent_solver():
    H, W, na, nd = 8, 7, 12, 14
    _, _, g = scenes.tomo_scene(H, W, na, nd, n_ellipses=4, noise=0.05, seed=10)
    lam = 2.0
    L2 = tomo.opnorm_sq(H, W, na, nd, 200)
    tau = 1.0 / math.sqrt(L2)
    sr, sp = 0.5 / math.sqrt(L2), math.sqrt(L2) / 16
    st = tomo.run(g, H, W, lam, tau, sr, sp, 10000, reg="tv")
    ref = tomo_tv_admm(dense_A(H, W, na, nd), g, lam, (H, W), rho=10.0, iters=3000)
    assert np.linalg.norm(st["f"] - ref) / np.linalg.norm(ref) < 1e-6
    # the data term's dual variable converges to the residual A f - g
    res = tomo.project(st["f"], na, nd) - g
    assert np.linalg.norm(st["r"] - res) / np.linalg.norm(res) < 1e-6


def test_energy_terms():
    H, W, na, nd = 11, 13, 9, 19
    f = rng(11).normal(size=(H, W))
    g = rng(12).normal(size=(na, nd))
    lam = 0.3
    A = dense_A(H, W, na, nd)
    res = A @ f.ravel() - g.ravel()
    from pins import grad_matrix
    Gf = (grad_matrix((H, W)) @ f.ravel()).reshape(2, -1)
    d, r, tot = tomo.energy(f, g, lam, "tv")
    assert d == pytest.approx(0.5 * res @ res, rel=1e-13)
    assert r == pytest.approx(lam * np.sum(np.hypot(Gf[0], Gf[1])), rel=1e-13)
    assert tot == pytest.approx(d + r, rel=1e-15)
    d2, r2, _ = tomo.energy(f, g, lam, "tikhonov")
    assert d2 == pytest.approx(d, rel=1e-15)
    assert r2 == pytest.approx(0.5 * lam * np.sum(f * f), rel=1e-13)


def test_single_entries_match_the_full_operators():
    H, W, na, nd = 23, 31, 17, 29          # detector narrower than the image
    f = rng(13).normal(size=(H, W))
    s = rng(14).normal(size=(na, nd))
    A = tomo.project(f, na, nd)
    B = tomo.backproject(s, H, W)
    ks, iis = np.meshgrid(np.arange(na), np.arange(nd), indexing="ij")
    np.testing.assert_allclose(tomo.project_at(f, na, nd, ks.ravel(), iis.ravel()),
                               A.ravel(), rtol=1e-12, atol=1e-12)
    rr, cc = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    np.testing.assert_allclose(tomo.backproject_at(s, H, W, rr.ravel(), cc.ravel()),
                               B.ravel(), rtol=1e-12, atol=1e-12)


def test_ramp_filter_impulse_response():
    # lam = 0: the response of an impulse is the ramp filter's kernel on the
    # L-periodic grid: h[0] = 1/4 exactly, and close to the band-limited ramp
    # kernel h[n] = -1/(pi n)^2 (n odd), 0 (n even) of the standard
    # inversion formula (Kak & Slaney, Section 3.3)
    nd = 200
    L = tomo.fbp_length(nd)
    assert L == 512
    e = np.zeros((1, nd))
    e[0, 100] = 1.0
    h = tomo.fbp_filter(e, 0.0)[0]
    assert h[100] == pytest.approx(0.25, abs=1e-12)
    for n in (1, 3, 5, 7):
        assert h[100 + n] == pytest.approx(-1.0 / (math.pi * n) ** 2, rel=2e-3)
        assert h[100 - n] == pytest.approx(h[100 + n], rel=1e-12)
    for n in (2, 4, 6):
        assert abs(h[100 + n]) < 1e-4
    # lam > 0 damps the high frequencies: a smaller centre tap, same sum
    h4 = tomo.fbp_filter(e, 4.0)[0]
    assert 0 < h4[100] < h[100]


def test_fbp_reconstructs_the_phantom():
    # lam = 0, exact line integrals of an ellipse phantom: the inversion
    # formula's discretisation error, a wrong scale, axis or filter fails
    N, na = 128, 180
    nd = int(math.ceil(math.hypot(N, N))) + 4
    img, clean, _ = scenes.tomo_scene(N, N, na, nd, n_ellipses=10, noise=0.0, seed=21)
    f = tomo.fbp(clean, N, N, 0.0)
    assert np.linalg.norm(f - img) / np.linalg.norm(img) < 0.15
    on = img > 0.05
    assert abs(float(np.median(f[on] / img[on])) - 1.0) < 0.02


def test_regularised_fbp_approximates_the_tikhonov_solution():
    # Section 6: f_lam = B F_lam g solves the (continuous) Tikhonov problem;
    # with B = dtheta A^T its discrete counterpart is (A^T A + lam/dtheta) f =
    # A^T g.  The two agree up to discretisation (7 % and 5 % here; a factor
    # of 2 in the weight gives 20 % and more)
    N, na = 24, 40
    nd = int(math.ceil(math.hypot(N, N))) + 4
    _, clean, _ = scenes.tomo_scene(N, N, na, nd, n_ellipses=5, noise=0.0, seed=22)
    A = dense_A(N, N, na, nd)
    dth = math.pi / na
    for lam in (4.0, 16.0):
        fb = tomo.fbp(clean, N, N, lam)
        ft = np.linalg.solve(A.T @ A + (lam / dth) * np.eye(N * N),
                             A.T @ clean.ravel()).reshape(N, N)
        assert np.linalg.norm(fb - ft) / np.linalg.norm(ft) < 0.1


def test_bst_spectra_are_the_dft_of_the_projections():
    # step 1-2 against an FFT of the zero-padded projections (a different
    # algorithm), with the kernel 1/|nu| and the origin rule 1/dnu
    na, nd, M = 5, 37, 128
    s = rng(15).normal(size=(na, nd))
    P = tomo.bst_spectra(s, M)
    t0 = tomo.detector(nd)[0]
    nu = (np.arange(M) - M // 2) / M
    G = np.fft.fftshift(np.fft.fft(s, n=M, axis=1), axes=1) * np.exp(-2j * np.pi * nu * t0)
    K = np.where(nu == 0, M, 1.0 / np.where(nu == 0, 1.0, np.abs(nu)))
    np.testing.assert_allclose(P, G * K, rtol=1e-10, atol=1e-10 * np.abs(G).max())


def test_bst_interpolation_is_exact_for_radial_affine_spectra():
    # a spectrum a + b |nu|, the same at every angle, is bilinear in
    # (theta, nu) piecewise, so its Cartesian samples are a + b rho exactly
    na, M, Q = 12, 64, 64
    nu = (np.arange(M) - M // 2) / M
    P = np.tile(2.0 + 3.0 * np.abs(nu), (na, 1)).astype(complex)
    F = tomo.bst_cartesian(P, Q)
    f = (np.arange(Q) - Q // 2) / Q
    u, v = np.meshgrid(f, f)
    rho = np.hypot(u, v)
    ok = rho <= 0.5 - 1.0 / M
    np.testing.assert_allclose(F[ok].real, 2.0 + 3.0 * rho[ok], rtol=1e-12, atol=1e-12)
    assert np.all(F[rho > 0.5] == 0)


def test_bst_interpolation_is_exact_for_bilinear_spectra():
    # (1 + theta)(2 + 3 |nu|) is bilinear in (theta, nu) on every cell of the
    # polar grid (|nu| bends only at the node nu = 0), so its Cartesian
    # samples are exact everywhere except in the last angular cell, where
    # theta wraps from pi back to 0 with nu -> -nu
    na, M, Q = 12, 64, 64
    th = tomo.angles(na)
    nu = (np.arange(M) - M // 2) / M
    P = ((1.0 + th)[:, None] * (2.0 + 3.0 * np.abs(nu))[None, :]).astype(complex)
    F = tomo.bst_cartesian(P, Q)
    f = (np.arange(Q) - Q // 2) / Q
    u, v = np.meshgrid(f, f)
    rho = np.hypot(u, v)
    theta = np.mod(np.arctan2(v, u), np.pi)
    ok = (rho <= 0.5 - 1.0 / M) & (theta <= th[-1])
    assert ok.sum() > 0.6 * Q * Q
    np.testing.assert_allclose(F[ok].real, (1 + theta[ok]) * (2 + 3 * rho[ok]),
                               rtol=1e-12, atol=1e-12)


def test_bst_equals_the_backprojection_up_to_the_origin_constant():
    # The BST reproduces B g = dtheta A^T g except for a constant: the
    # origin rule K(0) = 1/dnu misses part of the integral of 1/|nu| over the
    # cells next to the origin.  After removing the mean the two agree to
    # 0.6 %; the constant halves when the grids are refined twofold.
    N, na = 128, 400
    nd = int(math.ceil(math.hypot(N, N))) + 4
    _, clean, _ = scenes.tomo_scene(N, N, na, nd, n_ellipses=8, noise=0.0, seed=31)
    ref = (math.pi / na) * tomo.backproject(clean, N, N)
    b = tomo.bst(clean, N, N)
    d = b - ref
    assert np.linalg.norm(d - d.mean()) / np.linalg.norm(ref) < 0.008
    M, Q = tomo.bst_lengths(N, N, nd)
    F2 = tomo.bst_cartesian(tomo.bst_spectra(clean, 2 * M), 2 * Q)
    f = (np.arange(2 * Q) - Q) / (2 * Q)
    x = np.arange(N) + 0.5 - N / 2.0
    b2 = np.real(np.exp(2j * np.pi * np.outer(x, f)) @ F2 @
                 np.exp(2j * np.pi * np.outer(f, x))) / (2 * Q) ** 2
    d2 = b2 - ref
    assert 0.4 < d2.mean() / d.mean() < 0.6


def test_bst_of_a_disc_at_its_centre():
    # B R of a disc's indicator is its convolution with 1/|x| (Section 3,
    # Remark 1), 2 pi R at the centre: the BST is low there by the origin
    # constant only
    N, na, R = 128, 360, 30.0
    nd = int(math.ceil(math.hypot(N, N))) + 4
    t = tomo.detector(nd)
    g = np.tile(2.0 * np.sqrt(np.maximum(R * R - t * t, 0.0)), (na, 1))
    b = tomo.bst(g, N, N)
    ref = (math.pi / na) * tomo.backproject(g, N, N)
    c = slice(N // 2 - 1, N // 2 + 1)
    assert abs(ref[c, c].mean() / (2 * math.pi * R) - 1.0) < 0.002
    off = float(np.mean(b - ref))
    assert abs((b[c, c].mean() - off) / (2 * math.pi * R) - 1.0) < 0.01


def test_bst_slice_of_a_disc_follows_the_analytic_backprojection():
    # The comparison of the paper's slice figure (Section 7, Example 2 of
    # Section 4): the backprojection of a disc's exact sinogram along a row
    # through its centre.  Reference: B g(x) = int_0^pi g(x . xi_theta) dtheta
    # by adaptive quadrature, with g(t) = 2 sqrt(R^2 - t^2).  The BST follows
    # it up to the origin constant (about 10 % of 2 pi R at these grids):
    # after removing the constant, within 0.5 % of 2 pi R everywhere on the
    # row (the exact linear-interpolation backprojection: 0.35 %).
    from scipy.integrate import quad
    N, na, R = 128, 360, 30.0
    nd = int(math.ceil(math.hypot(N, N))) + 4
    t = tomo.detector(nd)
    g = np.tile(2.0 * np.sqrt(np.maximum(R * R - t * t, 0.0)), (na, 1))
    b = tomo.bst(g, N, N)
    a = N // 2
    y = a + 0.5 - N / 2.0

    def Bg(r):
        def f(th):
            return 2.0 * math.sqrt(max(R * R - (r * math.cos(th)) ** 2, 0.0))
        pts = [math.acos(R / r), math.pi - math.acos(R / r)] if r > R else None
        return quad(f, 0.0, math.pi, points=pts, limit=200)[0]

    x = np.arange(N) + 0.5 - N / 2.0
    prof = np.array([Bg(math.hypot(xx, y)) for xx in x])
    d = b[a] - prof
    c = float(np.median(d))
    assert -0.15 < c / (2 * math.pi * R) < -0.05
    assert np.max(np.abs(d - c)) <= 0.007 * 2 * math.pi * R


def _fbp_scene():
    N, na = 128, 400
    nd = int(math.ceil(math.hypot(N, N))) + 4
    img, clean, _ = scenes.tomo_scene(N, N, na, nd, n_ellipses=8, noise=0.0, seed=31)
    return N, img, clean


def test_fbp_through_the_bst_matches_the_exact_backprojection():
    # Section 6: f_lam = B F_lam g with B by the BST is the gridding of
    # g^(nu) / (1 + lam |nu|) (eq. reg_fst).  Against the FBP with the exact
    # backprojection they agree up to a constant (the discrete filter is zero
    # at DC and loses part of the mean; the slice theorem keeps K(0) = 1) and
    # the polar interpolation: 2 % at lam = 8 here, where twice or half the
    # weight, or lam nu^2 in place of lam |nu|, gives 10 % and more
    N, _, clean = _fbp_scene()
    a = tomo.fbp(clean, N, N, 8.0)
    b = tomo.fbp_bst(clean, N, N, 8.0)
    d = b - a
    assert np.linalg.norm(d - d.mean()) / np.linalg.norm(a) < 0.03


def test_fbp_through_the_bst_keeps_the_mass_and_reconstructs():
    # lam = 0: the image's total equals the projections' mass (the DC of
    # B F_0 g is G(0) in the limit nu -> 0), and it reconstructs the phantom
    N, img, clean = _fbp_scene()
    b = tomo.fbp_bst(clean, N, N, 0.0)
    assert abs(b.sum() / clean[0].sum() - 1.0) < 0.005
    on = img > 0.05
    assert abs(float(np.median(b[on] / img[on])) - 1.0) < 0.02
    assert np.linalg.norm(b - img) / np.linalg.norm(img) < 0.15
    with pytest.raises(ValueError):
        tomo.fbp_bst(clean, N, N, -1.0)


@pytest.mark.parametrize("lam", [None, 0.0, 2.5])
def test_sampled_bst_equals_the_whole_image(lam):
    # bst_at evaluates the inverse DFT of the same grid at listed pixels
    # (rows and columns of a non-square image in arbitrary order, repeats
    # included)
    H, W, na, nd = 20, 13, 11, 30
    s = np.random.default_rng(4).normal(size=(na, nd))
    full = tomo.bst(s, H, W, lam)
    rows = np.array([0, 19, 7, 7, 3, 12, 19, 0])
    cols = np.array([12, 0, 5, 6, 12, 1, 12, 0])
    got = tomo.bst_at(s, H, W, rows, cols, lam)
    np.testing.assert_allclose(got, full[rows, cols], rtol=0,
                               atol=1e-12 * np.max(np.abs(full)))


@pytest.mark.parametrize("lam", [None, 0.0, 2.5])
def test_bst_spectra_of_a_disc_follow_example_ii(lam):
    # Section 4, Example II: the projections of a disc have the transform of
    # the disc on every slice, J1(sigma)/sigma for the unit disc, and the
    # BST's Fourier samples of b are that over |sigma|.  In cycles per pixel,
    # for a disc of radius R centred at c, the projection at angle theta is
    # 2 sqrt(R^2 - (t - u0)^2) with u0 = c . xi_theta, and its transform is
    # G(nu) = exp(-2 pi i nu u0) R J1(2 pi R |nu|) / |nu| (pi R^2 at nu = 0).
    # The step-2 samples are K(nu) G(nu): K = 1/|nu| (compared after the
    # factor |nu|, away from the origin rule) or 1/(1 + lam |nu|).  The
    # remaining difference is the sampling of the projection (its square-root
    # edge), about 1e-3 of pi R^2; a conjugated phase gives 0.55.
    from scipy.special import j1
    R, cx, cy = 30.0, 7.3, -4.1
    nd, na, M = 256, 3, 512
    t = tomo.detector(nd)
    th = tomo.angles(na)
    u0 = cx * np.cos(th) + cy * np.sin(th)
    s = 2.0 * np.sqrt(np.maximum(R * R - (t[None, :] - u0[:, None]) ** 2, 0.0))
    nu = (np.arange(M) - M // 2) / M
    a = np.abs(nu)
    G = np.where(a == 0.0, math.pi * R * R,
                 R * j1(2.0 * math.pi * R * a) / np.where(a == 0.0, 1.0, a))
    G = G[None, :] * np.exp(-2j * math.pi * np.outer(u0, nu))
    P = tomo.bst_spectra(s, M, lam)
    if lam is None:
        sel = (a > 0.0) & (a <= 0.25)
        err = np.abs(P[:, sel] * a[sel] - G[:, sel])
    else:
        sel = a <= 0.25
        err = np.abs(P[:, sel] - G[:, sel] / (1.0 + lam * a[sel]))
    assert err.max() <= 3e-3 * math.pi * R * R


def test_sinogram_mesh_follows_the_table_of_symbols():
    # tests/golden/mesh_symbols.txt: angles k pi / N_theta and detector cell
    # centres on [-1, 1] with step 2 / N_t (Section 5, table of symbols); the
    # oracle's detector is in pixel units, the table's values times N_t / 2.
    import os
    fn = os.path.join(os.path.dirname(__file__), "golden", "mesh_symbols.txt")
    rows = [ln.split() for ln in open(fn) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 12
    for kind, n, i, v in rows:
        n, i, v = int(n), int(i), float(v)
        if kind == "angle":
            assert abs(tomo.angles(n)[i] - v) <= 1e-15
            assert len(tomo.angles(n)) == n
        else:
            assert abs(tomo.detector(n)[i] - v * n / 2.0) <= 1e-12
