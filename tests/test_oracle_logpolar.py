"""Pins of the FP64 oracle for the log-polar backprojection (no GPU).

Each step of the algorithm (Section 5, "Algorithm for log-polar
backprojection") is pinned by what fixes it exactly: the mesh by the paper's
worked example after eq. N_rho (tests/golden/logpolar_mesh.txt) and by the
step bound that eq. N_rho is derived from; the interpolation onto the
log-polar mesh by linear projections; the kernel by its unit mass and first
moment (the delta of eq. and_kernel has its root at a = -ln cos b); the FFT
convolution by the direct sum and by the backprojection over the circle
through the origin that the formula encodes (Section 2.1, step (d)); the
return to the Cartesian grid by bilinear data; the whole method by rotation
equivariance, by the exact backprojection with the lines through the
innermost ring removed (what the adaptive rho_0 of "Problem near the origin"
drops), by the point source of Example I and by the disc's slice of Section 7.
"""
import math
import os

import numpy as np
import pytest

import scenes
from oracle import logpolar as lp
from oracle import tomo

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "logpolar_mesh.txt")


def golden():
    vals = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split()
            vals[k] = int(v)
    return vals


def truncated_backprojection(s, H, W, r0):
    """dtheta A^T s without the lines that pass within r0 of the origin (the
    lines whose foot point lies below the mesh)."""
    na, nd = s.shape
    x, y = tomo.pixel_centres(H, W)
    out = np.zeros((H, W))
    for k, th in enumerate(tomo.angles(na)):
        u = x * math.cos(th) + y * math.sin(th)
        v = u - (0.5 - nd / 2.0)
        ext = np.concatenate(([0.0], s[k], [0.0]))
        i0 = np.floor(v).astype(np.int64)
        w = v - i0
        val = (1 - w) * ext[np.clip(i0, -1, nd) + 1] + w * ext[np.clip(i0 + 1, -1, nd) + 1]
        out += np.where(np.abs(u) >= r0, val, 0.0)
    return (math.pi / na) * out


def phantom(N=128, na=400, seed=31):
    nd = int(math.ceil(math.hypot(N, N))) + 4
    _, clean, _ = scenes.tomo_scene(N, N, na, nd, n_ellipses=8, noise=0.0, seed=seed)
    return N, na, nd, clean


# --------------------------------------------------------------------------
# The mesh.
# --------------------------------------------------------------------------

def test_mesh_matches_the_papers_example():
    g = golden()
    # an image inside the detector's disc: the mesh ends at rho = 0
    side = g["N_x"] * 707 // 1000
    m = lp.mesh(side, side, 180, g["N_t"])
    assert m.rho()[-1] == pytest.approx(0.0, abs=1e-12)
    assert m.n_rho == g["N_rho"]
    # the full N_x x N_x image: the corners add nodes above rho = 0 only
    m = lp.mesh(g["N_x"], g["N_x"], 180, g["N_t"])
    assert abs(int(np.sum(m.rho() <= 1e-12)) - g["N_rho"]) <= 1


@pytest.mark.parametrize("H,W,nd", [(128, 128, 185), (64, 100, 64), (7, 5, 12),
                                    (2048, 2048, 2048)])
def test_mesh_steps_and_ends(H, W, nd):
    m = lp.mesh(H, W, 30, nd)
    R = nd / 2.0
    r = R * np.exp(m.rho())
    # inside the detector's disc the largest radial step is at most one bin
    # (eq. N_rho), and not much less; beyond it (image corners outside the
    # disc) the steps keep growing in proportion to the radius
    inner = r <= R * (1 + 1e-12)
    assert np.max(np.diff(r[inner])) <= 1.0 + 1e-12
    assert np.max(np.diff(r[inner])) > 1.0 - 2.0 * m.drho
    assert np.all(np.diff(r) <= r[1:] / R + 1e-12)
    # innermost node just above half a pixel; the top node reaches the
    # farthest pixel centre (or the detector's edge)
    assert 0.5 < r[0] <= 0.5 * math.exp(m.drho) + 1e-12
    rmax = math.hypot(W / 2 - 0.5, H / 2 - 0.5)
    assert r[-1] == pytest.approx(max(rmax, R), rel=1e-12)
    assert m.n_phi == 60 and m.dphi == pytest.approx(math.pi / 30)
    assert lp.conv_length(m) >= 2 * m.n_rho - 1


# --------------------------------------------------------------------------
# Step 1: onto the log-polar mesh.
# --------------------------------------------------------------------------

def test_step1_is_exact_for_linear_projections():
    na, nd, N = 9, 40, 40         # image corners beyond the detector's disc
    rng = np.random.default_rng(1)
    al, be = rng.normal(size=na), rng.normal(size=na)
    t = tomo.detector(nd)
    s = al[:, None] + be[:, None] * t[None, :]
    m = lp.mesh(N, N, na, nd)
    gL = lp.to_logpolar(s, m)
    r = m.R * np.exp(m.rho())
    inside = r <= nd / 2.0 - 0.5
    for j in range(m.n_phi):
        k, sign = (j, 1.0) if j < na else (j - na, -1.0)
        np.testing.assert_allclose(gL[j, inside], al[k] + be[k] * sign * r[inside],
                                   rtol=0, atol=1e-12)
    # beyond the last bin the value falls linearly to 0 at half a bin further
    out = r >= nd / 2.0 + 0.5
    assert out.sum() >= 5 and np.all(gL[:, out] == 0.0)


# --------------------------------------------------------------------------
# Step 2: the kernel.
# --------------------------------------------------------------------------

def test_kernel_has_unit_mass_at_the_root():
    m = lp.mesh(96, 96, 50, 140)
    k = lp.kernel(m)
    a = np.arange(m.n_rho) * m.drho
    c = np.cos(m.phi())
    amax = (m.n_rho - 1) * m.drho
    full = (c > 0) & (-np.log(np.where(c > 0, c, 1.0)) <= amax - m.drho)
    mass = k.sum(axis=1) * m.drho
    np.testing.assert_allclose(mass[full], 1.0, rtol=0, atol=1e-12)
    centre = (k * a[None, :]).sum(axis=1) * m.drho
    np.testing.assert_allclose(centre[full], -np.log(c[full]), rtol=0, atol=1e-12)
    assert np.all(k[c <= 0] == 0.0)
    # the kernel's band is the paper's |e^a cos b - 1| <= drho to first order
    nz = k > 0
    band = np.abs(np.exp(a)[None, :] * c[:, None] - 1.0)
    assert np.all(band[nz] <= m.drho * (1 + 2 * m.drho))
    assert np.max(k) <= 1.0 / m.drho + 1e-9


# --------------------------------------------------------------------------
# Step 3: the convolution.
# --------------------------------------------------------------------------

def test_convolution_equals_the_direct_sum():
    m = lp.mesh(6, 6, 5, 8)
    rng = np.random.default_rng(2)
    gL = rng.normal(size=(m.n_phi, m.n_rho))
    k = rng.normal(size=(m.n_phi, m.n_rho))
    got = lp.convolve(gL, k, m)
    ref = np.zeros_like(got)
    for j in range(m.n_phi):
        for i in range(m.n_rho):
            acc = 0.0
            for jj in range(m.n_phi):
                for ll in range(i + 1):
                    acc += k[jj, ll] * gL[(j - jj) % m.n_phi, i - ll]
            ref[j, i] = acc * m.drho * m.dphi
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_convolution_is_the_circle_backprojection():
    # [B g]_L(rho, theta) = sum over the rays phi within 90 degrees of theta
    # of [g]_L at the foot point mu = rho + ln cos(theta - phi), times dphi;
    # the hat kernel reads it by linear interpolation along rho (zero below
    # the first node, through a ramp from the node below it)
    m = lp.mesh(40, 40, 24, 60)
    gL = np.random.default_rng(3).normal(size=(m.n_phi, m.n_rho))
    got = lp.convolve(gL, lp.kernel(m), m)
    ext = np.concatenate([np.zeros((m.n_phi, 1)), gL], axis=1)   # node -1 is 0
    ref = np.zeros_like(got)
    for j in range(m.n_phi):
        for jj in range(m.n_phi):
            c = math.cos(jj * m.dphi)
            if c <= 0:
                continue
            x = np.arange(m.n_rho) + math.log(c) / m.drho + 1.0   # index in ext
            i0 = np.floor(x).astype(np.int64)
            w = x - i0
            ok = i0 >= 0
            v = np.zeros(m.n_rho)
            row = ext[(j - jj) % m.n_phi]
            v[ok] = (1 - w[ok]) * row[i0[ok]] + w[ok] * row[np.minimum(i0[ok] + 1, m.n_rho)]
            ref[j] += v
    ref *= m.dphi
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11)


# --------------------------------------------------------------------------
# Step 4: back to the Cartesian grid.
# --------------------------------------------------------------------------

def test_cartesian_step_is_exact_for_bilinear_data():
    H, W = 30, 44
    m = lp.mesh(H, W, 20, 50)
    i = np.arange(m.n_rho)[None, :]
    j = np.arange(m.n_phi)[:, None]
    bL = 0.3 + 0.02 * i - 0.05 * j + 0.001 * i * j
    out = lp.to_cartesian(bL, m, H, W)
    x, y = tomo.pixel_centres(H, W)
    u = (np.log(np.hypot(x, y) / m.R) - (m.rho0 + m.drho)) / m.drho
    v = np.mod(np.arctan2(y, x), 2 * math.pi) / m.dphi
    ok = v < m.n_phi - 1           # away from the seam of the periodic angle
    assert ok.sum() > 0.9 * ok.size
    ref = 0.3 + 0.02 * u - 0.05 * v + 0.001 * u * v
    np.testing.assert_allclose(out[ok], ref[ok], rtol=0, atol=1e-11)


# --------------------------------------------------------------------------
# The whole method.
# --------------------------------------------------------------------------

def test_rotation_by_one_angle_step_shifts_the_result():
    # theta -> theta + dtheta: row k of the new sinogram is row k - 1 of the
    # old one, and row 0 is the old last row read at -t
    N, na, nd = 20, 15, 30
    s = np.random.default_rng(4).normal(size=(na, nd))
    s2 = np.concatenate([s[-1:, ::-1], s[:-1]], axis=0)
    b = lp.logpolar_result(s, N, N)
    b2 = lp.logpolar_result(s2, N, N)
    np.testing.assert_allclose(b2, np.roll(b, 1, axis=0), rtol=0, atol=1e-12)


def test_equals_the_backprojection_without_the_lines_through_the_origin():
    N, na, nd, clean = phantom()
    b = lp.backproject_logpolar(clean, N, N)
    m = lp.mesh(N, N, na, nd)
    r0 = m.R * math.exp(m.rho0)
    ref = truncated_backprojection(clean, N, N, r0)
    assert np.linalg.norm(b - ref) / np.linalg.norm(ref) < 0.008
    # the lines dropped are a fraction (2/pi) arcsin(r0/r) of the angles at
    # radius r, the lines through the centre, which carry the most mass here:
    # near the origin the plain backprojection is far larger
    full = (math.pi / na) * tomo.backproject(clean, N, N)
    x, y = tomo.pixel_centres(N, N)
    near = np.hypot(x, y) < 4
    assert np.mean(b[near] - full[near]) < -0.05 * np.mean(full[near])


def test_constant_projections():
    # g = 1 on every bin: B g = pi inside the detector's disc, less the
    # angles of the lines within r0 of the origin: pi - 2 arcsin(r0 / r)
    N, na = 64, 360
    nd = 100
    b = lp.backproject_logpolar(np.ones((na, nd)), N, N)
    m = lp.mesh(N, N, na, nd)
    r0 = m.R * math.exp(m.rho0)
    x, y = tomo.pixel_centres(N, N)
    r = np.hypot(x, y)
    ref = math.pi - 2.0 * np.arcsin(np.minimum(1.0, r0 / r))
    ok = r >= 2.0
    assert np.max(np.abs(b[ok] - ref[ok])) < 0.01 * math.pi


def test_point_source_example_i():
    # Section 4, Example I: the backprojection of a point source's sinogram
    # is 1/|x - a| (once the printed form's sine and cosine are put back in
    # place); with the hat-sampled source A e_a, on annulus means.  The lines
    # through a that pass within r0 of the origin are dropped: a fraction
    # (2/pi) arcsin(r0/|a|) of the source's angles, and so of every annulus
    N, na = 96, 1440
    nd = 140
    f = np.zeros((N, N))
    a, c = 40, 51
    f[a, c] = 1.0
    b = lp.backproject_logpolar(tomo.project(f, na, nd), N, N)
    x, y = tomo.pixel_centres(N, N)
    d = np.hypot(x - x[a, c], y - y[a, c])
    m = lp.mesh(N, N, na, nd)
    r0 = m.R * math.exp(m.rho0)
    kept = 1.0 - 2.0 / math.pi * math.asin(r0 / math.hypot(x[a, c], y[a, c]))
    for lo, hi in ((5, 15), (15, 25), (25, 35)):
        ring = (d >= lo) & (d <= hi)
        assert abs(float(np.mean(b[ring] * d[ring])) - kept) < 0.005


def test_disc_slice_of_section_7():
    # The paper's slice comparison (Section 7, the disc of Example II): B g
    # along the row through the disc's centre, g(t) = 2 sqrt(R^2 - t^2), by
    # quadrature over the angles whose lines miss the innermost ring
    from scipy.integrate import quad
    N, na, Rd = 128, 360, 30.0
    nd = int(math.ceil(math.hypot(N, N))) + 4
    t = tomo.detector(nd)
    g = np.tile(2.0 * np.sqrt(np.maximum(Rd * Rd - t * t, 0.0)), (na, 1))
    b = lp.backproject_logpolar(g, N, N)
    m = lp.mesh(N, N, na, nd)
    r0 = m.R * math.exp(m.rho0)
    row = N // 2
    y = row + 0.5 - N / 2.0

    def Bg(r):
        def fn(th):
            u = r * math.cos(th)
            return 2.0 * math.sqrt(max(Rd * Rd - u * u, 0.0)) if abs(u) >= r0 else 0.0
        pts = [math.acos(min(1.0, r0 / r)), math.pi - math.acos(min(1.0, r0 / r))]
        if r > Rd:
            pts += [math.acos(Rd / r), math.pi - math.acos(Rd / r)]
        return quad(fn, 0.0, math.pi, points=sorted(pts), limit=400)[0]

    x = np.arange(N) + 0.5 - N / 2.0
    prof = np.array([Bg(math.hypot(xx, y)) for xx in x])
    assert np.max(np.abs(b[row] - prof)) <= 0.01 * 2 * math.pi * Rd
