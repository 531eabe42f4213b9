"""GPU parity of the tomographic data term against the FP64 oracle.

Operators: the projection A and the backprojection A^T of the HIP path are
compared with the oracle's element by element on seeded inputs (several
projection blocks and backprojection tiles, ragged edges, detectors narrower
and wider than the image, angles on the 45-degree switch between row and
column walks), to a relative L2 error of 1e-5 (float32 sums of at most
3 * max(ny, nx) hat-weighted terms per bin, or n_angles interpolated terms per
pixel, against float64) and a max error of 1e-5 of the largest entry.  At the
full 2048^2 x 1000 x 2048 size: sampled entries, the mass of every projection
and adjointness.

Iteration: f, r and p after a fixed number of TV and Tikhonov iterations
match the oracle to a relative L2 error of 1e-5 (f, r) and 1e-4 (p, whose
small entries carry the cancellation of the gradient); calls that split the
iterations agree bit for bit with one call.
"""
import math

import numpy as np
import pytest
import torch

import paper_1608_03589_amd as tv
import scenes
from oracle import tomo

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
RTOL = 1e-5


def rel(a, b):
    a = np.asarray(a, np.complex128 if np.iscomplexobj(a) else np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    a = np.asarray(a, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


GEOMS = [
    (64, 64, 48, 92),        # detector covers the image
    (37, 53, 30, 70),        # non-square
    (300, 200, 100, 400),    # several blocks and tiles, ragged
    (40, 40, 33, 30),        # detector narrower than the image
    (20, 75, 4, 81),         # 0, 45, 90, 135 degrees
    (33, 129, 70, 150),      # three angle chunks, ragged
    (200, 200, 400, 300),    # many angles, fine angle step
    (1, 1, 5, 3),
    (1, 17, 3, 1),
    (9, 1, 1, 12),
]


@pytest.mark.parametrize("H,W,na,nd", GEOMS)
def test_projection_and_backprojection_match_the_oracle(H, W, na, nd):
    print(f"case: operators {H}x{W} angles {na} bins {nd}", flush=True)
    rng = np.random.default_rng(H * 1000 + W)
    f = rng.uniform(-1.0, 2.0, size=(H, W)).astype(np.float32)
    s = rng.normal(size=(na, nd)).astype(np.float32)
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    A = solver.radon(to_dev(f)).cpu().numpy()
    B = solver.backproject(to_dev(s)).cpu().numpy()
    A_ref = tomo.project(f.astype(np.float64), na, nd)
    B_ref = tomo.backproject(s.astype(np.float64), H, W)
    print(f"A rel {rel(A, A_ref):.2e} max {maxrel(A, A_ref):.2e}; "
          f"A^T rel {rel(B, B_ref):.2e} max {maxrel(B, B_ref):.2e}")
    assert rel(A, A_ref) <= RTOL and maxrel(A, A_ref) <= RTOL
    assert rel(B, B_ref) <= RTOL and maxrel(B, B_ref) <= RTOL


@pytest.mark.parametrize("H,W,na,nd", GEOMS + [(512, 300, 37, 700), (256, 256, 250, 64),
                                         (2048, 2048, 1000, 2048)])
def test_projection_staging_is_bitwise_neutral(H, W, na, nd):
    # blocks of 8 angles staging image rows in LDS read the same three
    # columns per lane and row as the direct gather, so A f is the same bit
    # for bit (and so are the iteration's dual update and residual)
    print(f"case: staged vs direct A {H}x{W} angles {na} bins {nd}", flush=True)
    rng = np.random.default_rng(H + 7 * W + na)
    f = rng.uniform(-1.0, 2.0, size=(H, W)).astype(np.float32)
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    fd = to_dev(f)
    try:
        tv.set_projection_staging(True)
        a1 = solver.radon(fd).cpu().numpy()
        tv.set_projection_staging(False)
        a0 = solver.radon(fd).cpu().numpy()
    finally:
        tv.set_projection_staging(True)
    assert np.array_equal(a1, a0)
    assert np.all(np.isfinite(a1))


def _full_size():
    w = scenes.WORKLOADS["tomo_2048x1000"]
    return w, w["H"], w["W"], w["n_angles"], w["n_det"]


def test_full_size_operators_sampled():
    w, H, W, na, nd = _full_size()
    print(f"case: operators {H}x{W} angles {na} bins {nd} (sampled)", flush=True)
    img, _, g = scenes.tomo_scene(H, W, na, nd, w["n_ellipses"], w["noise"], w["seed"])
    f32 = img.astype(np.float32)
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    A = solver.radon(to_dev(f32)).cpu().numpy().astype(np.float64)
    # every pixel of the phantom projects inside the detector: each
    # projection carries the image's mass
    mass = float(np.sum(f32.astype(np.float64)))
    assert np.max(np.abs(A.sum(axis=1) - mass)) <= 1e-5 * mass
    rng = np.random.default_rng(7)
    ks = np.concatenate(([0, na // 4, na // 2, 3 * na // 4, na - 1],
                         rng.integers(0, na, 27)))
    iis = np.concatenate(([nd // 2] * 5, rng.integers(nd // 4, 3 * nd // 4, 27)))
    ref = tomo.project_at(f32.astype(np.float64), na, nd, ks, iis)
    got = A[ks, iis]
    assert np.max(np.abs(got - ref)) <= RTOL * np.max(np.abs(A))
    s32 = g.astype(np.float32)
    B = solver.backproject(to_dev(s32)).cpu().numpy().astype(np.float64)
    rows = np.concatenate(([0, 0, H - 1, H - 1, H // 2, 31, 32, 63],
                           rng.integers(0, H, 24)))
    cols = np.concatenate(([0, W - 1, 0, W - 1, W // 2, 63, 64, 127],
                           rng.integers(0, W, 24)))
    ref = tomo.backproject_at(s32.astype(np.float64), H, W, rows, cols)
    assert np.max(np.abs(B[rows, cols] - ref)) <= RTOL * np.max(np.abs(B))
    # adjointness of the two device operators, in float64 dot products
    lhs = float(np.sum(A * s32.astype(np.float64)))
    rhs = float(np.sum(f32.astype(np.float64) * B))
    assert abs(lhs - rhs) <= RTOL * abs(lhs)


def _problem(H, W, na, nd, seed):
    _, _, g = scenes.tomo_scene(H, W, na, nd, n_ellipses=8, noise=0.02, seed=seed)
    return g.astype(np.float32)


def f32(x):
    return float(np.float32(x))


@pytest.mark.parametrize("reg,lam,H,W,na,nd,n", [
    ("tv", 2.0, 64, 64, 48, 92, 60), ("tikhonov", 3.0, 64, 64, 48, 92, 60),
    ("tv", 0.0, 64, 64, 48, 92, 60), ("tv", 1.0, 300, 200, 100, 400, 6),
    ("tikhonov", 1.0, 45, 130, 37, 120, 20)])
def test_iterations_match_the_oracle(reg, lam, H, W, na, nd, n):
    print(f"case: tomo {reg} lam {lam} {H}x{W} {na}x{nd} {n} iterations", flush=True)
    g = _problem(H, W, na, nd, 11)
    L2 = tomo.opnorm_sq(H, W, na, nd, 60)
    tau, sr, sp = tv.default_steps(L2, reg)
    tau, sr, sp, lam32 = f32(tau), f32(sr), f32(sp), f32(lam)
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    solver.init()
    solver.step(to_dev(g), n, lam32, tau, sr, sp, reg=reg)
    f, r, p, k = solver.state()
    assert k == n
    st = tomo.run(g.astype(np.float64), H, W, lam32, tau, sr, sp, n, reg=reg)
    ef, er = rel(f.cpu().numpy(), st["f"]), rel(r.cpu().numpy(), st["r"])
    print(f"rel L2 f {ef:.2e} r {er:.2e}")
    assert ef <= RTOL and er <= RTOL
    if reg == "tv" and lam > 0:
        ep = rel(p.cpu().numpy(), st["p"])
        print(f"rel L2 p {ep:.2e}")
        assert ep <= 10 * RTOL


def test_split_calls_equal_one_call_and_init_from_an_image():
    H, W, na, nd = 70, 90, 40, 120
    g = to_dev(_problem(H, W, na, nd, 12))
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    args = (1.5, 0.01, 0.005, 2.0)
    solver.init()
    solver.step(g, 7, *args)
    solver.step(g, 0, *args)
    solver.step(g, 6, *args)
    f1, r1, p1, k1 = solver.state()
    f2 = solver.solve(g, 13, *args)
    assert k1 == 13
    assert torch.equal(f1, f2)
    f_s, r_s, p_s, _ = solver.state()
    assert torch.equal(r1, r_s) and torch.equal(p1, p_s)
    # a warm start: f^0 = f^{-1} = f0
    f0 = torch.rand((H, W), device=DEV)
    solver.init(f0)
    solver.step(g, 3, *args)
    fw, _, _, _ = solver.state()
    st = tomo.run(g.cpu().numpy().astype(np.float64), H, W, *[f32(a) for a in args], 3,
                  reg="tv", f0=f0.cpu().numpy().astype(np.float64))
    assert rel(fw.cpu().numpy(), st["f"]) <= RTOL


def test_energy_and_operator_norm():
    H, W, na, nd = 64, 48, 40, 90
    g = _problem(H, W, na, nd, 13)
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    L2 = solver.opnorm_sq(40)
    L2_ref = tomo.opnorm_sq(H, W, na, nd, 40)
    assert abs(L2 - L2_ref) <= RTOL * L2_ref
    tau, sr, sp = tv.default_steps(L2, "tv")
    gd = to_dev(g)
    solver.init()
    for reg, lam in (("tv", 1.0), ("tikhonov", 2.0)):
        solver.step(gd, 25, lam, tau, sr, sp, reg="tv")
        f, _, _, _ = solver.state()
        e = solver.energy(gd, lam, reg)
        e_ref = tomo.energy(f.cpu().numpy().astype(np.float64), g.astype(np.float64),
                            f32(lam), reg)
        for a, b in zip(e, e_ref):
            assert abs(a - b) <= RTOL * abs(b)


def test_first_iteration_at_full_size():
    w, H, W, na, nd = _full_size()
    print(f"case: tomo first iteration {H}x{W} {na}x{nd}", flush=True)
    _, _, g = scenes.tomo_scene(H, W, na, nd, w["n_ellipses"], w["noise"], w["seed"])
    g32 = g.astype(np.float32)
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    tau, sr, sp = 1e-3, 5e-4, 20.0
    solver.init()
    solver.step(to_dev(g32), 1, 5.0, tau, sr, sp, reg="tv")
    f, r, p, k = solver.state()
    assert k == 1
    # from f^0 = 0: r^1 = -sr g / (1 + sr), p^1 = 0, f^1 = -tau A^T r^1
    r_ref = -f32(sr) * g32.astype(np.float64) / (1.0 + f32(sr))
    rn = r.cpu().numpy()
    assert rel(rn, r_ref) <= 1e-6
    assert torch.count_nonzero(p).item() == 0
    rng = np.random.default_rng(8)
    rows = np.concatenate(([0, H - 1, H // 2, 1000], rng.integers(0, H, 20)))
    cols = np.concatenate(([0, W - 1, W // 2, 1000], rng.integers(0, W, 20)))
    ref = -f32(tau) * tomo.backproject_at(rn.astype(np.float64), H, W, rows, cols)
    fn = f.cpu().numpy()
    assert np.max(np.abs(fn[rows, cols] - ref)) <= RTOL * np.max(np.abs(fn))


@pytest.mark.parametrize("H,W,na,nd,lam", [
    (64, 64, 48, 92, 0.0), (64, 64, 48, 92, 4.0), (37, 53, 30, 70, 1.5),
    (40, 40, 12, 2500, 0.0),     # padded length 8192: direct convolution with taps
    (33, 21, 45, 40, 1e30),      # FFT filtering, the filter ~1/lam beyond frequency 0
    (1, 1, 3, 1, 0.0)])          # padded length 2, an odd number of rays
def test_fbp_matches_the_oracle(H, W, na, nd, lam):
    print(f"case: fbp {H}x{W} angles {na} bins {nd} lam {lam}", flush=True)
    rng = np.random.default_rng(H + nd)
    s = rng.normal(size=(na, nd)).astype(np.float32)
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    f = solver.fbp(to_dev(s), lam).cpu().numpy()
    ref = tomo.fbp(s.astype(np.float64), H, W, f32(lam))
    print(f"fbp rel {rel(f, ref):.2e} max {maxrel(f, ref):.2e}")
    assert rel(f, ref) <= RTOL and maxrel(f, ref) <= RTOL


def test_fbp_at_full_size_sampled():
    w, H, W, na, nd = _full_size()
    print(f"case: fbp {H}x{W} angles {na} bins {nd} (sampled)", flush=True)
    img, clean, g = scenes.tomo_scene(H, W, na, nd, w["n_ellipses"], w["noise"], w["seed"])
    g32 = g.astype(np.float32)
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    f = solver.fbp(to_dev(g32), 0.0).cpu().numpy().astype(np.float64)
    q = tomo.fbp_filter(g32.astype(np.float64), 0.0)
    rng = np.random.default_rng(9)
    rows = np.concatenate(([0, H - 1, H // 2, 700, 1300], rng.integers(0, H, 27)))
    cols = np.concatenate(([0, W - 1, W // 2, 900, 1100], rng.integers(0, W, 27)))
    ref = (math.pi / na) * tomo.backproject_at(q, H, W, rows, cols)
    assert np.max(np.abs(f[rows, cols] - ref)) <= RTOL * np.max(np.abs(f))
    # from the exact line integrals it reconstructs the phantom (the ramp
    # filter amplifies the noise of g)
    fc = solver.fbp(to_dev(clean.astype(np.float32)), 0.0).cpu().numpy()
    assert np.linalg.norm(fc - img) / np.linalg.norm(img) < 0.15


@pytest.mark.parametrize("H,W,na,nd", [(64, 64, 48, 92), (37, 53, 30, 70), (16, 16, 7, 40),
                                       (200, 120, 100, 300)])
def test_bst_matches_the_oracle(H, W, na, nd):
    print(f"case: bst {H}x{W} angles {na} bins {nd}", flush=True)
    rng = np.random.default_rng(H * 7 + nd)
    s = rng.normal(size=(na, nd)).astype(np.float32)
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    M, Q = solver.bst_lengths()
    assert (M, Q) == tomo.bst_lengths(H, W, nd)
    spec = solver.bst_spectra(to_dev(s)).cpu().numpy()
    spec_ref = tomo.bst_spectra(s.astype(np.float64), M)
    print(f"spectra rel {rel(spec, spec_ref):.2e}")
    assert rel(spec, spec_ref) <= RTOL
    b = solver.bst(to_dev(s)).cpu().numpy()
    ref = tomo.bst(s.astype(np.float64), H, W)
    print(f"bst rel {rel(b, ref):.2e} max {maxrel(b, ref):.2e}")
    assert rel(b, ref) <= RTOL and maxrel(b, ref) <= 2 * RTOL


def test_bst_at_full_size_against_the_backprojection():
    # 2048^2 from 1000 projections: the BST equals B g = dtheta A^T g up to
    # the origin rule's constant and the bilinear interpolation in angle (at
    # the highest frequencies 1000 angles are 6.4 Cartesian cells apart; at
    # 128^2 from 400 angles, one cell, the oracle pins 0.6 %)
    w, H, W, na, nd = _full_size()
    print(f"case: bst {H}x{W} angles {na} bins {nd}", flush=True)
    _, clean, _ = scenes.tomo_scene(H, W, na, nd, w["n_ellipses"], 0.0, w["seed"])
    g = to_dev(clean.astype(np.float32))
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    b = solver.bst(g).cpu().numpy().astype(np.float64)
    ref = (math.pi / na) * solver.backproject(g).cpu().numpy().astype(np.float64)
    d = b - ref
    print(f"constant {d.mean():.4g}, rel after removing it "
          f"{np.linalg.norm(d - d.mean()) / np.linalg.norm(ref):.3e}")
    assert np.linalg.norm(d - d.mean()) / np.linalg.norm(ref) < 0.03


@pytest.mark.parametrize("lam", [0.0, 3.5, 1e30])
@pytest.mark.parametrize("H,W,na,nd", [(64, 64, 48, 92), (37, 53, 30, 70), (16, 16, 7, 40),
                                       (200, 120, 100, 300)])
def test_fbp_bst_matches_the_oracle(H, W, na, nd, lam):
    # lam = 1e30 leaves only the origin sample (K = 1 there, ~1e-27 elsewhere)
    print(f"case: fbp_bst {H}x{W} angles {na} bins {nd} lam {lam}", flush=True)
    rng = np.random.default_rng(H * 11 + nd)
    s = rng.normal(size=(na, nd)).astype(np.float32)
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    b = solver.fbp_bst(to_dev(s), lam).cpu().numpy()
    ref = tomo.fbp_bst(s.astype(np.float64), H, W, lam)
    print(f"fbp_bst rel {rel(b, ref):.2e} max {maxrel(b, ref):.2e}")
    assert rel(b, ref) <= RTOL and maxrel(b, ref) <= 2 * RTOL
    # the same workspace serves the plain BST afterwards
    bb = solver.bst(to_dev(s)).cpu().numpy()
    assert rel(bb, tomo.bst(s.astype(np.float64), H, W)) <= RTOL


def test_bst_and_fbp_bst_at_full_size_sampled():
    # 2048^2 from 1000 projections of 2048 rays: 40 pixels (corners, centre,
    # random) of both BST pipelines against the oracle's grid evaluated there
    w, H, W, na, nd = _full_size()
    print(f"case: bst/fbp_bst {H}x{W} angles {na} bins {nd} (sampled)", flush=True)
    img, clean, _ = scenes.tomo_scene(H, W, na, nd, w["n_ellipses"], 0.0, w["seed"])
    c32 = clean.astype(np.float32)
    g = to_dev(c32)
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    rng = np.random.default_rng(12)
    rows = np.concatenate(([0, 0, H - 1, H - 1, H // 2, 777, 1500, 31], rng.integers(0, H, 32)))
    cols = np.concatenate(([0, W - 1, 0, W - 1, W // 2, 1201, 300, 2000],
                           rng.integers(0, W, 32)))
    for lam in (None, 0.0, 10.0):
        out = solver.bst(g) if lam is None else solver.fbp_bst(g, lam)
        out = out.cpu().numpy().astype(np.float64)
        ref = tomo.bst_at(c32.astype(np.float64), H, W, rows, cols, lam)
        err = np.max(np.abs(out[rows, cols] - ref)) / np.max(np.abs(out))
        print(f"lam {lam}: max error / max |image| {err:.2e}", flush=True)
        assert err <= 2 * RTOL
        if lam == 0.0:
            # the mass of the projections is kept (no origin rule), and the
            # phantom is reconstructed
            assert abs(out.sum() / clean[0].sum() - 1.0) < 0.01
            on = img > 0.05
            assert abs(float(np.median(out[on] / img[on])) - 1.0) < 0.03
            assert np.linalg.norm(out - img) / np.linalg.norm(img) < 0.15
        if lam == 10.0:
            # against the FBP with the exact backprojection, up to its lost
            # mean: the difference is the bilinear interpolation in angle
            # (1000 angles are 6.4 grid cells apart at the highest frequencies)
            ex = solver.fbp(g, lam).cpu().numpy().astype(np.float64)
            d = out - ex
            r = np.linalg.norm(d - d.mean()) / np.linalg.norm(ex)
            print(f"against the exact backprojection: rel after the mean {r:.3e}")
            assert r < 0.07
