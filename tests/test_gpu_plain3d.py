"""GPU parity of the plain 3D solver (fused z-marching sweep) against the
FP64 oracle, and its invariances.

Tolerances as in 2D: relative L2 1e-5 for the iterate after a fixed number
of iterations, 1e-4 for the dual; tile invariance and agreement with the
unrolled forward are bitwise (the per-voxel arithmetic is shared).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1608_03589_amd as tv
from scenes import scene3d
from stopcheck import assert_stop_guard

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
S3 = 1.0 / math.sqrt(12.0)
RTOL = 1e-5
LAM32 = float(np.float32(0.1))


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) /
                 max(np.linalg.norm(b), 1e-300))


def vol32(D, H, W, seed, n_shapes=12, noise=0.1):
    _, g = scene3d(D, H, W, n_shapes, noise, seed)
    return g.astype(np.float32)


def gpu_fixed(g32, n, lam=0.1, tile=None):
    if tile is not None:
        tv.set_tile3d(g32.shape, *tile)
    s = tv.PlainSolver(g32.shape, DEV)
    s.solve(torch.from_numpy(g32).to(DEV), lam=lam, tau=S3, sigma=S3,
            max_iter=n, check_every=0, gap_tol=-1.0, use_graph=0)
    f, p = s.state()
    torch.cuda.synchronize()
    return f.cpu().numpy(), p.cpu().numpy(), s


@pytest.mark.parametrize("shape,n", [((20, 37, 45), 60), ((9, 14, 300), 40),
                                     ((33, 24, 16), 80)])
def test_parity_3d_fixed_iterations(shape, n):
    g32 = vol32(*shape, seed=sum(shape))
    print(f"case: 3D parity {shape} n={n}", flush=True)
    f, p, _ = gpu_fixed(g32, n)
    f_ref, _, p_ref = oracle.run_fixed(g32.astype(np.float64), 0.1, S3, S3, n)
    ef, ep = rel(f, f_ref), rel(p, p_ref)
    print(f"rel L2 f = {ef:.3e}, p = {ep:.3e}")
    assert ef <= RTOL
    assert ep <= 10 * RTOL


TILES = [(2, 1, 1), (4, 3, 2), (2, 7, 4), (4, 64, 4), (2, 2, 2), (4, 1, 1)]


@pytest.mark.parametrize("shape", [(13, 11, 517), (8, 9, 64), (17, 6, 259),
                                   (1, 5, 7), (5, 1, 300)])
def test_tiles_do_not_change_iterates(shape):
    g32 = vol32(*shape, seed=7 + shape[2])
    ref = None
    for t in TILES:
        print(f"case: 3D tile {t} shape {shape}", flush=True)
        f, p, _ = gpu_fixed(g32, 9, tile=t)
        if ref is None:
            ref = (f, p)
        else:
            assert np.array_equal(f, ref[0]), t
            assert np.array_equal(p, ref[1]), t
    f_ref, _, _ = oracle.run_fixed(g32.astype(np.float64), 0.1, S3, S3, 9)
    assert rel(ref[0], f_ref) <= RTOL


def test_energy_gap_and_fused_gap_match_oracle():
    g32 = vol32(18, 21, 40, seed=31)
    gt = torch.from_numpy(g32).to(DEV)
    s = tv.PlainSolver(g32.shape, DEV)
    s.init(gt)
    s.step(10, lam=0.1)
    P10, _, gap10 = s.energy_gap(0.1)
    s.step(10, lam=0.1)
    P, D, gap = s.energy_gap(0.1)
    f, p = s.state()
    Pr, Dr, gapr = oracle.energy_gap(f.cpu().numpy().astype(np.float64),
                                     p.cpu().numpy().astype(np.float64),
                                     g32.astype(np.float64), LAM32)
    assert abs(P - Pr) <= 1e-10 * Pr
    assert abs(gap - gapr) <= 1e-10 * Pr
    assert abs(D - Dr) <= 1e-10 * Pr
    # the gap fused into the sweep: a tolerance the k = 20 pair meets and the
    # k = 10 pair does not stops the solve at k = 20 with the same gap
    tol = gap / P * (1 + 1e-9)
    assert gap10 / P10 > tol
    f20, r = s.solve(gt, lam=0.1, max_iter=40, check_every=10, gap_tol=tol)
    assert r.converged and r.iters == 20
    assert abs(r.gap - gap) <= 1e-9 * P and abs(r.primal - P) <= 1e-9 * P
    assert np.array_equal(f20.cpu().numpy(), f.cpu().numpy())


def test_stopping_matches_oracle():
    g32 = vol32(16, 20, 24, seed=5)
    _, r = tv.PlainSolver(g32.shape, DEV).solve(
        torch.from_numpy(g32).to(DEV), lam=0.1, max_iter=400, check_every=10,
        gap_tol=1e-3)
    g64 = g32.astype(np.float64)
    ref = oracle.solve(g64, 0.1, S3, S3, max_iter=400, check_every=10,
                       gap_tol=1e-3, return_history=True)
    assert r.converged and ref["converged"]

    def state_at(k):
        s = tv.PlainSolver(g32.shape, DEV)
        s.init(torch.from_numpy(g32).to(DEV))
        if k > 0:
            s.step(k, 0.1)
        f, p = s.state()
        return f.cpu().numpy(), p.cpu().numpy()

    assert_stop_guard(ref, g64, LAM32, 1e-3, 10, state_at)
    assert r.iters == ref["iters"]


def test_plain_equals_unrolled_forward():
    """Constant coefficients: the unrolled 3D forward and the plain solver
    run the same per-voxel arithmetic, so f^K agrees bit for bit."""
    g32 = vol32(12, 19, 270, seed=11)
    K = 12
    f, _, _ = gpu_fixed(g32, K)
    u = tv.UnrolledSolver((1,) + g32.shape, K, ckpt_every=K, device=DEV)
    coeffs = torch.tensor([[0.1, S3, S3]] * K, dtype=torch.float32, device=DEV)
    fu = u.forward(torch.from_numpy(g32).to(DEV)[None], coeffs)
    assert np.array_equal(fu[0].cpu().numpy(), f)


def test_resume_and_graph_replay_are_bitwise():
    g32 = vol32(10, 12, 40, seed=3)
    gt = torch.from_numpy(g32).to(DEV)
    a = tv.PlainSolver(g32.shape, DEV)
    a.init(gt)
    a.step(7, lam=0.1)
    a.step(13, lam=0.1)
    fa = a.state(with_dual=False).cpu().numpy()
    b = tv.PlainSolver(g32.shape, DEV)
    fb, _ = b.solve(gt, lam=0.1, max_iter=20, check_every=0, gap_tol=-1.0,
                    use_graph=1)
    assert np.array_equal(fa, fb.cpu().numpy())


def _crop_bounds(c, r, n):
    return max(c - r, 0), min(c + r + 1, n)


def test_full_size_256cube_sampled_windows():
    """256^3 in the default launch configuration: after N iterations a voxel
    depends only on data within N + 1 voxels, so the oracle on a crop with
    a margin of N + 2 (or the true volume edge) reproduces sampled windows
    of the full-size run."""
    from scenes import WORKLOADS
    w = WORKLOADS["unrolled_256cube"]
    _, g = scene3d(w["D"], w["H"], w["W"], w["n_shapes"], w["noise"], w["seed"])
    g32 = g.astype(np.float32)
    del g
    N = 10
    th, tz, wpb = tv.get_tile3d(g32.shape)
    print(f"case: 256^3 sampled windows, tile {(th, tz, wpb)}", flush=True)
    f, p, _ = gpu_fixed(g32, N)
    D, H, W = g32.shape
    rng = np.random.default_rng(8)
    centres = [(0, 0, 0), (D - 1, H - 1, W - 1), (0, H - 1, 0), (tz - 1, th - 1, 100),
               (tz, th, 100), (2 * tz, 3 * th - 1, W - 1), (D // 2, H // 2, 0)]
    centres += [tuple(rng.integers(0, [D, H, W])) for _ in range(4)]
    m = N + 2
    for c in centres:
        b = [_crop_bounds(ci, m + 2, n) for ci, n in zip(c, (D, H, W))]
        crop = g32[b[0][0]:b[0][1], b[1][0]:b[1][1], b[2][0]:b[2][1]].astype(np.float64)
        fr, _, pr = oracle.run_fixed(crop, 0.1, S3, S3, N)
        sl_g, sl_c = [], []
        for (lo, hi), n in zip(b, (D, H, W)):
            i0 = 0 if lo == 0 else m
            i1 = (hi - lo) if hi == n else (hi - lo) - m
            sl_g.append(slice(lo + i0, lo + i1))
            sl_c.append(slice(i0, i1))
        got = f[tuple(sl_g)]
        exp = fr[tuple(sl_c)]
        assert got.size > 0
        assert rel(got, exp) <= RTOL, c
        gp = p[(slice(None),) + tuple(sl_g)]
        ep = pr[(slice(None),) + tuple(sl_c)]
        assert np.max(np.abs(gp - ep)) <= 1e-5 * 0.1, c


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 1, 1), (1, 1, 300), (1, 3, 1),
                                   (3, 2, 5), (70, 1, 1)])
def test_degenerate_3d_shapes(shape):
    """Volumes with unit axes (the forward difference along them vanishes)
    and a single voxel (the iterate stays g) match the oracle."""
    g32 = vol32(*shape, seed=3 + sum(shape), n_shapes=3) if min(shape) > 4 else \
        np.random.default_rng(sum(shape)).uniform(0, 1, shape).astype(np.float32)
    print(f"case: degenerate 3D {shape}", flush=True)
    f, p, _ = gpu_fixed(g32, 17)
    fr, _, pr = oracle.run_fixed(g32.astype(np.float64), 0.1, S3, S3, 17)
    assert rel(f, fr) <= RTOL
    assert np.max(np.abs(p - pr)) <= 1e-6
