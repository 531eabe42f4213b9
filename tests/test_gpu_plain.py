"""GPU parity of the plain 2D solver against the FP64 oracle.

Tolerances: the iterate after a fixed number of iterations must match the
oracle to a relative L2 error of 1e-5 (float32 device arithmetic against
float64); integer-valued results (iteration counts, bitwise tile invariance)
are compared exactly.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1608_03589_amd as tv
from scenes import WORKLOADS, scene2d
from stopcheck import assert_stop_guard

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
S2 = 1.0 / math.sqrt(8.0)
RTOL = 1e-5
LAM32 = float(np.float32(0.1))   # the device holds lam in float32


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) /
                 max(np.linalg.norm(b), 1e-300))


def gpu_fixed(g32, n, lam=0.1, tile=None, use_graph=-1):
    if tile is not None:
        tv.set_tile(g32.shape, *tile)
    s = tv.PlainSolver(g32.shape, DEV)
    s.solve(torch.from_numpy(g32).to(DEV), lam=lam, tau=S2, sigma=S2,
            max_iter=n, check_every=0, gap_tol=-1.0, use_graph=use_graph)
    f, p = s.state()
    torch.cuda.synchronize()
    return f.cpu().numpy(), p.cpu().numpy(), s


def device_state(g32, k, lam, theta=1.0):
    """(f^k, p^k) of the device's fixed-coefficient iteration from g."""
    s = tv.PlainSolver(g32.shape, DEV)
    s.init(torch.from_numpy(g32).to(DEV))
    if k > 0:
        s.step(k, lam, None, None, theta)
    f, p = s.state()
    return f.cpu().numpy(), p.cpu().numpy()


def scene32(H, W, n_shapes, noise, seed):
    _, g = scene2d(H, W, n_shapes, noise, seed)
    return g.astype(np.float32)


def test_parity_denoise_256_1000_iterations():
    w = WORKLOADS["denoise_256"]
    g32 = scene32(w["H"], w["W"], w["n_shapes"], w["noise"], w["seed"])
    print(f"case: denoise_256 fixed {w['iters']} iterations", flush=True)
    f, p, _ = gpu_fixed(g32, w["iters"], w["lam"])
    f_ref, _, p_ref = oracle.run_fixed(g32.astype(np.float64), w["lam"], S2,
                                       S2, w["iters"])
    ef, ep = rel(f, f_ref), rel(p, p_ref)
    print(f"rel L2 f = {ef:.3e}, p = {ep:.3e}")
    assert ef <= RTOL
    assert ep <= 10 * RTOL


@pytest.mark.parametrize("shape,tile", [
    ((1, 1), None), ((1, 7), None), ((7, 1), None), ((5, 3), (2, 1, 1)),
    ((37, 301), (3, 2, 0)), ((130, 513), (7, 4, 1)), ((300, 260), (64, 1, 0)),
    ((64, 1029), (5, 4, 0)), ((2, 2), (1, 1, 1)), ((41, 1100), (4, 2, 1)),
])
def test_parity_ragged_shapes(shape, tile):
    print(f"case: ragged {shape} tile {tile}", flush=True)
    g32 = scene32(shape[0], shape[1], 6, 0.1, 100 + shape[0] * 7 + shape[1])
    n = 60
    f, p, _ = gpu_fixed(g32, n, 0.1, tile)
    f_ref, _, p_ref = oracle.run_fixed(g32.astype(np.float64), 0.1, S2, S2, n)
    assert rel(f, f_ref) <= RTOL
    if np.linalg.norm(p_ref) > 0:
        assert rel(p, p_ref) <= 10 * RTOL
    else:
        assert np.all(p == 0)


def test_tile_invariance_bitwise():
    """Halo values are recomputed with the owner's arithmetic, so every tile
    shape gives bit-identical iterates."""
    shape = (300, 517)
    g32 = scene32(*shape, 10, 0.1, 77)
    outs = []
    for tile in [(1, 1, 1), (3, 2, 0), (8, 4, 1), (64, 4, 0), (300, 1, 1),
                 (7, 2, 0)]:
        print(f"case: tile {tile}", flush=True)
        f, p, _ = gpu_fixed(g32, 40, 0.1, tile)
        outs.append((f, p))
    for f, p in outs[1:]:
        assert np.array_equal(f, outs[0][0])
        assert np.array_equal(p, outs[0][1])


def test_resume_and_graph_replay_bitwise():
    shape = (200, 333)
    g32 = scene32(*shape, 10, 0.1, 78)
    gt = torch.from_numpy(g32).to(DEV)
    a = tv.PlainSolver(shape, DEV)
    a.init(gt)
    a.step(25, 0.1, S2, S2)
    a.step(25, 0.1, S2, S2)
    assert a.iteration() == 50
    fa, pa = a.state()
    b = tv.PlainSolver(shape, DEV)
    b.init(gt)
    b.step(50, 0.1, S2, S2)
    fb, pb = b.state()
    assert torch.equal(fa, fb) and torch.equal(pa, pb)
    f1, r1 = tv.PlainSolver(shape, DEV).solve(gt, 0.1, max_iter=300,
                                              check_every=10, gap_tol=-1.0,
                                              use_graph=1)
    f0, r0 = tv.PlainSolver(shape, DEV).solve(gt, 0.1, max_iter=300,
                                              check_every=10, gap_tol=-1.0,
                                              use_graph=0)
    assert torch.equal(f1, f0)
    assert r1.iters == r0.iters == 300 and r1.gap == r0.gap


@pytest.mark.parametrize("depth", [5, 1])
def test_steps_with_changing_coefficients(depth):
    """Coefficients that change between step calls, with step lengths that cut
    passes short.  The sweep forms the extrapolation of f^k from f^k, g, p^k
    and the step tau that produced f^k (kept in the device state), so the
    first pass after a change must use the previous call's tau; the oracle
    iterates the same schedule with the textbook extrapolation."""
    shape = (70, 301)
    g32 = scene32(*shape, 10, 0.1, 79)
    sched = [(7, 0.1, 0.30, 0.30), (3, 0.05, 0.20, 0.45), (11, 0.2, 0.35, 0.25),
             (5, 0.1, 0.25, 0.40)]
    print(f"case: depth {depth} shape {shape}", flush=True)
    tv.set_pass_depth(depth)
    try:
        s = tv.PlainSolver(shape, DEV)
        s.init(torch.from_numpy(g32).to(DEV))
        for n, lam, tau, sig in sched:
            s.step(n, lam, tau, sig)
        f, p = s.state()
        torch.cuda.synchronize()
    finally:
        tv.set_blocking(True)
    assert s.iteration() == sum(c[0] for c in sched)
    g = g32.astype(np.float64)
    fo, fprev, po = oracle.init_state(g)
    for n, lam, tau, sig in sched:
        lam, tau, sig = (float(np.float32(v)) for v in (lam, tau, sig))
        for _ in range(n):
            fn, po = oracle.pdhg_iteration(fo, fprev, po, g, lam, tau, sig)
            fprev, fo = fo, fn
    assert rel(f.cpu().numpy(), fo) < RTOL
    assert rel(p.cpu().numpy(), po) < 1e-4


def test_solve_stops_like_oracle():
    w = WORKLOADS["denoise_256"]
    g32 = scene32(w["H"], w["W"], w["n_shapes"], w["noise"], w["seed"])
    g64 = g32.astype(np.float64)
    ref = oracle.solve(g64, w["lam"], S2, S2, max_iter=w["iters"], check_every=10,
                       gap_tol=1e-4, return_history=True)
    for use_graph in (0, 1):
        print(f"case: stopping solve use_graph={use_graph}", flush=True)
        f, res = tv.PlainSolver(g32.shape, DEV).solve(
            torch.from_numpy(g32).to(DEV), w["lam"], max_iter=w["iters"],
            check_every=10, gap_tol=1e-4, use_graph=use_graph)
        assert res.converged and ref["converged"]
        if use_graph == 0:
            assert_stop_guard(ref, g64, LAM32, 1e-4, 10,
                              lambda k: device_state(g32, k, w["lam"]))
        assert res.iters == ref["iters"]
        hist = {h[0]: h for h in ref["history"]}
        _, P_ref, _, gap_ref = hist[res.iters]
        assert abs(res.primal - P_ref) <= 1e-5 * P_ref
        assert abs(res.gap - gap_ref) <= 1e-2 * gap_ref
        f_ref, _, _ = oracle.run_fixed(g64, w["lam"], S2, S2, res.iters)
        assert rel(f.cpu().numpy(), f_ref) <= RTOL


def test_energy_gap_of_device_state_matches_oracle():
    shape = (173, 289)
    g32 = scene32(*shape, 12, 0.1, 79)
    s = tv.PlainSolver(shape, DEV)
    s.init(torch.from_numpy(g32).to(DEV))
    s.step(70, 0.1, S2, S2)
    f, p = s.state()
    P, D, gap = s.energy_gap(0.1)
    Pr, Dr, gr = oracle.energy_gap(f.cpu().numpy().astype(np.float64),
                                   p.cpu().numpy().astype(np.float64),
                                   g32.astype(np.float64), LAM32)
    assert abs(P - Pr) <= 1e-10 * abs(Pr)
    assert abs(gap - gr) <= 1e-10 * abs(Pr)
    assert abs(D - Dr) <= 1e-10 * abs(Pr)


def test_fused_gap_equals_standalone_gap():
    """A solve that stops at a check reports the gap reduced inside the sweep;
    re-evaluating the frozen pair with the standalone kernel (float64 terms)
    gives the same value up to the rounding of the sweep's float32 per-pixel
    terms: a few units in the last place of each of 1/2 r^2, lam |grad f| and
    <grad f, p> (|<grad f, p>| <= lam |grad f|), so at most 4 * 2^-24 (P +
    lam TV) <= 5e-7 P (observed about 3e-9 P)."""
    shape = (257, 300)
    g32 = scene32(*shape, 12, 0.1, 80)
    s = tv.PlainSolver(shape, DEV)
    f, res = s.solve(torch.from_numpy(g32).to(DEV), 0.1, max_iter=2000,
                     check_every=10, gap_tol=1e-2)
    assert res.converged and res.iters > 0
    assert s.iteration() == res.iters
    P, D, gap = s.energy_gap(0.1)
    assert abs(P - res.primal) <= 5e-7 * P
    assert abs(gap - res.gap) <= 5e-7 * P
    assert torch.equal(f, s.state(with_dual=False))


def _crop_bounds(c, r, n):
    return max(c - r, 0), min(c + r + 1, n)


def test_full_size_4096_sampled_windows():
    """At 4096 x 4096 in the default launch configuration: after N
    iterations a pixel depends only on data within N + 1 pixels, so the
    oracle on a crop with a margin of N + 2 (or the true image edge)
    reproduces sampled windows of the full-size run exactly."""
    w = WORKLOADS["denoise_4096"]
    g32 = scene32(w["H"], w["W"], w["n_shapes"], w["noise"], w["seed"])
    N = 12
    print(f"case: 4096 sampled windows, tile {tv.get_tile(g32.shape)}", flush=True)
    f, p, _ = gpu_fixed(g32, N, w["lam"])
    th = tv.get_tile(g32.shape)[0]
    H, W = g32.shape
    rng = np.random.default_rng(7)
    centres = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, 255),
               (H // 2, 256), (th - 1, 1000), (th, 1000), (5 * th, 511),
               (H - 1, 2047), (17, W - 1), (100, 239), (100, 240), (3 * th, 480)]
    centres += [tuple(rng.integers(0, [H, W])) for _ in range(6)]
    m = N + 2
    for (cy, cx) in centres:
        y0, y1 = _crop_bounds(cy, m + 3, H)
        x0, x1 = _crop_bounds(cx, m + 3, W)
        crop = g32[y0:y1, x0:x1].astype(np.float64)
        fr, _, pr = oracle.run_fixed(crop, w["lam"], S2, S2, N)
        # compare the part of the window that is at least m away from any
        # crop edge that is not a true image edge
        iy0 = 0 if y0 == 0 else m
        iy1 = (y1 - y0) if y1 == H else (y1 - y0) - m
        ix0 = 0 if x0 == 0 else m
        ix1 = (x1 - x0) if x1 == W else (x1 - x0) - m
        got = f[y0 + iy0:y0 + iy1, x0 + ix0:x0 + ix1]
        exp = fr[iy0:iy1, ix0:ix1]
        assert got.size > 0
        assert rel(got, exp) <= RTOL, (cy, cx)
        gotp = p[:, y0 + iy0:y0 + iy1, x0 + ix0:x0 + ix1]
        expp = pr[:, iy0:iy1, ix0:ix1]
        assert np.max(np.abs(gotp - expp)) <= 1e-5 * max(w["lam"], 1e-12), (cy, cx)


def test_full_size_4096_properties():
    """The benchmarked run itself (2000 iterations, gap every 10): mass is
    conserved, the dual stays feasible, the gap is non-negative, and the
    gap of the final pair agrees with the oracle's evaluation of it."""
    w = WORKLOADS["denoise_4096"]
    g32 = scene32(w["H"], w["W"], w["n_shapes"], w["noise"], w["seed"])
    s = tv.PlainSolver(g32.shape, DEV)
    gt = torch.from_numpy(g32).to(DEV)
    print("case: 4096 full run properties", flush=True)
    f, res = s.solve(gt, w["lam"], max_iter=w["iters"], check_every=10,
                     gap_tol=-1.0)
    assert res.iters == w["iters"] and not res.converged
    fd, pd = s.state()
    fn = fd.double().cpu().numpy()
    pn = pd.double().cpu().numpy()
    assert abs(fn.sum() - g32.astype(np.float64).sum()) <= 1e-6 * np.abs(g32).sum()
    nrm = np.sqrt((pn ** 2).sum(axis=0))
    assert nrm.max() <= w["lam"] * (1 + 1e-6)
    assert res.gap >= 0 and res.gap < 1e-2 * res.primal
    Pr, Dr, gr = oracle.energy_gap(fn, pn, g32.astype(np.float64),
                                   float(np.float32(w["lam"])))
    assert abs(res.primal - Pr) <= 1e-9 * Pr
    assert abs(res.gap - gr) <= 1e-9 * Pr


def test_autotune_choice_and_cache_roundtrip(tmp_path):
    shape = (512, 700)
    cache = str(tmp_path / "tiles.txt")
    print("case: autotune 512x700", flush=True)
    (th, wpb, order), us = tv.autotune(shape, DEV, cache)
    assert us > 0 and th >= 1 and wpb in (1, 2, 4) and order in (0, 1)
    assert tv.get_tile(shape) == (th, wpb, order)
    tv.set_tile(shape, 5, 1, 1)
    assert tv.tune_load(cache) == 1
    assert tv.get_tile(shape) == (th, wpb, order)
    g32 = scene32(*shape, 12, 0.1, 81)
    f, _, _ = gpu_fixed(g32, 30, 0.1)
    f_ref, _, _ = oracle.run_fixed(g32.astype(np.float64), 0.1, S2, S2, 30)
    assert rel(f, f_ref) <= RTOL


@pytest.mark.parametrize("shape,tile", [
    ((300, 517), (1, 1, 1)), ((300, 517), (2, 2, 0)), ((300, 517), (3, 4, 0)),
    ((300, 517), (64, 4, 0)), ((37, 1030), (5, 2, 1)), ((1, 9), (1, 1, 0)),
    ((2, 300), (1, 4, 0)), ((3, 3), (2, 1, 1)), ((513, 257), (300, 1, 0)),
    ((20, 248), (4, 4, 0)), ((21, 249), (7, 2, 1)), ((9, 744), (2, 4, 0)),
    ((70, 497), (16, 1, 0)), ((6, 4), (1, 1, 0)), ((11, 240), (3, 4, 0)),
    ((12, 241), (2, 2, 1)), ((31, 480), (9, 4, 0)),
])
def test_blocked_passes_are_bitwise_equal(shape, tile):
    """Temporal blocking of every depth (1 to 6 iterations per launch)
    reproduces one-iteration passes bit for bit, for iteration counts that do
    and do not divide into whole passes and for stopping solves whose checks
    cut passes short."""
    g32 = scene32(*shape, 10, 0.1, 90 + shape[0])
    tv.set_tile(shape, *tile)
    out = {}
    try:
        for depth in (1, 2, 3, 4, 5, 6):
            print(f"case: depth {depth} shape {shape} tile {tile}", flush=True)
            tv.set_pass_depth(depth)
            for n in (7, 20):
                f, p, _ = gpu_fixed(g32, n, 0.1)
                out[(depth, n)] = (f, p)
            s = tv.PlainSolver(shape, DEV)
            for ce in (10, 7, 3):
                fs, rs = s.solve(torch.from_numpy(g32).to(DEV), 0.1,
                                 max_iter=400, check_every=ce, gap_tol=2e-3)
                out[(depth, "solve", ce)] = (fs.cpu().numpy(), rs.iters)
    finally:
        tv.set_blocking(True)
    for depth in (2, 3, 4, 5, 6):
        for n in (7, 20):
            assert np.array_equal(out[(depth, n)][0], out[(1, n)][0]), (depth, n)
            assert np.array_equal(out[(depth, n)][1], out[(1, n)][1]), (depth, n)
        for ce in (10, 7, 3):
            a, b = out[(depth, "solve", ce)], out[(1, "solve", ce)]
            assert a[1] == b[1] and np.array_equal(a[0], b[0]), (depth, ce)


@pytest.mark.parametrize("seed,lam", [(15, 0.3), (16, 0.1)])
def test_solution_level_against_the_minimiser(seed, lam):
    """Solution-level parity.  E is 1-strongly convex, so for any feasible
    pair (f, p) the gap bounds the distance to the unique minimiser:
    0.5 ||f - u*||^2 <= P(f) - P(u*) <= gap(f, p).  The GPU's iterate after
    many iterations therefore lies within sqrt(2 gap) of u*, which a generic
    constrained optimiser finds on the explicit dual problem of an 8x8 image
    (to about 2e-6 per pixel); the device's own gap of its float32 pair
    enters the bound."""
    import pins
    rng = np.random.default_rng(seed)
    g32 = rng.normal(size=(8, 8)).astype(np.float32)
    f_bf, _ = pins.tv2d_bruteforce(g32.astype(np.float64), lam)
    print(f"case: minimiser 8x8 seed {seed} lam {lam}", flush=True)
    f, res = tv.PlainSolver(g32.shape, DEV).solve(
        torch.from_numpy(g32).to(DEV), lam, max_iter=60000, check_every=100,
        gap_tol=-1.0)
    d = float(np.linalg.norm(f.cpu().numpy().astype(np.float64) - f_bf))
    bound = math.sqrt(2.0 * max(res.gap, 0.0)) + 2e-6 * 8
    print(f"distance {d:.3e}, gap {res.gap:.3e}, bound {bound:.3e}")
    assert res.gap >= -1e-9 * res.primal
    assert d <= bound
    assert d <= 1e-4 * np.linalg.norm(f_bf)   # the bound is not vacuous here


def test_stream_copy_copies():
    # the plain copy kernel that calibrates byte counters copies exactly
    import ctypes
    from paper_1608_03589_amd import _lib
    n = 1 << 20
    a = torch.rand(n, device=DEV)
    b = torch.zeros_like(a)
    print("case: plain copy of 2^20 floats", flush=True)
    _lib.call("tvpd_stream_copy", ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
              ctypes.c_int64(n), ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
