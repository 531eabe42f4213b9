"""GPU tests of the batched solver.

Every image of a batch must come out exactly as the plain solver returns it
alone: the same stopping iteration and a bit-identical iterate (the per-pixel
arithmetic is shared).  Against the FP64 oracle the usual 1e-5 relative L2
bound applies.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1608_03589_amd as tv
from scenes import WORKLOADS, batch_scenes, scene2d
from stopcheck import assert_stop_guard

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
S2 = 1.0 / math.sqrt(8.0)
LAM32 = float(np.float32(0.1))   # the device holds lam in float32

SMALL_SHAPES = [(37, 301), (130, 513), (64, 64), (5, 3), (200, 140), (1, 9),
                (257, 260)]


def small_batch(seed=300):
    imgs = []
    for i, (h, w) in enumerate(SMALL_SHAPES):
        _, g = scene2d(h, w, 8, 0.05 + 0.02 * i, seed + i)
        imgs.append(g.astype(np.float32))
    return imgs


def plain(g32, **kw):
    s = tv.PlainSolver(g32.shape, DEV)
    f, r = s.solve(torch.from_numpy(g32).to(DEV), **kw)
    return f.cpu().numpy(), r


def plain_state(g32, k):
    s = tv.PlainSolver(g32.shape, DEV)
    s.init(torch.from_numpy(g32).to(DEV))
    if k > 0:
        s.step(k, 0.1)
    f, p = s.state()
    return f.cpu().numpy(), p.cpu().numpy()


@pytest.mark.parametrize("mode", ["persistent", "graph", "launches"])
def test_batch_equals_plain_per_image(mode):
    imgs = small_batch()
    b = tv.BatchedSolver([g.shape for g in imgs], DEV)
    print(f"case: batch mode {mode}", flush=True)
    fs, rs = b.solve([torch.from_numpy(g).to(DEV) for g in imgs], lam=0.1,
                     max_iter=400, check_every=10, gap_tol=2e-3, mode=mode)
    torch.cuda.synchronize()
    iters = set()
    for g, f, r in zip(imgs, fs, rs):
        fp, rp = plain(g, lam=0.1, max_iter=400, check_every=10, gap_tol=2e-3)
        assert r.iters == rp.iters and r.converged == rp.converged
        assert np.array_equal(f.cpu().numpy(), fp)
        assert abs(r.gap - rp.gap) <= 1e-9 * max(rp.primal, 1e-30)
        assert abs(r.primal - rp.primal) <= 1e-9 * max(rp.primal, 1e-30)
        iters.add(r.iters)
    assert len(iters) > 1   # the images really stopped at different k


def test_batch_tile_shapes_do_not_change_iterates():
    imgs = small_batch(400)
    b = tv.BatchedSolver([g.shape for g in imgs], DEV)
    gts = [torch.from_numpy(g).to(DEV) for g in imgs]
    ref = None
    for th, wpb in [(8, 4), (3, 1), (64, 2), (1, 4), (16, 8)]:
        print(f"case: batch tile th={th} wpb={wpb}", flush=True)
        fs, rs = b.solve(gts, lam=0.1, max_iter=120, check_every=10,
                         gap_tol=-1.0, th=th, wpb=wpb)
        out = [f.cpu().numpy().copy() for f in fs]
        if ref is None:
            ref = out
        else:
            for a, c in zip(out, ref):
                assert np.array_equal(a, c)


@pytest.mark.parametrize("mode", ["persistent", "graph", "launches"])
def test_batch_blocked_passes_match_single(mode):
    """Passes of several iterations (up to the pass depth, ending before each
    gap check) give the same iterates, stopping iterations and gaps as
    one-iteration passes, also with odd iteration budgets and check
    intervals."""
    imgs = small_batch(700)
    b = tv.BatchedSolver([g.shape for g in imgs], DEV)
    gts = [torch.from_numpy(g).to(DEV) for g in imgs]
    for kw in [dict(max_iter=121, check_every=0, gap_tol=-1.0),
               dict(max_iter=333, check_every=12, gap_tol=3e-3),
               dict(max_iter=95, check_every=7, gap_tol=3e-3)]:
        out = {}
        for depth in (1, 2, 3, 4):
            print(f"case: batch {mode} depth={depth} {kw}", flush=True)
            tv.set_pass_depth(depth)
            try:
                fs, rs = b.solve(gts, lam=0.1, mode=mode, **kw)
                out[depth] = ([f.cpu().numpy().copy() for f in fs],
                              [(r.iters, r.converged, r.gap, r.primal) for r in rs])
            finally:
                tv.set_blocking(True)
        for depth in (2, 3, 4):
            assert out[depth][1] == out[1][1], depth
            for a, c in zip(out[depth][0], out[1][0]):
                assert np.array_equal(a, c), depth


def test_batch_against_oracle():
    imgs = small_batch(500)[:4]
    b = tv.BatchedSolver([g.shape for g in imgs], DEV)
    fs, rs = b.solve([torch.from_numpy(g).to(DEV) for g in imgs], lam=0.1,
                     max_iter=600, check_every=10, gap_tol=1e-3)
    for g, f, r in zip(imgs, fs, rs):
        g64 = g.astype(np.float64)
        ref = oracle.solve(g64, 0.1, S2, S2, max_iter=600, check_every=10,
                           gap_tol=1e-3, return_history=True)
        # the plain solver's iterates stand for the batch's (equal bit for bit,
        # tested above)
        assert_stop_guard(ref, g64, LAM32, 1e-3, 10,
                          lambda k: plain_state(g, k))
        assert r.iters == ref["iters"]
        fr, _, _ = oracle.run_fixed(g64, 0.1, S2, S2, r.iters)
        err = np.linalg.norm(f.cpu().numpy() - fr) / max(np.linalg.norm(fr), 1e-30)
        assert err <= 1e-5


def test_batch_edge_cases():
    imgs = [np.full((4, 4), 0.3, np.float32),
            scene2d(9, 11, 3, 0.1, 9)[1].astype(np.float32)]
    b = tv.BatchedSolver([g.shape for g in imgs], DEV)
    gts = [torch.from_numpy(g).to(DEV) for g in imgs]
    # max_iter = 0 returns g with the energies of (g, 0)
    fs, rs = b.solve(gts, lam=0.1, max_iter=0, check_every=10, gap_tol=1e-4)
    for g, f, r in zip(imgs, fs, rs):
        assert np.array_equal(f.cpu().numpy(), g) and r.iters == 0
        P, D, gap = oracle.energy_gap(g.astype(np.float64), np.zeros((2,) + g.shape),
                                      g.astype(np.float64), float(np.float32(0.1)))
        assert abs(r.gap - gap) <= 1e-9 * max(P, 1e-30)
    # a constant image stops at k = 0, the other one runs on
    fs, rs = b.solve(gts, lam=0.1, max_iter=50, check_every=10, gap_tol=1e-6)
    assert rs[0].converged and rs[0].iters == 0 and rs[0].gap == 0.0
    assert not rs[1].converged and rs[1].iters == 50
    # a single image
    one = tv.BatchedSolver([imgs[1].shape], DEV)
    f1, r1 = one.solve([gts[1]], lam=0.1, max_iter=50, check_every=10,
                       gap_tol=-1.0)
    fp, rp = plain(imgs[1], lam=0.1, max_iter=50, check_every=10, gap_tol=-1.0)
    assert np.array_equal(f1[0].cpu().numpy(), fp) and r1[0].iters == 50


def test_batch_autotune():
    imgs = small_batch(600)
    b = tv.BatchedSolver([g.shape for g in imgs], DEV)
    (th, wpb), ms = b.autotune([torch.from_numpy(g).to(DEV) for g in imgs])
    assert th in (8, 16, 32, 64, 128) and wpb in (1, 2, 4, 8) and ms > 0


def test_batch64_workload():
    """The 64-image workload in the benchmark's configuration: every image
    stops at relative gap 1e-4; a sample of images equals the plain solver
    bit for bit, and the smallest image matches the oracle."""
    w = WORKLOADS["batch64_uneven"]
    data = batch_scenes(w["n"], w["seed"], w["n_shapes"])
    imgs = [d[1].astype(np.float32) for d in data]
    b = tv.BatchedSolver([g.shape for g in imgs], DEV)
    print("case: batch64 workload", flush=True)
    fs, rs = b.solve([torch.from_numpy(g).to(DEV) for g in imgs], lam=w["lam"],
                     max_iter=w["max_iter"], check_every=w["check_every"],
                     gap_tol=w["gap_tol"])
    assert all(r.converged for r in rs)
    assert all(r.gap <= w["gap_tol"] * r.primal for r in rs)
    sizes = [g.size for g in imgs]
    sample = sorted(set([int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 31]))
    for i in sample:
        fp, rp = plain(imgs[i], lam=w["lam"], max_iter=w["max_iter"],
                       check_every=w["check_every"], gap_tol=w["gap_tol"])
        assert rs[i].iters == rp.iters
        assert np.array_equal(fs[i].cpu().numpy(), fp)
    i = int(np.argmin(sizes))
    g64 = imgs[i].astype(np.float64)
    fr, _, _ = oracle.run_fixed(g64, w["lam"], S2, S2, rs[i].iters)
    err = np.linalg.norm(fs[i].cpu().numpy() - fr) / np.linalg.norm(fr)
    assert err <= 1e-5


@pytest.mark.parametrize("mode", ["persistent", "graph"])
def test_batch_table_switches_do_not_change_iterates(mode):
    """The 64-image workload stopping image by image, so that the driver
    moves from the tall bands through the 8-, 4- and 2-row tables (or the
    halvings of another first short band) while the images stop: every
    tiling gives the same stopping iterations and the same iterates bit for
    bit."""
    w = WORKLOADS["batch64_uneven"]
    data = batch_scenes(w["n"], w["seed"], w["n_shapes"])
    gts = [torch.from_numpy(d[1].astype(np.float32)).to(DEV) for d in data]
    b = tv.BatchedSolver([tuple(g.shape) for g in gts], DEV)
    ref = None
    for th, th_short, wpb in [(32, 8, 4), (16, 4, 4), (24, 3, 4), (64, 1, 4), (32, 8, 8)]:
        print(f"case: batch64 {mode} th={th} th_short={th_short} wpb={wpb}", flush=True)
        fs, rs = b.solve(gts, lam=w["lam"], max_iter=w["max_iter"],
                         check_every=w["check_every"], gap_tol=w["gap_tol"],
                         mode=mode, th=th, wpb=wpb, th_short=th_short)
        out = ([f.cpu().numpy().copy() for f in fs], [r.iters for r in rs])
        assert all(r.converged for r in rs)
        if ref is None:
            ref = out
            assert len(set(out[1])) > 10   # many stopping iterations
        else:
            assert out[1] == ref[1]
            for a, c in zip(out[0], ref[0]):
                assert np.array_equal(a, c)
