"""Workspace contents before a solve do not reach its results.

Every plane, reduction slot and table of the plain (2D, 3D) and batched
workspaces is written before it is read: a workspace filled with NaN bytes
(0xFF) gives the same iterates, duals, stopping iterations and energies, bit
for bit, as a zeroed one.
"""
import math

import numpy as np
import pytest
import torch

import paper_1608_03589_amd as tv
from scenes import scene2d, scene3d

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def plain_run(g, fill, max_iter, check_every, gap_tol):
    s = tv.PlainSolver(g.shape, DEV)
    s.ws.fill_(fill)
    gt = torch.from_numpy(g).to(DEV)
    f, res = s.solve(gt, lam=0.1, max_iter=max_iter, check_every=check_every,
                     gap_tol=gap_tol)
    _, p = s.state()
    torch.cuda.synchronize()
    return (f.cpu().numpy(), p.cpu().numpy(),
            (res.iters, res.converged, res.primal, res.dual, res.gap))


@pytest.mark.parametrize("depth", [1, 5])
@pytest.mark.parametrize("shape", [(300, 517), (7, 9), (1, 261)])
def test_plain_2d_nan_workspace(shape, depth):
    print(f"case: NaN workspace plain 2D {shape} depth {depth}", flush=True)
    _, g = scene2d(*shape, 12, 0.1, 4100 + shape[0])
    g = g.astype(np.float32)
    old = tv.get_pass_depth()
    tv.set_pass_depth(depth)
    try:
        a = plain_run(g, 0x00, 300, 10, 1e-4)
        b = plain_run(g, 0xFF, 300, 10, 1e-4)
    finally:
        tv.set_pass_depth(old)
    assert np.isfinite(a[0]).all() and np.isfinite(a[1]).all()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2] == b[2]


@pytest.mark.parametrize("shape", [(9, 23, 270), (3, 5, 7)])
def test_plain_3d_nan_workspace(shape):
    print(f"case: NaN workspace plain 3D {shape}", flush=True)
    _, g = scene3d(*shape, 6, 0.1, 4200 + shape[0])
    g = g.astype(np.float32)
    a = plain_run(g, 0x00, 60, 10, 1e-3)
    b = plain_run(g, 0xFF, 60, 10, 1e-3)
    assert np.isfinite(a[0]).all() and np.isfinite(a[1]).all()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2] == b[2]


@pytest.mark.parametrize("mode", ["persistent", "graph"])
def test_batch_nan_workspace(mode):
    shapes = [(300, 517), (7, 9), (130, 260), (1, 300), (64, 64)]
    print(f"case: NaN workspace batch {mode} {shapes}", flush=True)
    imgs = [torch.from_numpy(scene2d(h, w, 10, 0.1, 4300 + i)[1].astype(np.float32)).to(DEV)
            for i, (h, w) in enumerate(shapes)]
    out = []
    for fill in (0x00, 0xFF):
        b = tv.BatchedSolver(shapes, DEV)
        b.ws.fill_(fill)
        fs, res = b.solve(imgs, lam=0.1, max_iter=2000, check_every=10, gap_tol=1e-4,
                          mode=mode)
        torch.cuda.synchronize()
        out.append(([f.cpu().numpy() for f in fs],
                    [(r.iters, r.converged, r.primal, r.dual, r.gap) for r in res]))
    for fa, fb in zip(out[0][0], out[1][0]):
        assert np.isfinite(fa).all() and np.array_equal(fa, fb)
    assert out[0][1] == out[1][1]
    # the images stop at different iterations, so the deferred decisions and
    # the rebuilt active lists are exercised
    assert len({r[0] for r in out[0][1]}) > 1
