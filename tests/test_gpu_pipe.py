"""Pipelined passes of the plain 2D solver against the strip walk.

A pipelined pass runs the walk's stages on the waves of one block, one stage
per wave, so for every pass length (1 to 10 iterations per launch) it must
give the walk's iterates and duals bit for bit, with the same stopping
iterations; the full-size image is checked against the walk too (parity
with the oracle at that size is in test_gpu_plain.py)."""
import numpy as np
import pytest
import torch

import paper_1608_03589_amd as tv
from scenes import scene2d

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
S2 = 1.0 / np.sqrt(8.0)


def scene32(H, W, seed):
    return scene2d(H, W, 12, 0.1, seed)[1].astype(np.float32)


def run(g32, depth, tile, n_fixed, solves):
    tv.set_tile(g32.shape, *tile)
    tv.set_pass_depth(depth)
    s = tv.PlainSolver(g32.shape, DEV)
    gt = torch.from_numpy(g32).to(DEV)
    s.solve(gt, lam=0.1, tau=S2, sigma=S2, max_iter=n_fixed, check_every=0,
            gap_tol=-1.0)
    f, p = s.state()
    out = {"fixed": (f.cpu().numpy(), p.cpu().numpy())}
    for ce in solves:
        fs, rs = s.solve(gt, 0.1, max_iter=400, check_every=ce, gap_tol=2e-3)
        out[ce] = (fs.cpu().numpy(), rs.iters, rs.converged)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("shape,th", [
    ((300, 517), 300), ((300, 517), 64), ((300, 517), 7), ((1, 261), 1),
    ((7, 9), 3), ((37, 1030), 20), ((600, 250), 128), ((2, 470), 1),
    ((20, 464), 4), ((21, 465), 5), ((31, 233), 9), ((12, 232), 12),
    ((513, 257), 500), ((130, 700), 33),
])
def test_pipelined_passes_equal_the_walk(shape, th):
    g32 = scene32(*shape, 7000 + shape[0] + shape[1])
    solves = (10, 7, 3)
    saved = tv.get_tile(shape)
    try:
        print(f"case: walk depth 1 shape {shape}", flush=True)
        ref = run(g32, 1, (4, 4, 0), 23, solves)
        for depth in (10, 7, 5, 2, 1):
            print(f"case: pipelined depth {depth} shape {shape} th {th}", flush=True)
            got = run(g32, depth, (th, 1, 2), 23, solves)
            assert np.array_equal(got["fixed"][0], ref["fixed"][0]), depth
            assert np.array_equal(got["fixed"][1], ref["fixed"][1]), depth
            for ce in solves:
                a, b = got[ce], ref[ce]
                assert a[1] == b[1] and a[2] == b[2], (depth, ce, a[1], b[1])
                assert np.array_equal(a[0], b[0]), (depth, ce)
    finally:
        tv.set_blocking(True)
        tv.set_tile(shape, *saved)


def test_full_size_pipelined_passes_equal_the_walk():
    # one band of 293 rows per CU (4096 / floor(256 CUs / 18 strips)), the
    # band the pipelined passes were measured on; the default stays the walk
    shape = (4096, 4096)
    default = tv.get_tile(shape)
    assert default[2] != 2
    g32 = scene32(*shape, 7100)
    try:
        print("case: 4096^2 pipelined vs walk, 25 iterations", flush=True)
        ref = run(g32, 0, (37, 4, 0), 25, ())
        got = run(g32, 0, (293, 1, 2), 25, ())
    finally:
        tv.set_blocking(True)
        tv.set_tile(shape, *default)
    assert np.array_equal(got["fixed"][0], ref["fixed"][0])
    assert np.array_equal(got["fixed"][1], ref["fixed"][1])


def test_timed_out_wait_is_reported():
    # with a one-poll limit the first wait that is not satisfied almost at
    # once gives up (stage 2 waits for stage 1's first row, which needs loads
    # from memory); every wave still ends its pass, and the solve raises
    shape = (300, 517)
    saved = tv.get_tile(shape)
    g32 = scene32(*shape, 7200)
    gt = torch.from_numpy(g32).to(DEV)
    kw = dict(tau=S2, sigma=S2, max_iter=20, check_every=10, gap_tol=-1.0)
    try:
        tv.set_pass_depth(0)
        tv.set_tile(shape, 4, 4, 0)
        s = tv.PlainSolver(shape, DEV)
        ref, _ = s.solve(gt, 0.1, **kw)
        ref = ref.cpu().numpy()
        tv.set_tile(shape, 64, 1, 2)
        tv.set_wait_limit(1)
        print("case: pipelined solve with a one-poll wait limit", flush=True)
        with pytest.raises(tv.TVPDError):
            s.solve(gt, 0.1, **kw)
        torch.cuda.synchronize()
        tv.set_wait_limit(0)
        print("case: the same solve with the default limit", flush=True)
        f, r = s.solve(gt, 0.1, **kw)
        f = f.cpu().numpy()
    finally:
        tv.set_wait_limit(0)
        tv.set_blocking(True)
        tv.set_tile(shape, *saved)
    assert r.iters == 20
    assert np.array_equal(f, ref)
