"""GPU parity at coefficient values away from the default ones.

theta = 0.5 (a weaker extrapolation, accepted for theta in [0, 1]) in the plain
2D solver at pass depths 1 and 5, the plain 3D solver and the unrolled 2D
solver; lam = 0, where the projection onto the zero ball makes the dual exactly
0 and the data prox keeps f at g; and a weight so large that the projection
never acts, where the iteration is linear.  Every case is compared with the
FP64 oracle after a fixed number of iterations.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1608_03589_amd as tv
from oracle.unrolled import unrolled_backward_batch, unrolled_forward_batch
from scenes import scene2d, scene3d

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
S2 = 1.0 / math.sqrt(8.0)
S3 = 1.0 / math.sqrt(12.0)
RTOL = 1e-5


def rel(a, b):
    a = np.asarray(a, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def f32(v):
    return float(np.float32(v))


def device_fixed(g32, n, lam, theta, tau, sigma):
    s = tv.PlainSolver(g32.shape, DEV)
    s.init(torch.from_numpy(g32).to(DEV))
    s.step(n, lam, tau, sigma, theta)
    f, p = s.state()
    torch.cuda.synchronize()
    assert s.iteration() == n
    return f.cpu().numpy(), p.cpu().numpy()


@pytest.mark.parametrize("depth", [1, 5])
@pytest.mark.parametrize("shape", [(37, 301), (130, 513), (5, 3)])
def test_theta_half_2d(depth, shape):
    print(f"case: theta 0.5 2D {shape} depth {depth}", flush=True)
    _, g = scene2d(*shape, 8, 0.1, 40 + shape[0])
    g32 = g.astype(np.float32)
    n = 47
    tv.set_pass_depth(depth)
    try:
        f, p = device_fixed(g32, n, 0.1, 0.5, S2, S2)
    finally:
        tv.set_blocking(True)
    fr, _, pr = oracle.run_fixed(g32.astype(np.float64), f32(0.1), f32(S2),
                                 f32(S2), n, theta=0.5)
    assert rel(f, fr) <= RTOL
    assert rel(p, pr) <= 10 * RTOL


def test_theta_half_3d():
    print("case: theta 0.5 3D (14, 19, 270)", flush=True)
    _, g = scene3d(14, 19, 270, 10, 0.1, 41)
    g32 = g.astype(np.float32)
    n = 31
    f, p = device_fixed(g32, n, 0.1, 0.5, S3, S3)
    fr, _, pr = oracle.run_fixed(g32.astype(np.float64), f32(0.1), f32(S3),
                                 f32(S3), n, theta=0.5)
    assert rel(f, fr) <= RTOL
    assert rel(p, pr) <= 10 * RTOL


@pytest.mark.parametrize("shape,K,ckpt", [((2, 37, 301), 9, 4), ((1, 9, 17), 5, 5)])
def test_theta_half_unrolled_2d(shape, K, ckpt):
    print(f"case: theta 0.5 unrolled {shape} K={K}", flush=True)
    B, H, W = shape
    g = np.stack([scene2d(H, W, 8, 0.1, 50 + i)[1] for i in range(B)]).astype(np.float32)
    rng = np.random.default_rng(51)
    c = (np.tile([0.1, S2, S2], (K, 1)) * rng.uniform(0.8, 1.2, (K, 3))).astype(np.float32)
    grad_f = rng.normal(size=g.shape).astype(np.float32)
    solver = tv.UnrolledSolver(g.shape, K, ckpt, 0.5, DEV)
    ct = torch.from_numpy(c).to(DEV)
    f = solver.forward(torch.from_numpy(g).to(DEV), ct)
    gg, gc = solver.backward(ct, torch.from_numpy(grad_f).to(DEV))
    torch.cuda.synchronize()
    g64, c64 = g.astype(np.float64), c.astype(np.float64)
    assert rel(f.cpu().numpy(), unrolled_forward_batch(g64, c64, theta=0.5)) <= RTOL
    gg_ref, gc_ref = unrolled_backward_batch(g64, c64, grad_f.astype(np.float64),
                                             theta=0.5)
    assert rel(gg.cpu().numpy(), gg_ref) <= 1e-4
    assert rel(gc.cpu().numpy(), gc_ref) <= 1e-4


@pytest.mark.parametrize("shape", [(130, 513), (12, 17, 70)])
def test_lam_zero(shape):
    """lam = 0: every projection lands on the zero ball, so p^k is exactly 0;
    f^{k+1} = (f^k + tau g) / (1 + tau) then stays at g up to the rounding of
    the data prox (a contraction towards g by 1/(1 + tau), so the deviation
    stays below a few float32 units in the last place)."""
    print(f"case: lam 0 {shape}", flush=True)
    if len(shape) == 2:
        _, g = scene2d(*shape, 8, 0.1, 42)
        s = S2
    else:
        _, g = scene3d(*shape, 8, 0.1, 42)
        s = S3
    g32 = g.astype(np.float32)
    f, p = device_fixed(g32, 40, 0.0, 1.0, s, s)
    assert np.all(p == 0.0)
    assert np.all(np.abs(f - g32) <= 8 * np.spacing(np.abs(g32)))
    fr, _, pr = oracle.run_fixed(g32.astype(np.float64), 0.0, f32(s), f32(s), 40)
    assert np.all(pr == 0.0)
    assert rel(f, fr) <= 1e-6


@pytest.mark.parametrize("shape", [(130, 513), (12, 17, 70)])
def test_projection_never_acts(shape):
    """lam = 1000 exceeds every |q| the 60 iterations reach (the oracle's run at
    lam = 1e30, where no projection can act, is identical), so the iteration
    is the linear one; the device follows the oracle to the usual bound."""
    print(f"case: inactive projection {shape}", flush=True)
    if len(shape) == 2:
        _, g = scene2d(*shape, 8, 0.1, 43)
        s = S2
    else:
        _, g = scene3d(*shape, 8, 0.1, 43)
        s = S3
    g32 = g.astype(np.float32)
    n = 60
    f, p = device_fixed(g32, n, 1000.0, 1.0, s, s)
    g64 = g32.astype(np.float64)
    fr, _, pr = oracle.run_fixed(g64, 1000.0, f32(s), f32(s), n)
    fi, _, pi = oracle.run_fixed(g64, 1e30, f32(s), f32(s), n)
    assert np.array_equal(fr, fi) and np.array_equal(pr, pi)
    assert rel(f, fr) <= RTOL
    assert rel(p, pr) <= 10 * RTOL
