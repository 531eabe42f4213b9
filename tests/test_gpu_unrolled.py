"""GPU tests of the unrolled solver and its hand-written adjoint.

Forward: relative L2 <= 1e-5 against the FP64 oracle.  Backward: the device
gradient is float32 arithmetic through K projections, compared with the
oracle's FP64 reverse-mode gradient to a relative L2 of 1e-4 (the oracle's
gradient is itself pinned to FP64 finite differences on the CPU).
Checkpoint intervals change nothing: recomputed states are bit-identical.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1608_03589_amd as tv
from oracle.unrolled import unrolled_backward_batch, unrolled_forward_batch
from scenes import WORKLOADS, scene2d, scene3d

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def rel(a, b):
    a = np.asarray(a, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def coeffs_for(K, ndim, seed, spread=0.2):
    rng = np.random.default_rng(seed)
    s = 1.0 / math.sqrt(4.0 * ndim)
    c = np.tile([0.1, s, s], (K, 1)) * rng.uniform(1 - spread, 1 + spread, (K, 3))
    return c.astype(np.float32)


def batch2d(B, H, W, seed):
    out_c, out_n = [], []
    for i in range(B):
        c, n = scene2d(H, W, 8, 0.1, seed + i)
        out_c.append(c)
        out_n.append(n)
    return np.stack(out_c).astype(np.float32), np.stack(out_n).astype(np.float32)


def run_gpu(g, c, ckpt, grad_f):
    solver = tv.UnrolledSolver(g.shape, c.shape[0], ckpt, 1.0, DEV)
    gt = torch.from_numpy(g).to(DEV)
    ct = torch.from_numpy(c).to(DEV)
    f = solver.forward(gt, ct)
    gg, gc = solver.backward(ct, torch.from_numpy(grad_f).to(DEV))
    torch.cuda.synchronize()
    return f.cpu().numpy(), gg.cpu().numpy(), gc.cpu().numpy()


@pytest.mark.parametrize("shape,K,ckpt", [((3, 37, 301), 8, 3),
                                          ((2, 64, 70), 11, 11),
                                          ((1, 5, 3), 4, 2)])
def test_unrolled_2d_parity(shape, K, ckpt):
    print(f"case: unrolled 2d {shape} K={K} ckpt={ckpt}", flush=True)
    clean, g = batch2d(*shape, seed=700)
    c = coeffs_for(K, 2, 7)
    rng = np.random.default_rng(8)
    grad_f = rng.normal(size=g.shape).astype(np.float32)
    f, gg, gc = run_gpu(g, c, ckpt, grad_f)
    g64, c64 = g.astype(np.float64), c.astype(np.float64)
    f_ref = unrolled_forward_batch(g64, c64)
    assert rel(f, f_ref) <= 1e-5
    gg_ref, gc_ref = unrolled_backward_batch(g64, c64, grad_f.astype(np.float64))
    assert rel(gg, gg_ref) <= 1e-4
    assert rel(gc, gc_ref) <= 1e-4


@pytest.mark.parametrize("shape,K,ckpt", [((2, 70, 301), 13, 13),
                                          ((3, 37, 520), 12, 5),
                                          ((1, 9, 17), 7, 3)])
def test_forward_passes_are_bitwise_equal(shape, K, ckpt):
    """The 2D forward runs as passes of up to five iterations that store every
    iterate; one-iteration passes give the same iterates, dL/dg and
    coefficient gradients bit for bit (checkpointed segments included)."""
    print(f"case: unrolled passes {shape} K={K} ckpt={ckpt}", flush=True)
    _, g = batch2d(*shape, seed=910)
    c = coeffs_for(K, 2, 11)
    grad_f = np.random.default_rng(12).normal(size=g.shape).astype(np.float32)
    out = {}
    try:
        for depth in (1, 5):
            tv.set_pass_depth(depth)
            out[depth] = run_gpu(g, c, ckpt, grad_f)
    finally:
        tv.set_blocking(True)
    for a, b in zip(out[5], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shape,K,ckpt", [((2, 37, 301), 6, 3),
                                          ((1, 130, 520), 5, 5),
                                          ((3, 9, 17), 4, 2),
                                          ((1, 1, 260), 3, 3)])
def test_fused_adjoint_equals_two_pass_adjoint(shape, K, ckpt):
    """The single-pass 2D adjoint and the two-pass reference give the same
    dL/dg bit for bit; the coefficient gradients differ only in the order of
    their float64 sums."""
    print(f"case: fused vs two-pass adjoint {shape} K={K}", flush=True)
    _, g = batch2d(*shape, seed=900)
    c = coeffs_for(K, 2, 9)
    grad_f = np.random.default_rng(10).normal(size=g.shape).astype(np.float32)
    out = []
    for fused in (True, False):
        tv.set_fused_adjoint(fused)
        try:
            out.append(run_gpu(g, c, ckpt, grad_f))
        finally:
            tv.set_fused_adjoint(True)
    (f1, gg1, gc1), (f2, gg2, gc2) = out
    assert np.array_equal(f1, f2)
    assert np.array_equal(gg1, gg2)
    assert np.allclose(gc1, gc2, rtol=1e-5, atol=1e-7 * np.abs(gc2).max())


@pytest.mark.parametrize("shape,K,ckpt", [((1, 9, 14, 300), 4, 2),
                                          ((2, 13, 7, 20), 5, 5),
                                          ((1, 40, 6, 9), 3, 3)])
def test_fused_adjoint_equals_two_pass_adjoint_3d(shape, K, ckpt):
    print(f"case: fused vs two-pass adjoint 3d {shape} K={K}", flush=True)
    g = np.stack([scene3d(*shape[1:], 6, 0.1, 950 + i)[1]
                  for i in range(shape[0])]).astype(np.float32)
    c = coeffs_for(K, 3, 11)
    grad_f = np.random.default_rng(12).normal(size=g.shape).astype(np.float32)
    out = []
    for fused in (True, False):
        tv.set_fused_adjoint(fused)
        try:
            out.append(run_gpu(g, c, ckpt, grad_f))
        finally:
            tv.set_fused_adjoint(True)
    (f1, gg1, gc1), (f2, gg2, gc2) = out
    assert np.array_equal(f1, f2)
    assert np.array_equal(gg1, gg2)
    assert np.allclose(gc1, gc2, rtol=1e-5, atol=1e-7 * np.abs(gc2).max())


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("shape,K,ckpt", [((2, 21, 301), 6, 3),
                                          ((1, 7, 9, 266), 5, 2)])
def test_workspace_contents_do_not_matter(shape, K, ckpt, fused):
    """The forward initialises only g and p^0; every other plane is written
    whole before it is read.  A workspace full of NaN gives the same results
    bit for bit as a zeroed one."""
    print(f"case: NaN workspace {shape} fused={fused}", flush=True)
    ndim = len(shape) - 1
    if ndim == 2:
        _, g = batch2d(*shape, seed=960)
    else:
        g = np.stack([scene3d(*shape[1:], 6, 0.1, 970 + i)[1]
                      for i in range(shape[0])]).astype(np.float32)
    c = coeffs_for(K, ndim, 13)
    grad_f = np.random.default_rng(14).normal(size=g.shape).astype(np.float32)
    tv.set_fused_adjoint(fused)
    try:
        out = []
        for fill in (0x00, 0xFF):
            solver = tv.UnrolledSolver(g.shape, K, ckpt, 1.0, DEV)
            solver.ws.fill_(fill)
            gt = torch.from_numpy(g).to(DEV)
            ct = torch.from_numpy(c).to(DEV)
            f = solver.forward(gt, ct)
            gg, gc = solver.backward(ct, torch.from_numpy(grad_f).to(DEV))
            torch.cuda.synchronize()
            out.append((f.cpu().numpy(), gg.cpu().numpy(), gc.cpu().numpy()))
    finally:
        tv.set_fused_adjoint(True)
    for a, b in zip(out[0], out[1]):
        assert np.isfinite(a).all() and np.array_equal(a, b)


def test_unrolled_3d_parity():
    print("case: unrolled 3d", flush=True)
    vols = [scene3d(10, 12, 13, 5, 0.1, 900 + i)[1] for i in range(2)]
    g = np.stack(vols).astype(np.float32)
    K = 6
    c = coeffs_for(K, 3, 9)
    grad_f = np.random.default_rng(10).normal(size=g.shape).astype(np.float32)
    f, gg, gc = run_gpu(g, c, 4, grad_f)
    g64, c64 = g.astype(np.float64), c.astype(np.float64)
    assert rel(f, unrolled_forward_batch(g64, c64)) <= 1e-5
    gg_ref, gc_ref = unrolled_backward_batch(g64, c64, grad_f.astype(np.float64))
    assert rel(gg, gg_ref) <= 1e-4
    assert rel(gc, gc_ref) <= 1e-4


@pytest.mark.parametrize("ndim", [2, 3])
def test_checkpoint_interval_is_bitwise_neutral(ndim):
    if ndim == 2:
        _, g = batch2d(2, 50, 270, seed=710)
    else:
        g = np.stack([scene3d(9, 10, 11, 4, 0.1, 920)[1]]).astype(np.float32)
    K = 13
    c = coeffs_for(K, ndim, 11)
    grad_f = np.random.default_rng(12).normal(size=g.shape).astype(np.float32)
    outs = [run_gpu(g, c, ck, grad_f) for ck in (2, 5, 13, 40)]
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_forward_equals_plain_solver():
    """K iterations with constant coefficients equal the plain solver's
    first K iterations up to rounding: the unrolled forward forms the
    extrapolation from the stored f^{k-1}, the plain solver from f^k, g and
    p^k (the same value in exact arithmetic)."""
    _, g = batch2d(1, 96, 300, seed=720)
    K = 9
    s = 1.0 / math.sqrt(8.0)
    c = np.tile(np.array([[0.1, s, s]], np.float32), (K, 1))
    solver = tv.UnrolledSolver(g.shape, K, 4, 1.0, DEV)
    f = solver.forward(torch.from_numpy(g).to(DEV), torch.from_numpy(c).to(DEV))
    p = tv.PlainSolver(g.shape[1:], DEV)
    fp, _ = p.solve(torch.from_numpy(g[0]).to(DEV), lam=float(c[0, 0]),
                    tau=float(c[0, 1]), sigma=float(c[0, 2]), max_iter=K,
                    check_every=0, gap_tol=-1.0)
    err = float(torch.linalg.norm(f[0] - fp) / torch.linalg.norm(fp))
    assert err < 1e-6, err


def test_autograd_function_and_crop_fd():
    """torch.autograd through UnrolledTV on 16x16 crops of the first
    noisy/clean pair (K = 20): gradients match the FP64 oracle adjoint, which
    the CPU tests pin to FP64 finite differences, and a direct FP64 finite
    difference of two coefficients."""
    clean, noisy = scene2d(512, 512, 20, 0.1, 4000)
    c16 = clean[:16, :16].astype(np.float32)
    g16 = noisy.astype(np.float32)[:16, :16].copy()
    K = 20
    coeffs = torch.from_numpy(coeffs_for(K, 2, 13, spread=0.1)).to(DEV).requires_grad_(True)
    g = torch.from_numpy(g16[None]).to(DEV).requires_grad_(True)
    target = torch.from_numpy(c16[None]).to(DEV)
    f = tv.unrolled_tv(g, coeffs, ckpt_every=5)
    loss = torch.mean((f - target) ** 2)
    loss.backward()
    c64 = coeffs.detach().cpu().numpy().astype(np.float64)
    g64 = g16.astype(np.float64)
    fK = oracle.unrolled_forward(g64, c64)
    gg_ref, gc_ref = oracle.unrolled_backward(g64, c64, 2 * (fK - c16) / fK.size)
    assert rel(coeffs.grad.cpu().numpy(), gc_ref) <= 1e-4
    assert rel(g.grad.cpu().numpy()[0], gg_ref) <= 1e-4
    h = 1e-7
    for (k, j) in [(3, 0), (17, 2)]:
        cp, cm = c64.copy(), c64.copy()
        cp[k, j] += h
        cm[k, j] -= h
        fd = (np.mean((oracle.unrolled_forward(g64, cp) - c16) ** 2)
              - np.mean((oracle.unrolled_forward(g64, cm) - c16) ** 2)) / (2 * h)
        assert abs(coeffs.grad[k, j].item() - fd) <= 1e-3 * abs(fd) + 1e-9


def test_unrolled_32x512_workload():
    """The 2D unrolled workload (32 x 512^2, K = 20): two images against the
    oracle, and the batch's coefficient gradient equals the sum of per-image
    device gradients."""
    w = WORKLOADS["unrolled_32x512"]
    clean, g = [], []
    for i in range(w["B"]):
        c, n = scene2d(w["H"], w["W"], w["n_shapes"], w["noise"], w["seed"] + i)
        clean.append(c)
        g.append(n)
    clean = np.stack(clean).astype(np.float32)
    g = np.stack(g).astype(np.float32)
    K = w["K"]
    c = coeffs_for(K, 2, 14, spread=0.0)
    print("case: unrolled 32x512 workload", flush=True)
    solver = tv.UnrolledSolver(g.shape, K, 5, 1.0, DEV)
    gt, ct = torch.from_numpy(g).to(DEV), torch.from_numpy(c).to(DEV)
    f = solver.forward(gt, ct)
    grad_f = 2 * (f - torch.from_numpy(clean).to(DEV)) / f.numel()
    gg, gc = solver.backward(ct, grad_f)
    gf = grad_f.cpu().numpy()
    for i in (0, w["B"] - 1):
        g64 = g[i].astype(np.float64)
        assert rel(f[i].cpu().numpy(), oracle.unrolled_forward(g64, c.astype(np.float64))) <= 1e-5
        ggr, _ = oracle.unrolled_backward(g64, c.astype(np.float64), gf[i].astype(np.float64))
        assert rel(gg[i].cpu().numpy(), ggr) <= 1e-4
    tot = np.zeros((K, 3))
    one = tv.UnrolledSolver((1,) + g.shape[1:], K, 5, 1.0, DEV)
    for i in range(w["B"]):
        one.forward(gt[i:i + 1].contiguous(), ct)
        tot += one.backward(ct, grad_f[i:i + 1].contiguous())[1].double().cpu().numpy()
    assert rel(gc.cpu().numpy(), tot) <= 1e-5


def test_unrolled_256cube_properties():
    """The 3D workload (256^3, K = 100, checkpoint every 10) at full size:
    exact identities of the unrolled map hold for the device gradients.
    Shift equivariance f^K(g + e 1) = f^K(g) + e 1 gives
    sum(dL/dg) = sum(dL/df^K); scale equivariance f^K(a g; a lam) = a f^K
    gives <g, dL/dg> + sum_k lam_k dL/dlam_k = <f^K, dL/df^K>."""
    w = WORKLOADS["unrolled_256cube"]
    clean, noisy = scene3d(w["D"], w["H"], w["W"], w["n_shapes"], w["noise"], w["seed"])
    g = noisy[None].astype(np.float32)
    K = w["K"]
    c = coeffs_for(K, 3, 15, spread=0.1)
    print("case: unrolled 256^3 K=100 ckpt=10", flush=True)
    torch.cuda.reset_peak_memory_stats()
    solver = tv.UnrolledSolver(g.shape, K, w["ckpt_every"], 1.0, DEV)
    gt, ct = torch.from_numpy(g).to(DEV), torch.from_numpy(c).to(DEV)
    f = solver.forward(gt, ct)
    grad_f = 2 * (f - torch.from_numpy(clean[None].astype(np.float32)).to(DEV)) / f.numel()
    gg, gc = solver.backward(ct, grad_f)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() / 2 ** 30
    print(f"peak device memory {peak:.2f} GiB, workspace {solver.nbytes / 2**30:.2f} GiB")
    f64, gf64, gg64 = f.double(), grad_f.double(), gg.double()
    assert abs(gg64.sum().item() - gf64.sum().item()) <= 1e-4 * gf64.abs().sum().item()
    lhs = (gt.double() * gg64).sum().item() + float((ct[:, 0].double() * gc[:, 0].double()).sum())
    rhs = (f64 * gf64).sum().item()
    assert abs(lhs - rhs) <= 1e-3 * (abs(rhs) + (gt.double() * gg64).abs().sum().item())
    # mass conservation of the forward
    assert abs(f64.sum().item() - gt.double().sum().item()) <= 1e-5 * gt.double().abs().sum().item()
    assert peak < 12.0


def test_unrolled_256cube_corner_windows_against_the_oracle():
    """The 3D workload in its own launch configuration (256^3, K = 100,
    checkpoint every 10) against the oracle on crops.  One iteration couples a
    voxel only to voxels at most one step away along each axis, so f^K on a
    window of side w at a corner of the volume depends only on the crop of side
    w + K + 1 at that corner, whose three outer faces are the volume's own
    boundary.  For the gradient, dL/df^K is supported on the window: the
    adjoint of iteration k then reaches at most w + K - k voxels deep, while
    the crop's forward state of iteration k is exact up to c - k - 1 voxels
    deep, so on the same crop dL/dg and the coefficient gradients are those of
    the full volume."""
    w = WORKLOADS["unrolled_256cube"]
    clean, noisy = scene3d(w["D"], w["H"], w["W"], w["n_shapes"], w["noise"], w["seed"])
    g = noisy[None].astype(np.float32)
    K, ck, win = w["K"], w["ckpt_every"], 8
    c = K + win + 2
    coeffs = coeffs_for(K, 3, 16, spread=0.1)
    print(f"case: unrolled 256^3 K={K} ckpt={ck} corner windows {win}, crops {c}",
          flush=True)
    solver = tv.UnrolledSolver(g.shape, K, ck, 1.0, DEV)
    gt, ct = torch.from_numpy(g).to(DEV), torch.from_numpy(coeffs).to(DEV)
    f = solver.forward(gt, ct)
    grad_f = torch.zeros_like(f)
    grad_f[0, :win, :win, :win] = 1.0 / win ** 3
    gg, gc = solver.backward(ct, grad_f)
    torch.cuda.synchronize()
    f, gg, gc = f[0].cpu().numpy(), gg[0].cpu().numpy(), gc.cpu().numpy()
    c64 = coeffs.astype(np.float64)
    g64 = g[0].astype(np.float64)
    hi = g64[-c:, -c:, -c:]
    f_hi = oracle.unrolled_forward(hi, c64)
    print("oracle forward at the far corner done", flush=True)
    assert rel(f[-win:, -win:, -win:], f_hi[-win:, -win:, -win:]) <= 1e-5
    lo = g64[:c, :c, :c]
    gf_lo = np.zeros_like(lo)
    gf_lo[:win, :win, :win] = 1.0 / win ** 3
    f_lo = oracle.unrolled_forward(lo, c64)
    assert rel(f[:win, :win, :win], f_lo[:win, :win, :win]) <= 1e-5
    gg_ref, gc_ref = oracle.unrolled_backward(lo, c64, gf_lo)
    print("oracle backward at the near corner done", flush=True)
    assert rel(gg[:c - 1, :c - 1, :c - 1], gg_ref[:c - 1, :c - 1, :c - 1]) <= 1e-4
    assert np.all(gg[c:, :, :] == 0) and np.all(gg[:, c:, :] == 0) and np.all(gg[:, :, c:] == 0)
    assert rel(gc, gc_ref) <= 1e-4


def test_second_backward_through_the_same_graph_raises():
    _, g = batch2d(1, 9, 17, seed=730)
    K = 3
    coeffs = torch.from_numpy(coeffs_for(K, 2, 17)).to(DEV).requires_grad_(True)
    gt = torch.from_numpy(g).to(DEV).requires_grad_(True)
    loss = tv.unrolled_tv(gt, coeffs).square().sum()
    loss.backward(retain_graph=True)
    with pytest.raises(RuntimeError, match="second backward"):
        loss.backward()
