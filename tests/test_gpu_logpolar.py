"""GPU parity of the log-polar backprojection (Andersson's formula, Section
2.1; the four steps of Section 5) against the FP64 oracle.

Both the log-polar result [B g]_L (after Step 3) and the image (after Step 4)
are compared, relative L2 <= 1e-5, on random sinograms over several mesh
shapes (rho transforms of lengths 64 to 2048, ray counts with factors 2, 3 and
5, images inside and beyond the detector's disc, odd sides with a pixel at the
origin), and at the full tomography workload (2048^2 from 1000 projections
of 2048 bins: N_rho = 8159, L = 16384, 2000 rays) on the whole log-polar
result and the whole image.
"""
import math

import numpy as np
import pytest
import torch

import paper_1608_03589_amd as tv
import scenes
from oracle import logpolar as lp
from oracle import tomo

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
RTOL = 1e-5


def rel(a, b):
    a = np.asarray(a, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def run(H, W, na, nd, s):
    solver = tv.TomoSolver(H, W, na, nd, DEV)
    n_rho, n_phi, L, _, _ = solver.lp_mesh()
    bl = torch.empty((n_phi, n_rho), dtype=torch.float32, device=DEV)
    img = solver.logpolar(to_dev(s), lp_out=bl)
    torch.cuda.synchronize()
    return img.cpu().numpy(), bl.cpu().numpy(), solver


@pytest.mark.parametrize("H,W,na,nd", [
    (64, 64, 48, 92),        # detector covers the image; 96 rays
    (37, 53, 30, 70),        # non-square, 60 rays (2^2 3 5)
    (33, 21, 45, 40),        # odd sides (a pixel at the origin), corners beyond the disc
    (128, 128, 400, 185),    # 800 rays
    (200, 120, 75, 300),     # 150 rays (2 3 5^2), rho transform of 2048
    (6, 6, 1, 8),            # two rays, rho transform of 16 (one fused radix-16 stage)
    (4, 4, 2, 4),            # rho transform of 8: no radix-16 stage to fuse
])
def test_logpolar_matches_the_oracle(H, W, na, nd):
    print(f"case: logpolar {H}x{W} angles {na} bins {nd}", flush=True)
    s = np.random.default_rng(H * 5 + nd).normal(size=(na, nd)).astype(np.float32)
    img, bl, solver = run(H, W, na, nd, s)
    s64 = s.astype(np.float64)
    bl_ref = lp.logpolar_result(s64, H, W)
    m = lp.mesh(H, W, na, nd)
    assert bl.shape == bl_ref.shape == (m.n_phi, m.n_rho)
    img_ref = lp.to_cartesian(bl_ref, m, H, W)
    print(f"[B g]_L rel {rel(bl, bl_ref):.2e}, image rel {rel(img, img_ref):.2e}")
    assert rel(bl, bl_ref) <= RTOL
    assert rel(img, img_ref) <= RTOL


def test_logpolar_of_a_phantom_matches_the_oracle():
    N, na = 128, 400
    nd = int(math.ceil(math.hypot(N, N))) + 4
    _, clean, _ = scenes.tomo_scene(N, N, na, nd, n_ellipses=8, noise=0.0, seed=31)
    print(f"case: logpolar phantom {N}x{N} angles {na} bins {nd}", flush=True)
    img, bl, _ = run(N, N, na, nd, clean)
    ref = lp.backproject_logpolar(clean.astype(np.float32).astype(np.float64), N, N)
    print(f"image rel {rel(img, ref):.2e}")
    assert rel(img, ref) <= RTOL


def test_logpolar_at_full_size():
    w = scenes.WORKLOADS["tomo_2048x1000"]
    H, W, na, nd = w["H"], w["W"], w["n_angles"], w["n_det"]
    print(f"case: logpolar {H}x{W} angles {na} bins {nd}", flush=True)
    _, clean, _ = scenes.tomo_scene(H, W, na, nd, w["n_ellipses"], 0.0, w["seed"])
    s = clean.astype(np.float32)
    img, bl, solver = run(H, W, na, nd, s)
    n_rho, n_phi, L, rho0, drho = solver.lp_mesh()
    m = lp.mesh(H, W, na, nd)
    assert (n_rho, n_phi, L) == (m.n_rho, m.n_phi, lp.conv_length(m)) == (8159, 2000, 16384)
    bl_ref = lp.logpolar_result(s.astype(np.float64), H, W)
    print(f"[B g]_L rel {rel(bl, bl_ref):.2e}", flush=True)
    assert rel(bl, bl_ref) <= RTOL
    img_ref = lp.to_cartesian(bl_ref, m, H, W)
    print(f"image rel {rel(img, img_ref):.2e}", flush=True)
    assert rel(img, img_ref) <= RTOL
    # against the exact backprojection, without the lines through the
    # innermost ring (the method's loss near the origin): within the
    # interpolation error of the two steps
    ref = (math.pi / na) * solver.backproject(to_dev(s)).cpu().numpy().astype(np.float64)
    x, y = tomo.pixel_centres(H, W)
    far = np.hypot(x, y) > 256
    print(f"far from the origin, against dtheta A^T: rel {rel(img[far], ref[far]):.2e}")
    assert rel(img[far], ref[far]) < 0.01


def test_workspace_planned_for_another_geometry_gives_nan():
    s = np.random.default_rng(1).normal(size=(30, 70)).astype(np.float32)
    a = tv.TomoSolver(37, 53, 30, 70, DEV)
    b = tv.TomoSolver(36, 53, 30, 70, DEV)
    ws, n = b._lp_ws()                    # planned for 36 x 53
    a._lp = (ws, n)
    img = a.logpolar(to_dev(s))
    torch.cuda.synchronize()
    assert torch.isnan(img).all()
