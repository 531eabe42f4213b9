"""The allocation-free FBP entry point (tvpd_fbp_noalloc) against tvpd_fbp.

Both run the same kernels, so the results must agree bit for bit; two calls in
a row, the second on a smaller geometry, show that the shared static scratch
keeps no state between calls.  Requests beyond the scratch are refused.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_1608_03589_amd as tv
from paper_1608_03589_amd import _lib
from scenes import tomo_scene

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def noalloc_call(sino, ny, nx, lam):
    out = torch.full((ny, nx), float("nan"), dtype=torch.float32, device=DEV)
    geom = _lib.TomoGeom(ny, nx, sino.shape[0], sino.shape[1])
    st = _lib.lib().tvpd_fbp_noalloc(
        C.byref(geom), C.c_void_p(sino.data_ptr()), C.c_float(lam),
        C.c_void_p(out.data_ptr()),
        C.c_void_p(torch.cuda.current_stream(DEV).cuda_stream))
    assert st == 0, _lib.lib().tvpd_status_string(st)
    return out


def test_noalloc_fbp_equals_fbp_on_two_calls():
    cases = [(256, 240, 300, 370, 2.5), (64, 80, 45, 96, 0.0)]
    for ny, nx, na, nd, lam in cases:
        print(f"case: fbp_noalloc {ny}x{nx}, {na} angles, {nd} bins, lam {lam}",
              flush=True)
        _, clean, _ = tomo_scene(ny, nx, na, nd, n_ellipses=6, noise=0.0, seed=ny)
        sino = torch.from_numpy(clean.astype(np.float32)).to(DEV)
        got = noalloc_call(sino, ny, nx, lam)
        ref = tv.TomoSolver(ny, nx, na, nd, DEV).fbp(sino, lam)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref)
    # the package wrapper reaches the same entry point
    wrapped = tv.fbp_noalloc(sino, ny, nx, lam)
    assert torch.equal(wrapped, ref)


def test_noalloc_fbp_refuses_requests_beyond_the_scratch():
    geom = _lib.TomoGeom(16, 16, 4096, 2048)      # 8.4 M bins > 8093696
    dummy = C.c_void_p(256)
    st = _lib.lib().tvpd_fbp_noalloc(C.byref(geom), dummy, C.c_float(0.0), dummy,
                                     None)
    assert st == -9
    assert _lib.lib().tvpd_status_string(st) == b"request exceeds the static scratch area"
