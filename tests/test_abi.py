"""The C ABI without a GPU: symbols, signatures and argument validation.

Validation runs before any HIP call, so every error path here is reachable
on a machine without a GPU.
"""
import ctypes as C
import os
import re

import pytest

from paper_1608_03589_amd import _lib
from paper_1608_03589_amd._lib import Coeffs, Params, Result, Shape

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tvpd.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tvpd_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def test_every_declared_symbol_is_exported_and_bound(L):
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L, n), n
        assert n in _lib.SIGNATURES, f"{n} has no ctypes signature"


def test_status_strings(L):
    assert L.tvpd_status_string(0) == b"ok"
    for code in range(-9, 0):
        s = L.tvpd_status_string(code)
        assert s and s != b"unknown status"
    assert L.tvpd_status_string(12345) == b"unknown status"
    assert L.tvpd_version() >= 10000


def test_struct_layouts():
    assert C.sizeof(Shape) == 16
    assert C.sizeof(Coeffs) == 16
    assert C.sizeof(Params) == 40
    assert Params.gap_tol.offset == 24
    assert C.sizeof(Result) == 32


def _ws(shape):
    n = C.c_size_t()
    st = _lib.lib().tvpd_workspace_size(C.byref(shape), C.byref(n))
    return st, n.value


def test_workspace_size_grows_and_validates():
    # 7 planes: two slots of f and of the dual (x, y), and g; a pass reads one
    # slot and writes the other (the sweep keeps no f^{k-1})
    st, a = _ws(Shape(2, 1, 256, 256))
    assert st == 0 and a >= 7 * 256 * 256 * 4
    st, b = _ws(Shape(2, 1, 4096, 4096))
    assert st == 0 and b >= 7 * 4096 * 4096 * 4 and b < 7.1 * 4096 * 4096 * 4
    st, c = _ws(Shape(2, 1, 7, 5))   # ragged: pitch rounds 5 up to 8
    assert st == 0 and c >= 7 * 7 * 8 * 4
    # 3D: 10 planes (f ring of 3, dual ring of 2 x 3, g)
    st, d = _ws(Shape(3, 32, 32, 32))
    assert st == 0 and d >= 10 * 32 ** 3 * 4 and d < 10.5 * 32 ** 3 * 4
    for bad in [Shape(2, 2, 4, 4), Shape(4, 1, 4, 4), Shape(2, 1, 0, 4),
                Shape(2, 1, 4, -1), Shape(3, 0, 4, 4)]:
        assert _ws(bad)[0] == -2
    assert _lib.lib().tvpd_workspace_size(C.byref(Shape(2, 1, 4, 4)), None) == -1


def _solve(shape, prm, ws, nbytes, g=0x1000, f=0x2000):
    return _lib.lib().tvpd_solve(C.byref(shape), C.c_void_p(g), C.c_void_p(f),
                                 C.byref(prm), C.c_void_p(ws), nbytes,
                                 C.byref(Result()), None)


def test_solve_argument_errors_before_any_device_call():
    sh = Shape(2, 1, 64, 64)
    _, need = _ws(sh)
    s = 1 / 8 ** 0.5
    good = Params(Coeffs(0.1, s, s, 1.0), 100, 10, 1e-4, -1, 0)
    aligned = 1 << 20
    assert _solve(Shape(2, 1, 0, 4), good, aligned, need) == -2
    assert _solve(sh, good, 0, need) == -1                      # null ws
    assert _solve(sh, good, aligned, need, g=0) == -1            # null g
    assert _solve(sh, good, aligned + 16, need) == -3            # misaligned
    assert _solve(sh, good, aligned, need - 1) == -4             # too small
    bad_step = Params(Coeffs(0.1, 0.5, 0.5, 1.0), 100, 10, 1e-4, -1, 0)
    assert _solve(sh, bad_step, aligned, need) == -7
    neg_lam = Params(Coeffs(-0.1, s, s, 1.0), 100, 10, 1e-4, -1, 0)
    assert _solve(sh, neg_lam, aligned, need) == -1
    bad_theta = Params(Coeffs(0.1, s, s, 1.5), 100, 10, 1e-4, -1, 0)
    assert _solve(sh, bad_theta, aligned, need) == -1
    neg_iter = Params(Coeffs(0.1, s, s, 1.0), -1, 10, 1e-4, -1, 0)
    assert _solve(sh, neg_iter, aligned, need) == -1
    nan_tol = Params(Coeffs(0.1, s, s, 1.0), 10, 10, float("nan"), -1, 0)
    assert _solve(sh, nan_tol, aligned, need) == -1


def test_step_bound_is_the_grid_norm():
    """tau sigma ||grad||^2 < 1 is checked with the exact grid norm: on a
    2 x 2 image ||grad||^2 = 4, so tau = sigma = 0.49 passes and 0.51 fails."""
    sh = Shape(2, 1, 2, 2)
    _, need = _ws(sh)
    L = _lib.lib()
    ok = Coeffs(0.1, 0.49, 0.49, 1.0)
    bad = Coeffs(0.1, 0.51, 0.51, 1.0)
    # tvpd_step validates coefficients before touching the workspace
    assert L.tvpd_step(C.byref(sh), C.byref(bad), 1, C.c_void_p(1 << 20), need,
                       None) == -7
    assert L.tvpd_step(C.byref(sh), C.byref(ok), -1, C.c_void_p(1 << 20), need,
                       None) == -1


def test_loud_failure_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.lib()


def test_tomo_validation_without_gpu(L):
    from paper_1608_03589_amd._lib import TomoGeom, TomoParams
    assert C.sizeof(TomoGeom) == 16 and C.sizeof(TomoParams) == 24
    n = C.c_size_t()
    good = TomoGeom(64, 48, 30, 90)
    assert L.tvpd_tomo_workspace_size(C.byref(good), C.byref(n)) == 0
    assert n.value > 4 * 64 * 48 * 8
    for bad in (TomoGeom(0, 4, 4, 4), TomoGeom(4, 4, 0, 4), TomoGeom(4, 4, 4, 0),
                TomoGeom(40000, 4, 4, 4), TomoGeom(4, 4, 70000, 4)):
        assert L.tvpd_tomo_workspace_size(C.byref(bad), C.byref(n)) == -2
    assert L.tvpd_tomo_workspace_size(None, C.byref(n)) == -2
    dummy = C.c_void_p(256)
    ok = TomoParams(0.1, 0.01, 0.01, 1.0, 1.0, 0)
    # parameters are checked before the workspace (and before any HIP call)
    for prm, code in ((TomoParams(0.1, 0.0, 0.01, 1.0, 1.0, 0), -7),
                      (TomoParams(0.1, 0.01, -1.0, 1.0, 1.0, 0), -7),
                      (TomoParams(0.1, 0.01, 0.01, 0.0, 1.0, 0), -7),
                      (TomoParams(-0.1, 0.01, 0.01, 1.0, 1.0, 0), -1),
                      (TomoParams(0.1, 0.01, 0.01, 1.0, 1.5, 0), -1),
                      (TomoParams(0.1, 0.01, 0.01, 1.0, 1.0, 7), -1)):
        assert L.tvpd_tomo_step(C.byref(good), dummy, C.byref(prm), 1, None, 0,
                                None) == code
    # Tikhonov ignores sigma_p
    tik = TomoParams(0.1, 0.01, 0.01, 0.0, 1.0, 1)
    assert L.tvpd_tomo_step(C.byref(good), dummy, C.byref(tik), 1, None, 0, None) == -1
    assert L.tvpd_tomo_step(C.byref(good), dummy, C.byref(ok), -1, None, 0, None) == -1
    assert L.tvpd_tomo_step(C.byref(good), None, C.byref(ok), 1, None, 0, None) == -1
    assert L.tvpd_tomo_step(C.byref(good), dummy, C.byref(ok), 1, C.c_void_p(256 + 8),
                            1 << 40, None) == -3
    assert L.tvpd_tomo_step(C.byref(good), dummy, C.byref(ok), 1, dummy, 16,
                            None) == -4
    assert L.tvpd_radon_forward(C.byref(good), None, dummy, dummy, 1 << 40, None) == -1
    assert L.tvpd_radon_backward(C.byref(good), dummy, None, dummy, 1 << 40, None) == -1
    out = C.c_double()
    assert L.tvpd_tomo_opnorm(C.byref(good), 0, dummy, 1 << 40, C.byref(out), None) == -1
    assert L.tvpd_fbp(C.byref(good), dummy, -1.0, dummy, dummy, 1 << 40, None) == -1
    assert L.tvpd_fbp(C.byref(good), None, 0.0, dummy, dummy, 1 << 40, None) == -1
    assert L.tvpd_fbp(C.byref(good), dummy, 0.0, dummy, dummy, 16, None) == -4
    res = (C.c_double * 3)()
    assert L.tvpd_tomo_energy(C.byref(good), dummy, 0.1, 5, dummy, 1 << 40, res,
                              None) == -1


def test_bst_validation_without_gpu(L):
    from paper_1608_03589_amd._lib import TomoGeom
    good = TomoGeom(64, 48, 30, 90)
    M, Q = C.c_int32(), C.c_int32()
    assert L.tvpd_bst_lengths(C.byref(good), C.byref(M), C.byref(Q)) == 0
    assert (M.value, Q.value) == (256, 128)
    n = C.c_size_t()
    assert L.tvpd_bst_workspace_size(C.byref(good), C.byref(n)) == 0
    # lengths beyond the LDS transforms: n_det 2049 needs M = 8192
    big = TomoGeom(64, 48, 30, 2049)
    assert L.tvpd_bst_workspace_size(C.byref(big), C.byref(n)) == -6
    dummy = C.c_void_p(256)
    # the regularisation weight is checked first, then shape, pointers and
    # workspace, all before any HIP call
    for lam in (-1.0, float("nan"), float("inf"), -1e-30):
        assert L.tvpd_fbp_bst(C.byref(good), dummy, lam, dummy, dummy, 1 << 40, None) == -1
    assert L.tvpd_fbp_bst(C.byref(TomoGeom(0, 4, 4, 4)), dummy, 1.0, dummy, dummy, 1 << 40,
                          None) == -2
    assert L.tvpd_fbp_bst(C.byref(good), None, 1.0, dummy, dummy, 1 << 40, None) == -1
    assert L.tvpd_fbp_bst(C.byref(good), dummy, 1.0, None, dummy, 1 << 40, None) == -1
    assert L.tvpd_fbp_bst(C.byref(good), dummy, 1.0, dummy, None, 1 << 40, None) == -1
    assert L.tvpd_fbp_bst(C.byref(good), dummy, 1.0, dummy, C.c_void_p(256 + 8), 1 << 40,
                          None) == -3
    assert L.tvpd_fbp_bst(C.byref(good), dummy, 1.0, dummy, dummy, 16, None) == -4
    assert L.tvpd_fbp_bst(C.byref(big), dummy, 1.0, dummy, dummy, 1 << 40, None) == -6
    assert L.tvpd_bst_backproject(C.byref(good), dummy, dummy, dummy, 16, None) == -4


def test_batch_workspace_size_bounds_the_tile_tables(L):
    from paper_1608_03589_amd._lib import Shape
    n = C.c_size_t()
    ok = (Shape * 2)(Shape(2, 1, 300, 700), Shape(2, 1, 17, 5))
    assert L.tvpd_batch_workspace_size(2, ok, C.byref(n)) == 0
    # the arena alone: 8 planes (three f slots, two dual slots of x and y, g)
    # of 300 x 700 and of 17 x 8 (pitch) floats
    assert n.value > 8 * 4 * (300 * 700 + 17 * 8)
    # 4 tile tables of one entry per row and 256-column strip must fit int32
    big = (Shape * 1)(Shape(2, 1, 1 << 20, 1 << 20))
    assert L.tvpd_batch_workspace_size(1, big, C.byref(n)) == -6
    assert L.tvpd_batch_workspace_size(0, ok, C.byref(n)) == -2
    assert L.tvpd_batch_workspace_size(2, ok, None) == -1


def test_noalloc_fbp_refuses_requests_beyond_the_scratch(L):
    # refused on the host before any device work: runs without a GPU
    geom = _lib.TomoGeom(16, 16, 4096, 2048)      # 8.4 M bins > 8093696
    dummy = C.c_void_p(256)
    assert L.tvpd_fbp_noalloc(C.byref(geom), dummy, C.c_float(0.0), dummy, None) == -9
    assert L.tvpd_fbp_noalloc(C.byref(geom), None, C.c_float(0.0), dummy, None) == -1


@pytest.mark.parametrize("H,W,na,nd", [(64, 64, 48, 92), (33, 21, 45, 40), (2048, 2048, 1000, 2048),
                                       (724, 724, 180, 1024), (5, 7, 1, 4)])
def test_logpolar_mesh_equals_the_oracle(L, H, W, na, nd):
    # host-only call: the library's mesh is the oracle's, node for node
    from oracle import logpolar as lp
    m = lp.mesh(H, W, na, nd)
    n_rho, n_phi, Lr = C.c_int32(), C.c_int32(), C.c_int32()
    rho0, drho = C.c_double(), C.c_double()
    st = L.tvpd_lp_mesh(C.byref(_lib.TomoGeom(H, W, na, nd)), C.byref(n_rho), C.byref(n_phi),
                        C.byref(Lr), C.byref(rho0), C.byref(drho))
    assert st == 0
    assert (n_rho.value, n_phi.value, Lr.value) == (m.n_rho, m.n_phi, lp.conv_length(m))
    assert rho0.value == pytest.approx(m.rho0, rel=1e-15)
    assert drho.value == pytest.approx(m.drho, rel=1e-14)


def test_logpolar_limits(L):
    n = C.c_size_t()
    # 14 rays: a prime factor 7
    assert L.tvpd_lp_workspace_size(C.byref(_lib.TomoGeom(16, 16, 7, 40)), C.byref(n)) == -6
    # N_rho beyond 8192
    assert L.tvpd_lp_workspace_size(C.byref(_lib.TomoGeom(16, 16, 8, 4096)), C.byref(n)) == -6
    assert L.tvpd_lp_workspace_size(C.byref(_lib.TomoGeom(16, 16, 8, 3)), C.byref(n)) == -6
    assert L.tvpd_lp_workspace_size(C.byref(_lib.TomoGeom(16, 16, 8, 40)), C.byref(n)) == 0


def test_tile_and_depth_settings_are_validated(L):
    # host-side settings: no GPU needed
    from paper_1608_03589_amd._lib import Shape
    s = Shape(2, 1, 300, 517)
    th, wpb, order = C.c_int32(), C.c_int32(), C.c_int32()
    # the pipelined passes (order 2) take any wpb; the walks 1, 2 or 4
    assert L.tvpd_set_tile(C.byref(s), 300, 0, 2) == 0
    assert L.tvpd_get_tile(C.byref(s), C.byref(th), C.byref(wpb), C.byref(order)) == 0
    assert (th.value, order.value) == (300, 2)
    assert L.tvpd_set_tile(C.byref(s), 8, 3, 0) == -1
    assert L.tvpd_set_tile(C.byref(s), 8, 4, 3) == -1
    assert L.tvpd_set_tile(C.byref(s), 0, 1, 2) == -1
    assert L.tvpd_set_tile(C.byref(s), 8, 4, 1) == 0
    d = C.c_int32()
    assert L.tvpd_get_pass_depth(C.byref(d)) == 0
    old = d.value
    try:
        for ok in (0, 1, 6, 10):
            assert L.tvpd_set_pass_depth(ok) == 0
            assert L.tvpd_get_pass_depth(C.byref(d)) == 0 and d.value == ok
        for bad in (-1, 11):
            assert L.tvpd_set_pass_depth(bad) == -1
        assert L.tvpd_set_blocking(0) == 0
        assert L.tvpd_get_pass_depth(C.byref(d)) == 0 and d.value == 1
        assert L.tvpd_set_blocking(1) == 0
        assert L.tvpd_get_pass_depth(C.byref(d)) == 0 and d.value == 0
        assert L.tvpd_set_wait_limit(-1) == -1
        assert L.tvpd_set_wait_limit(5) == 0
        assert L.tvpd_set_projection_staging(2) == -1
        assert L.tvpd_set_projection_staging(-1) == -1
        assert L.tvpd_set_projection_staging(0) == 0
    finally:
        L.tvpd_set_pass_depth(old)
        L.tvpd_set_wait_limit(0)
        L.tvpd_set_projection_staging(1)


def test_stream_copy_validates(L):
    # host-side checks only: no device memory is touched
    P = C.c_void_p
    assert L.tvpd_stream_copy(None, P(256), 4, None) == -1
    assert L.tvpd_stream_copy(P(256), None, 4, None) == -1
    assert L.tvpd_stream_copy(P(256), P(512), 6, None) == -1      # not a multiple of 4
    assert L.tvpd_stream_copy(P(256), P(512), 0, None) == -1
    assert L.tvpd_stream_copy(P(260), P(512), 4, None) == -1      # misaligned
