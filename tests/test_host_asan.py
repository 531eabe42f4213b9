"""Host code under AddressSanitizer (no GPU needed).

The library is rebuilt with AddressSanitizer on its host code only (argument
checks, layouts, tile tables, the tuning-cache parser); a fresh interpreter
with the sanitizer runtime preloaded then drives every host-only entry point
with valid, degenerate and invalid arguments.  Any invalid memory access
aborts that process with a report; the test requires a clean exit.
"""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

from paper_1608_03589_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    pats = ["/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so",
            "/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"]
    for p in pats:
        hits = sorted(glob.glob(p))
        if hits:
            return hits[-1]
    return None


DRIVER = textwrap.dedent(r'''
    import ctypes as C, sys
    sys.path.insert(0, ROOT)
    from paper_1608_03589_amd import _lib as T
    L = C.CDLL(LIB)
    for name, (res, args) in T.SIGNATURES.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    n = C.c_size_t()
    S = T.Shape
    for code in range(-12, 3):
        assert L.tvpd_status_string(code)
    shapes = [S(2, 1, 1, 1), S(2, 1, 1, 4096), S(2, 1, 4096, 1), S(2, 1, 300, 517),
              S(3, 1, 1, 1), S(3, 7, 9, 266), S(3, 256, 256, 256), S(1, 1, 5, 5),
              S(2, 1, 0, 5), S(2, 1, -3, 5), S(3, 0, 4, 4), S(2, 1, 1 << 30, 1 << 30)]
    for s in shapes:
        L.tvpd_workspace_size(C.byref(s), C.byref(n))
        L.tvpd_workspace_size(C.byref(s), None)
        for K in (0, 1, 7, 100):
            for ck in (0, 1, 3, 1000):
                L.tvpd_unrolled_workspace_size(C.byref(s), 2, K, ck, C.byref(n))
        th, wpb, o = C.c_int32(), C.c_int32(), C.c_int32()
        L.tvpd_set_tile(C.byref(s), 8, 4, 0)
        L.tvpd_get_tile(C.byref(s), C.byref(th), C.byref(wpb), C.byref(o))
        L.tvpd_set_tile3d(C.byref(s), 4, 16, 4)
        L.tvpd_get_tile3d(C.byref(s), C.byref(th), C.byref(wpb), C.byref(o))
    L.tvpd_workspace_size(None, C.byref(n))
    for lst in ([S(2, 1, 1, 1)], [S(2, 1, 300, 700), S(2, 1, 17, 5), S(2, 1, 1, 1)],
                [S(2, 1, h, w) for h, w in zip(range(1, 200, 7), range(300, 1, -11))],
                [S(2, 1, 1 << 20, 1 << 20)], [S(3, 2, 2, 2)]):
        arr = (S * len(lst))(*lst)
        L.tvpd_batch_workspace_size(len(lst), arr, C.byref(n))
    L.tvpd_batch_workspace_size(0, None, C.byref(n))
    G = T.TomoGeom
    for g in (G(16, 16, 4, 8), G(2048, 2048, 1000, 2048), G(5, 7, 1, 4), G(0, 4, 4, 4),
              G(33, 21, 45, 40), G(16, 16, 4096, 2048)):
        L.tvpd_tomo_workspace_size(C.byref(g), C.byref(n))
        a, b = C.c_int32(), C.c_int32()
        L.tvpd_bst_lengths(C.byref(g), C.byref(a), C.byref(b))
        L.tvpd_bst_workspace_size(C.byref(g), C.byref(n))
        nr, nphi, lr = C.c_int32(), C.c_int32(), C.c_int32()
        r0, dr = C.c_double(), C.c_double()
        L.tvpd_lp_mesh(C.byref(g), C.byref(nr), C.byref(nphi), C.byref(lr), C.byref(r0),
                       C.byref(dr))
        L.tvpd_lp_workspace_size(C.byref(g), C.byref(n))
        L.tvpd_fbp_noalloc(C.byref(g), None, 0.0, None, None)
    for d in (0, 1, 5, 6, 7, -1):
        L.tvpd_set_pass_depth(d)
    dd = C.c_int32()
    L.tvpd_get_pass_depth(C.byref(dd))
    L.tvpd_set_pass_depth(5)
    L.tvpd_set_blocking(1)
    L.tvpd_set_fused_adjoint(1)
    # invalid arguments of compute entry points are refused before any device work
    s = S(2, 1, 64, 64)
    prm = T.Params(T.Coeffs(0.1, 0.3, 0.3, 1.0), 10, 10, 1e-4, 0, 0)
    L.tvpd_init(C.byref(s), None, None, 0, None)
    L.tvpd_step(C.byref(s), None, 1, None, 0, None)
    L.tvpd_solve(C.byref(s), None, None, C.byref(prm), None, 0, None, None)
    L.tvpd_solve(C.byref(s), C.c_void_p(256), C.c_void_p(256), None, C.c_void_p(256), 1, None, None)
    L.tvpd_solve_batched(0, None, None, None, None, None, None, None, 0, None, None)
    # the tuning-cache parser on malformed, truncated and overlong lines
    cache = CACHE
    with open(cache, "w") as fh:
        fh.write("gfx950 2 1 64 64 8 4 0 1.5\n")
        fh.write("gfx950 2 1 64\n")
        fh.write("x" * 5000 + "\n")
        fh.write("gfx950 3 7 9 266 4 4 16 2.0 extra tokens\n")
        fh.write("gfx950 2 1 64 64 -1 3 7 nan\n")
        fh.write("\n\n" + "y" * 700)
    cnt = C.c_int32()
    L.tvpd_tune_load(cache.encode(), C.byref(cnt))
    L.tvpd_tune_load(b"/nonexistent/cache/file", C.byref(cnt))
    L.tvpd_release_thread_resources()
    print("host paths done", flush=True)
''')


def test_host_code_under_address_sanitizer(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this ROCm install")
    try:
        lib = B.build(out=str(tmp_path / "libtvpd_asan.so"), host_asan=True,
                      obj_dir=str(tmp_path / "obj"))
    except RuntimeError as e:  # no hipcc: nothing to check here
        pytest.skip(str(e))
    script = (f"ROOT = {ROOT!r}\nLIB = {lib!r}\nCACHE = {str(tmp_path / 'tune.txt')!r}\n"
              + DRIVER)
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt + ((":" + env["LD_PRELOAD"]) if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:exitcode=23:abort_on_error=0"
    env["HIP_VISIBLE_DEVICES"] = ""   # host paths only, also on a machine with a GPU
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True,
                       text=True, timeout=600)
    report = r.stdout + r.stderr
    assert "AddressSanitizer" not in report, report[-4000:]
    assert r.returncode == 0 and "host paths done" in r.stdout, report[-4000:]
