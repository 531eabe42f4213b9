"""Build the HIP library ``libtvpd.so`` in-tree for gfx950.

    python -m paper_1608_03589_amd.build

compiles every ``csrc/*.hip`` with hipcc into an object (in parallel, under
``paper_1608_03589_amd/_build/``) and links them into
``paper_1608_03589_amd/libtvpd.so``.  ``host_asan=True`` builds a variant whose
host code carries AddressSanitizer (the device code is the same as the
product's; GPU code is never built with a sanitizer).
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtvpd.so")
OBJ_DIR = os.path.join(PKG, "_build")

ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # identical arithmetic in every kernel that shares a device function:
    # no implicit multiply-add contraction
    "-ffp-contract=off",
    # no packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
# host-side AddressSanitizer: each flag applies to the host compilation only
HOST_ASAN = ["-g", "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fno-omit-frame-pointer"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libtvpd.so)")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed with status {r.returncode}: {cmd[-1]}")


def build(verbose: bool = False, out: str | None = None, host_asan: bool = False,
          obj_dir: str | None = None, jobs: int | None = None) -> str:
    """Compile every source to an object, in parallel, and link the library.

    Returns the path of the library (``out``, by default the in-tree
    ``libtvpd.so``, replaced atomically)."""
    out = out or LIB
    obj_dir = obj_dir or (OBJ_DIR + ("_asan" if host_asan else ""))
    os.makedirs(obj_dir, exist_ok=True)
    extra = HOST_ASAN if host_asan else []
    cc = hipcc()
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = [os.path.join(obj_dir, os.path.basename(s)[:-4] + ".o") for s in srcs]
    jobs = jobs or max(1, min(len(srcs), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_run, [cc, "-c", *FLAGS, *extra, f"-I{INCLUDE}", f"-I{CSRC}",
                                 src, "-o", obj], verbose)
                for src, obj in zip(srcs, objs)]
        for f in futs:
            f.result()
    tmp = out + ".tmp"
    _run([cc, "-shared", *FLAGS, *extra, *objs, "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
