"""Batched solver: many images of different sizes solved together on the
device, each exactly as :class:`PlainSolver` would solve it alone.

PyTorch supplies the arenas and the workspace; ``libtvpd.so`` does the work.
"""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import BatchOpts, Params, Result, Shape, call
from .solver import (SolveResult, _check_image, _stream, alloc_workspace,
                     default_step, make_shape)

MODES = {"persistent": 0, "graph": 1, "launches": 2}


class BatchedSolver:
    """Solver for a fixed list of 2D shapes.

    ``solve(images, ...)`` takes a list of float32 CUDA tensors (one per
    shape) and returns the list of solutions and of :class:`SolveResult`.
    """

    def __init__(self, shapes, device="cuda"):
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        if not self.shapes or any(len(s) != 2 for s in self.shapes):
            raise ValueError("the batched solver takes a non-empty list of 2D shapes")
        self.n = len(self.shapes)
        self.cshapes = (Shape * self.n)(*[make_shape(s) for s in self.shapes])
        self.device = torch.device(device)
        offs, o = [], 0
        for h, w in self.shapes:
            offs.append(o)
            o += h * w
        self.total = o
        self.offsets = (C.c_int64 * self.n)(*offs)
        self._offs = offs
        nbytes = C.c_size_t()
        call("tvpd_batch_workspace_size", self.n, self.cshapes, C.byref(nbytes))
        self.nbytes = nbytes.value
        self.ws = alloc_workspace(self.nbytes, self.device)
        self.g_arena = torch.empty(self.total, dtype=torch.float32, device=self.device)
        self.f_arena = torch.empty_like(self.g_arena)

    def pack(self, images):
        if len(images) != self.n:
            raise ValueError(f"expected {self.n} images, got {len(images)}")
        for i, (im, s) in enumerate(zip(images, self.shapes)):
            _check_image(im, f"images[{i}]")
            if tuple(im.shape) != s:
                raise ValueError(f"images[{i}] has shape {tuple(im.shape)}, expected {s}")
            o = self._offs[i]
            self.g_arena[o:o + s[0] * s[1]].copy_(im.reshape(-1))

    def unpack(self):
        return [self.f_arena[o:o + h * w].view(h, w)
                for o, (h, w) in zip(self._offs, self.shapes)]

    def _params(self, lam, tau, sigma, theta, max_iter, check_every, gap_tol):
        def per(v, i):
            return v[i] if isinstance(v, (list, tuple)) else v
        s = default_step(2)
        ps = []
        for i in range(self.n):
            t = per(tau, i)
            sg = per(sigma, i)
            ps.append(Params((float(per(lam, i)), float(s if t is None else t),
                              float(s if sg is None else sg), float(per(theta, i))),
                             int(max_iter), int(check_every), float(per(gap_tol, i)),
                             -1, 0))
        return (Params * self.n)(*ps)

    def solve(self, images=None, lam=0.1, tau=None, sigma=None, theta=1.0,
              max_iter=20000, check_every=10, gap_tol=1e-4, mode="persistent",
              th=0, wpb=0, th_short=0):
        """Solve every image; ``images=None`` reuses the packed arena."""
        if images is not None:
            self.pack(images)
        prm = self._params(lam, tau, sigma, theta, max_iter, check_every, gap_tol)
        opts = BatchOpts(MODES[mode] if isinstance(mode, str) else int(mode),
                         int(th), int(wpb), int(th_short))
        res = (Result * self.n)()
        call("tvpd_solve_batched", self.n, self.cshapes, self.offsets,
             C.c_void_p(self.g_arena.data_ptr()), C.c_void_p(self.f_arena.data_ptr()),
             prm, C.byref(opts), C.c_void_p(self.ws.data_ptr()), self.nbytes, res,
             C.c_void_p(_stream(self.device)))
        return self.unpack(), [SolveResult(r.iters, bool(r.converged), r.primal,
                                           r.dual, r.gap) for r in res]

    def autotune(self, images=None, lam=0.1, tau=None, sigma=None, theta=1.0):
        """Pick the batch tile (rows per band, waves per block) by timing;
        the choice becomes the default for later solves in this process."""
        if images is not None:
            self.pack(images)
        prm = self._params(lam, tau, sigma, theta, 30, 10, -1.0)
        th, wpb, ms = C.c_int32(), C.c_int32(), C.c_float()
        call("tvpd_batch_autotune", self.n, self.cshapes, self.offsets,
             C.c_void_p(self.g_arena.data_ptr()), C.c_void_p(self.f_arena.data_ptr()),
             prm, C.c_void_p(self.ws.data_ptr()), self.nbytes, C.byref(th),
             C.byref(wpb), C.byref(ms), C.c_void_p(_stream(self.device)))
        return (th.value, wpb.value), ms.value
