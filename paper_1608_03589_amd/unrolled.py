"""Unrolled (differentiable) solver with a hand-written adjoint.

``unrolled_tv(g, coeffs)`` runs K = coeffs.shape[0] iterations of the
primal-dual method on a batch of images [B, H, W] (or volumes [B, D, H, W])
with per-iteration coefficients coeffs[k] = (lam_k, tau_k, sigma_k), and is
differentiable with respect to g and coeffs through ``torch.autograd``; the
backward pass is the library's adjoint kernels, not autograd of torch ops.
"""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import Shape, call
from .solver import _stream, alloc_workspace, default_step, make_shape


def _shape_of(g: torch.Tensor) -> Shape:
    if g.dim() not in (3, 4):
        raise ValueError("g must be [B, H, W] or [B, D, H, W]")
    return make_shape(tuple(g.shape[1:]))


def set_fused_adjoint(on: bool):
    """Adjoint steps as one fused pass (the default) or as the two-pass
    reference; both give the same dL/dg bit for bit.  Process-wide."""
    call("tvpd_set_fused_adjoint", 1 if on else 0)


def default_coeffs(K: int, ndim: int, lam: float = 0.1, device="cuda"):
    s = default_step(ndim)
    c = torch.tensor([[lam, s, s]], dtype=torch.float32, device=device)
    return c.repeat(K, 1)


class UnrolledSolver:
    """Workspace-owning unrolled solver for a fixed batch shape."""

    def __init__(self, batch_shape, K: int, ckpt_every: int | None = None,
                 theta: float = 1.0, device="cuda"):
        self.batch_shape = tuple(int(v) for v in batch_shape)
        self.B = self.batch_shape[0]
        self.cshape = make_shape(self.batch_shape[1:])
        self.ndim = len(self.batch_shape) - 1
        self.K = int(K)
        self.ckpt = int(ckpt_every) if ckpt_every else self.K
        self.theta = float(theta)
        self.device = torch.device(device)
        n = C.c_size_t()
        call("tvpd_unrolled_workspace_size", C.byref(self.cshape), self.B,
             self.K, self.ckpt, C.byref(n))
        self.nbytes = n.value
        self.ws = alloc_workspace(self.nbytes, self.device)

    def _check(self, t, name, shape):
        if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")

    def forward(self, g: torch.Tensor, coeffs: torch.Tensor,
                out: torch.Tensor | None = None):
        self._check(g, "g", self.batch_shape)
        self._check(coeffs, "coeffs", (self.K, 3))
        f = torch.empty_like(g) if out is None else out
        call("tvpd_unrolled_forward", C.byref(self.cshape), self.B,
             C.c_void_p(g.data_ptr()), C.c_void_p(coeffs.data_ptr()), self.K,
             self.ckpt, C.c_float(self.theta), C.c_void_p(f.data_ptr()),
             C.c_void_p(self.ws.data_ptr()), self.nbytes,
             C.c_void_p(_stream(self.device)))
        return f

    def backward(self, coeffs: torch.Tensor, grad_f: torch.Tensor):
        self._check(coeffs, "coeffs", (self.K, 3))
        grad_f = grad_f.contiguous()
        self._check(grad_f, "grad_f", self.batch_shape)
        grad_g = torch.empty_like(grad_f)
        grad_c = torch.empty((self.K, 3), dtype=torch.float32, device=self.device)
        call("tvpd_unrolled_backward", C.byref(self.cshape), self.B,
             C.c_void_p(coeffs.data_ptr()), self.K, self.ckpt,
             C.c_float(self.theta), C.c_void_p(grad_f.data_ptr()),
             C.c_void_p(grad_g.data_ptr()), C.c_void_p(grad_c.data_ptr()),
             C.c_void_p(self.ws.data_ptr()), self.nbytes,
             C.c_void_p(_stream(self.device)))
        return grad_g, grad_c


class UnrolledTV(torch.autograd.Function):
    """f^K = unrolled(g, coeffs); backward by the library's adjoint."""

    @staticmethod
    def forward(ctx, g, coeffs, ckpt_every, theta):
        g = g.contiguous()
        coeffs = coeffs.contiguous()
        solver = UnrolledSolver(tuple(g.shape), coeffs.shape[0], ckpt_every,
                                theta, g.device)
        f = solver.forward(g, coeffs)
        ctx.solver = solver
        ctx.save_for_backward(coeffs)
        return f

    @staticmethod
    def backward(ctx, grad_f):
        (coeffs,) = ctx.saved_tensors
        if ctx.solver is None:
            raise RuntimeError(
                "UnrolledTV: a second backward through the same graph is not "
                "supported (the forward states were released after the first)")
        grad_g, grad_c = ctx.solver.backward(coeffs, grad_f)
        ctx.solver = None  # release the workspace
        return grad_g, grad_c, None, None


def unrolled_tv(g: torch.Tensor, coeffs: torch.Tensor,
                ckpt_every: int | None = None, theta: float = 1.0):
    """Differentiable K-iteration solver; see :class:`UnrolledTV`."""
    return UnrolledTV.apply(g, coeffs, ckpt_every, theta)
