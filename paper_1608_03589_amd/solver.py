"""Python face of the plain solver: torch tensors in, torch tensors out.

PyTorch supplies device memory and the current stream; every computation is
done by ``libtvpd.so``.  The problem solved is

    min_f  1/2 ||f - g||^2 + lam * TV(f)

(the paper's regularised problem of Section 6, eq. opt, with identity forward
operator and total-variation regulariser) by the first-order primal-dual
iteration; see ``include/tvpd.h`` for the exact definitions.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import torch

from ._lib import Coeffs, Params, Result, Shape, call

WS_ALIGN = 256


def default_step(ndim: int) -> float:
    """tau = sigma = 1/sqrt(4 ndim): tau sigma ||grad||^2 < 1 on any grid."""
    return 1.0 / math.sqrt(4.0 * ndim)


def make_shape(shape) -> Shape:
    shape = tuple(int(s) for s in shape)
    if len(shape) == 2:
        return Shape(2, 1, shape[0], shape[1])
    if len(shape) == 3:
        return Shape(3, shape[0], shape[1], shape[2])
    raise ValueError(f"expected a 2D or 3D shape, got {shape}")


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_image(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def alloc_workspace(nbytes: int, device) -> torch.Tensor:
    """A uint8 device buffer whose data pointer is 256-byte aligned."""
    buf = torch.empty(nbytes + WS_ALIGN, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % WS_ALIGN
    return buf[off:off + nbytes]


def workspace_size(shape) -> int:
    n = C.c_size_t()
    call("tvpd_workspace_size", C.byref(make_shape(shape)), C.byref(n))
    return n.value


@dataclass
class SolveResult:
    iters: int
    converged: bool
    primal: float
    dual: float
    gap: float

    @property
    def rel_gap(self) -> float:
        return self.gap / self.primal if self.primal > 0 else 0.0


class PlainSolver:
    """Solver state for one image (2D) or volume (3D) of a fixed shape.

    The workspace (allocated once, reused across calls) holds the iterate
    ring, the dual ring, a padded copy of g and the reduction scratch.
    """

    def __init__(self, shape, device="cuda"):
        self.shape = tuple(int(s) for s in shape)
        self.cshape = make_shape(self.shape)
        self.device = torch.device(device)
        self.nbytes = workspace_size(self.shape)
        self.ws = alloc_workspace(self.nbytes, self.device)

    # -- state ------------------------------------------------------------
    def init(self, g: torch.Tensor):
        _check_image(g, "g")
        if tuple(g.shape) != self.shape:
            raise ValueError(f"g has shape {tuple(g.shape)}, expected {self.shape}")
        call("tvpd_init", C.byref(self.cshape), C.c_void_p(g.data_ptr()),
             C.c_void_p(self.ws.data_ptr()), self.nbytes, C.c_void_p(_stream(self.device)))

    def step(self, n_iter: int, lam: float, tau: float | None = None,
             sigma: float | None = None, theta: float = 1.0):
        c = self._coeffs(lam, tau, sigma, theta)
        call("tvpd_step", C.byref(self.cshape), C.byref(c), int(n_iter),
             C.c_void_p(self.ws.data_ptr()), self.nbytes, C.c_void_p(_stream(self.device)))

    def state(self, with_dual: bool = True):
        f = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        p = (torch.empty((len(self.shape),) + self.shape, dtype=torch.float32,
                         device=self.device) if with_dual else None)
        call("tvpd_read_state", C.byref(self.cshape), C.c_void_p(self.ws.data_ptr()),
             self.nbytes, C.c_void_p(f.data_ptr()),
             C.c_void_p(p.data_ptr() if p is not None else None),
             C.c_void_p(_stream(self.device)))
        return (f, p) if with_dual else f

    def iteration(self) -> int:
        k = C.c_int32()
        call("tvpd_iteration", C.byref(self.cshape), C.c_void_p(self.ws.data_ptr()),
             self.nbytes, C.byref(k), C.c_void_p(_stream(self.device)))
        return k.value

    def energy_gap(self, lam: float):
        out = (C.c_double * 3)()
        call("tvpd_energy_gap", C.byref(self.cshape), C.c_float(lam),
             C.c_void_p(self.ws.data_ptr()), self.nbytes, out,
             C.c_void_p(_stream(self.device)))
        return float(out[0]), float(out[1]), float(out[2])

    # -- full solve ---------------------------------------------------------
    def solve(self, g: torch.Tensor, lam: float = 0.1, tau: float | None = None,
              sigma: float | None = None, theta: float = 1.0,
              max_iter: int = 1000, check_every: int = 10,
              gap_tol: float = 1e-4, use_graph: int = -1,
              out: torch.Tensor | None = None):
        _check_image(g, "g")
        if tuple(g.shape) != self.shape:
            raise ValueError(f"g has shape {tuple(g.shape)}, expected {self.shape}")
        if out is None:
            out = torch.empty_like(g)
        _check_image(out, "out")
        prm = Params(self._coeffs(lam, tau, sigma, theta), int(max_iter),
                     int(check_every), float(gap_tol), int(use_graph), 0)
        res = Result()
        call("tvpd_solve", C.byref(self.cshape), C.c_void_p(g.data_ptr()),
             C.c_void_p(out.data_ptr()), C.byref(prm),
             C.c_void_p(self.ws.data_ptr()), self.nbytes, C.byref(res),
             C.c_void_p(_stream(self.device)))
        return out, SolveResult(res.iters, bool(res.converged), res.primal,
                                res.dual, res.gap)

    def _coeffs(self, lam, tau, sigma, theta) -> Coeffs:
        s = default_step(len(self.shape))
        return Coeffs(float(lam), float(s if tau is None else tau),
                      float(s if sigma is None else sigma), float(theta))


def set_tile(shape, th: int, wpb: int = 4, order: int = 1):
    """Force the 2D sweep tile for ``shape`` in this process: rows per wave
    band, waves per block, tile order (0 band by band, 1 strip by strip; 2
    selects the pipelined passes, one block per band of ``th`` rows, and
    ignores ``wpb``)."""
    call("tvpd_set_tile", C.byref(make_shape(shape)), int(th), int(wpb),
         int(order))


def get_tile(shape):
    th, wpb, order = C.c_int32(), C.c_int32(), C.c_int32()
    call("tvpd_get_tile", C.byref(make_shape(shape)), C.byref(th),
         C.byref(wpb), C.byref(order))
    return th.value, wpb.value, order.value


def set_tile3d(shape, th: int, tz: int, wpb: int = 4):
    """Force the 3D sweep tile for ``shape`` (nz, ny, nx) in this process:
    rows per wave band (2 or 4), planes per wave segment, waves per block."""
    call("tvpd_set_tile3d", C.byref(make_shape(shape)), int(th), int(tz),
         int(wpb))


def get_tile3d(shape):
    th, tz, wpb = C.c_int32(), C.c_int32(), C.c_int32()
    call("tvpd_get_tile3d", C.byref(make_shape(shape)), C.byref(th),
         C.byref(tz), C.byref(wpb))
    return th.value, tz.value, wpb.value


def set_pass_depth(depth: int):
    """Longest pass (iterations per launch) of the plain 2D solver: 0 for
    each kernel's default (5 for the strip walk, 10 for the pipelined
    passes), else 1 .. 10, capped at 6 for the strip walk; the iterates are
    the same for every depth.  Process-wide."""
    call("tvpd_set_pass_depth", int(depth))


def get_pass_depth() -> int:
    d = C.c_int32()
    call("tvpd_get_pass_depth", C.byref(d))
    return d.value


def pass_length(shape) -> int:
    """Longest pass the plain solver takes for the 2D ``shape`` now (its
    tile's kernel and the depth setting)."""
    n = C.c_int32()
    call("tvpd_pass_length", C.byref(make_shape(shape)), C.byref(n))
    return n.value


def set_wait_limit(polls: int):
    """Polls after which a wait between the waves of a pipelined pass gives
    up (0: the default, about half a second), process-wide.  A pass whose
    wait gave up makes the solve raise (TVPD_ERR_DEVICE)."""
    call("tvpd_set_wait_limit", int(polls))


def set_blocking(on: bool):
    """Temporal blocking of the plain and batched 2D solvers on (passes of
    up to the default depth) or off (one iteration per launch), process-wide;
    the iterates are the same either way."""
    call("tvpd_set_blocking", 1 if on else 0)


def autotune(shape, device="cuda", cache_path: str | None = None,
             g: torch.Tensor | None = None):
    """Time the candidate sweep tiles for ``shape`` and keep the fastest for
    this process (optionally appending it to ``cache_path``).  Returns
    ``((th, wpb, order), microseconds_per_iteration)`` for a 2D shape and
    ``((th, tz, wpb), microseconds_per_iteration)`` for a 3D one."""
    s = PlainSolver(shape, device)
    if g is None:
        g = torch.rand(s.shape, dtype=torch.float32, device=s.device)
    s.init(g)
    th, wpb, order = C.c_int32(), C.c_int32(), C.c_int32()
    us = C.c_float()
    call("tvpd_autotune", C.byref(s.cshape), C.c_void_p(s.ws.data_ptr()),
         s.nbytes, cache_path.encode() if cache_path else None, C.byref(th),
         C.byref(wpb), C.byref(order), C.byref(us),
         C.c_void_p(_stream(s.device)))
    if len(s.shape) == 3:
        return (th.value, order.value, wpb.value), us.value
    return (th.value, wpb.value, order.value), us.value


def tune_load(cache_path: str) -> int:
    """Load autotuned tiles for this device's architecture from a cache
    file; returns how many entries were taken."""
    n = C.c_int32()
    call("tvpd_tune_load", cache_path.encode(), C.byref(n))
    return n.value


def solve(g: torch.Tensor, lam: float = 0.1, **kw):
    """One-shot solve; see :meth:`PlainSolver.solve`."""
    return PlainSolver(tuple(g.shape), g.device).solve(g, lam, **kw)
