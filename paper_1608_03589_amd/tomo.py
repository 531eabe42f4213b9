"""Python face of the tomographic data term: torch tensors in and out.

    minimise_f  1/2 ||A f - g||^2 + lam TV(f)          (reg="tv")
    minimise_f  1/2 ||A f - g||^2 + lam/2 ||f||^2      (reg="tikhonov")

with A the discrete Radon transform (hat weights, pixel units, angles
k pi / n_angles, bins i + 1/2 - n_det/2) and A^T its adjoint, the linear-
interpolation backprojection of the paper's Section 2 (eq. bp_app) without
the factor pi / n_angles; the solver is the primal-dual iteration with a
sinogram dual and a gradient dual.  ``include/tvpd.h`` gives the exact
definitions.  Every computation runs in ``libtvpd.so``.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from ._lib import REG_TIKHONOV, REG_TV, TomoGeom, TomoParams, call
from .solver import _check_image, _stream, alloc_workspace

REGS = {"tv": REG_TV, "tikhonov": REG_TIKHONOV}


def tomo_workspace_size(ny: int, nx: int, n_angles: int, n_det: int) -> int:
    n = C.c_size_t()
    call("tvpd_tomo_workspace_size", C.byref(TomoGeom(ny, nx, n_angles, n_det)),
         C.byref(n))
    return n.value


def set_projection_staging(on: bool):
    """A stages image rows in LDS for blocks of 8 angles (True, the default)
    or gathers every lane's columns from memory (False); the results are the
    same bit for bit.  Process-wide."""
    call("tvpd_set_projection_staging", 1 if on else 0)


def default_steps(opnorm_sq: float, reg: str = "tv"):
    """(tau, sigma_r, sigma_p) meeting the convergence condition with
    equality: TV tau = 1/L, sigma_r = 1/(2L), sigma_p = L/16 (so that
    tau sigma_r L^2 = tau sigma_p ||grad||^2 <= 1/2, ||grad||^2 < 8);
    Tikhonov tau = sigma_r = 0.99/L.  L = sqrt(opnorm_sq)."""
    L = math.sqrt(opnorm_sq)
    if reg == "tv":
        return 1.0 / L, 0.5 / L, L / 16.0
    if reg == "tikhonov":
        return 0.99 / L, 0.99 / L, 0.0
    raise ValueError(reg)


def fbp_noalloc(s: torch.Tensor, ny: int, nx: int, lam: float = 0.0,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """The regularised filtered backprojection of TomoSolver.fbp without a
    workspace: the library keeps its scratch in a static device array
    (n_angles * n_det <= 8093696).  Calls on one device must not overlap."""
    _check_image(s, "sino")
    if s.dim() != 2:
        raise ValueError("sino must be [n_angles][n_det]")
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.float32, device=s.device)
    _check_image(out, "out")
    if tuple(out.shape) != (ny, nx):
        raise ValueError(f"out has shape {tuple(out.shape)}, expected {(ny, nx)}")
    geom = TomoGeom(ny, nx, s.shape[0], s.shape[1])
    call("tvpd_fbp_noalloc", C.byref(geom), C.c_void_p(s.data_ptr()), float(lam),
         C.c_void_p(out.data_ptr()), C.c_void_p(_stream(s.device)))
    return out


class TomoSolver:
    """Reconstruction state for one image shape and scan geometry.

    The workspace (allocated once) holds the iterate ring, the sinogram and
    gradient duals, padded copies of the extrapolated image and its
    transpose, the angle table and reduction scratch.
    """

    def __init__(self, ny: int, nx: int, n_angles: int, n_det: int, device="cuda"):
        self.ny, self.nx = int(ny), int(nx)
        self.n_angles, self.n_det = int(n_angles), int(n_det)
        self.geom = TomoGeom(self.ny, self.nx, self.n_angles, self.n_det)
        self.device = torch.device(device)
        self.nbytes = tomo_workspace_size(self.ny, self.nx, self.n_angles, self.n_det)
        self.ws = alloc_workspace(self.nbytes, self.device)

    def _args(self):
        return (C.c_void_p(self.ws.data_ptr()), self.nbytes,
                C.c_void_p(_stream(self.device)))

    def _check(self, t, name, shape):
        _check_image(t, name)
        if tuple(t.shape) != shape:
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")

    # -- operators ----------------------------------------------------------
    def radon(self, f: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """A f."""
        self._check(f, "f", (self.ny, self.nx))
        if out is None:
            out = torch.empty((self.n_angles, self.n_det), dtype=torch.float32,
                              device=self.device)
        self._check(out, "out", (self.n_angles, self.n_det))
        call("tvpd_radon_forward", C.byref(self.geom), C.c_void_p(f.data_ptr()),
             C.c_void_p(out.data_ptr()), *self._args())
        return out

    def backproject(self, s: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """A^T s."""
        self._check(s, "sino", (self.n_angles, self.n_det))
        if out is None:
            out = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        self._check(out, "out", (self.ny, self.nx))
        call("tvpd_radon_backward", C.byref(self.geom), C.c_void_p(s.data_ptr()),
             C.c_void_p(out.data_ptr()), *self._args())
        return out

    def fbp(self, s: torch.Tensor, lam: float = 0.0,
            out: torch.Tensor | None = None) -> torch.Tensor:
        """Regularised filtered backprojection (pi/n_angles) A^T F_lam s,
        F_lam the filter |nu| / (1 + lam |nu|) (lam = 0: the ramp filter)."""
        self._check(s, "sino", (self.n_angles, self.n_det))
        if out is None:
            out = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        self._check(out, "out", (self.ny, self.nx))
        call("tvpd_fbp", C.byref(self.geom), C.c_void_p(s.data_ptr()), float(lam),
             C.c_void_p(out.data_ptr()), *self._args())
        return out

    # -- backprojection slice theorem -------------------------------------------
    def _bst_ws(self):
        if getattr(self, "_bst", None) is None:
            n = C.c_size_t()
            call("tvpd_bst_workspace_size", C.byref(self.geom), C.byref(n))
            self._bst = (alloc_workspace(n.value, self.device), n.value)
        return self._bst

    def bst_lengths(self):
        """(M, Q): the 1D transform length and the Cartesian grid side."""
        M, Q = C.c_int32(), C.c_int32()
        call("tvpd_bst_lengths", C.byref(self.geom), C.byref(M), C.byref(Q))
        return M.value, Q.value

    def bst(self, s: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Fast backprojection by the backprojection slice theorem (approximates
        (pi / n_angles) A^T s up to the origin rule's constant)."""
        self._check(s, "sino", (self.n_angles, self.n_det))
        if out is None:
            out = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        self._check(out, "out", (self.ny, self.nx))
        ws, n = self._bst_ws()
        call("tvpd_bst_backproject", C.byref(self.geom), C.c_void_p(s.data_ptr()),
             C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()), n,
             C.c_void_p(_stream(self.device)))
        return out

    def fbp_bst(self, s: torch.Tensor, lam: float,
                out: torch.Tensor | None = None) -> torch.Tensor:
        """Regularised filtered backprojection B F_lam s with B by the slice
        theorem: the spectra times 1/(1 + lam |nu|) (Section 6, eq. reg_fst)
        gridded and inverted as in bst().  lam >= 0."""
        self._check(s, "sino", (self.n_angles, self.n_det))
        if out is None:
            out = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        self._check(out, "out", (self.ny, self.nx))
        ws, n = self._bst_ws()
        call("tvpd_fbp_bst", C.byref(self.geom), C.c_void_p(s.data_ptr()), float(lam),
             C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()), n,
             C.c_void_p(_stream(self.device)))
        return out

    def bst_spectra(self, s: torch.Tensor) -> torch.Tensor:
        """The polar samples K(nu_j) G_k(nu_j), complex64 [n_angles][M]."""
        self._check(s, "sino", (self.n_angles, self.n_det))
        M, _ = self.bst_lengths()
        out = torch.empty((self.n_angles, M), dtype=torch.complex64, device=self.device)
        ws, n = self._bst_ws()
        call("tvpd_bst_spectra", C.byref(self.geom), C.c_void_p(s.data_ptr()),
             C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()), n,
             C.c_void_p(_stream(self.device)))
        return out

    # -- log-polar backprojection ----------------------------------------------
    def lp_mesh(self):
        """(N_rho, n_phi, L, rho_0, drho) of the log-polar mesh."""
        n_rho, n_phi, L = C.c_int32(), C.c_int32(), C.c_int32()
        rho0, drho = C.c_double(), C.c_double()
        call("tvpd_lp_mesh", C.byref(self.geom), C.byref(n_rho), C.byref(n_phi),
             C.byref(L), C.byref(rho0), C.byref(drho))
        return n_rho.value, n_phi.value, L.value, rho0.value, drho.value

    def _lp_ws(self):
        if getattr(self, "_lp", None) is None:
            n = C.c_size_t()
            call("tvpd_lp_workspace_size", C.byref(self.geom), C.byref(n))
            ws = alloc_workspace(n.value, self.device)
            call("tvpd_lp_plan", C.byref(self.geom), C.c_void_p(ws.data_ptr()), n.value,
                 C.c_void_p(_stream(self.device)))
            self._lp = (ws, n.value)
        return self._lp

    def logpolar(self, s: torch.Tensor, out: torch.Tensor | None = None,
                 lp_out: torch.Tensor | None = None) -> torch.Tensor:
        """B s by the log-polar algorithm (Andersson's convolution formula,
        Section 2.1; the four steps of Section 5).  lp_out, if given, receives
        [B s]_L as [2 n_angles][N_rho]."""
        self._check(s, "sino", (self.n_angles, self.n_det))
        if out is None:
            out = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        self._check(out, "out", (self.ny, self.nx))
        ws, n = self._lp_ws()
        if lp_out is not None:
            n_rho, n_phi = self.lp_mesh()[:2]
            self._check(lp_out, "lp_out", (n_phi, n_rho))
        call("tvpd_lp_backproject", C.byref(self.geom), C.c_void_p(s.data_ptr()),
             C.c_void_p(out.data_ptr()),
             C.c_void_p(lp_out.data_ptr() if lp_out is not None else None),
             C.c_void_p(ws.data_ptr()), n, C.c_void_p(_stream(self.device)))
        return out

    def opnorm_sq(self, iters: int = 50) -> float:
        """||A||^2 by power iteration on A^T A from the constant image."""
        v = C.c_double()
        call("tvpd_tomo_opnorm", C.byref(self.geom), int(iters),
             C.c_void_p(self.ws.data_ptr()), self.nbytes, C.byref(v),
             C.c_void_p(_stream(self.device)))
        return v.value

    # -- iteration ------------------------------------------------------------
    def init(self, f0: torch.Tensor | None = None):
        if f0 is not None:
            self._check(f0, "f0", (self.ny, self.nx))
        call("tvpd_tomo_init", C.byref(self.geom),
             C.c_void_p(f0.data_ptr() if f0 is not None else None), *self._args())

    @staticmethod
    def params(lam, tau, sigma_r, sigma_p=0.0, theta=1.0, reg="tv") -> TomoParams:
        return TomoParams(float(lam), float(tau), float(sigma_r), float(sigma_p),
                          float(theta), REGS[reg])

    def step(self, g: torch.Tensor, n_iter: int, lam: float, tau: float,
             sigma_r: float, sigma_p: float = 0.0, theta: float = 1.0,
             reg: str = "tv"):
        self._check(g, "g", (self.n_angles, self.n_det))
        prm = self.params(lam, tau, sigma_r, sigma_p, theta, reg)
        call("tvpd_tomo_step", C.byref(self.geom), C.c_void_p(g.data_ptr()),
             C.byref(prm), int(n_iter), *self._args())

    def state(self):
        """(f^k, r^k, p^k, k)."""
        f = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        r = torch.empty((self.n_angles, self.n_det), dtype=torch.float32,
                        device=self.device)
        p = torch.empty((2, self.ny, self.nx), dtype=torch.float32, device=self.device)
        k = C.c_int32()
        call("tvpd_tomo_read", C.byref(self.geom), C.c_void_p(self.ws.data_ptr()),
             self.nbytes, C.c_void_p(f.data_ptr()), C.c_void_p(r.data_ptr()),
             C.c_void_p(p.data_ptr()), C.byref(k), C.c_void_p(_stream(self.device)))
        return f, r, p, k.value

    def energy(self, g: torch.Tensor, lam: float, reg: str = "tv"):
        """(data term, regulariser term, total) of the current f^k."""
        self._check(g, "g", (self.n_angles, self.n_det))
        out = (C.c_double * 3)()
        call("tvpd_tomo_energy", C.byref(self.geom), C.c_void_p(g.data_ptr()),
             float(lam), REGS[reg], C.c_void_p(self.ws.data_ptr()), self.nbytes, out,
             C.c_void_p(_stream(self.device)))
        return out[0], out[1], out[2]

    def solve(self, g: torch.Tensor, n_iter: int, lam: float, tau: float,
              sigma_r: float, sigma_p: float = 0.0, theta: float = 1.0,
              reg: str = "tv") -> torch.Tensor:
        """n_iter iterations from f^0 = 0; returns f^n_iter."""
        self._check(g, "g", (self.n_angles, self.n_det))
        f = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        prm = self.params(lam, tau, sigma_r, sigma_p, theta, reg)
        call("tvpd_tomo_solve", C.byref(self.geom), C.c_void_p(g.data_ptr()),
             C.byref(prm), int(n_iter), C.c_void_p(f.data_ptr()), *self._args())
        return f
