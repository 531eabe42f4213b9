"""MI355X-native primal-dual image sweep (total-variation regularised
denoising, and reconstruction from a Radon-transform sinogram), after the
regularised inverse problem of arXiv 1608.03589, Section 6.

The compute path is ``libtvpd.so`` (HIP, gfx950) behind the C ABI in
``include/tvpd.h``; this package only marshals arguments and supplies device
memory and streams through PyTorch.
"""
from ._lib import TVPDError, lib  # noqa: F401
from .batch import BatchedSolver  # noqa: F401
from .tomo import (  # noqa: F401
    TomoSolver, default_steps, fbp_noalloc, set_projection_staging,
    tomo_workspace_size,
)
from .unrolled import (  # noqa: F401
    UnrolledSolver, UnrolledTV, default_coeffs, set_fused_adjoint,
    unrolled_tv,
)
from .solver import (  # noqa: F401
    PlainSolver, SolveResult, alloc_workspace, autotune, default_step,
    get_pass_depth, get_tile, pass_length, get_tile3d, make_shape, set_blocking,
    set_pass_depth, set_tile, set_tile3d, set_wait_limit, solve, tune_load,
    workspace_size,
)

__all__ = [
    "BatchedSolver", "PlainSolver", "SolveResult", "TVPDError", "TomoSolver",
    "default_steps", "fbp_noalloc", "set_projection_staging", "tomo_workspace_size",
    "UnrolledSolver", "UnrolledTV", "default_coeffs", "set_fused_adjoint",
    "unrolled_tv",
    "alloc_workspace", "autotune",
    "tune_load",
    "default_step", "get_pass_depth", "pass_length", "get_tile", "get_tile3d", "lib",
    "make_shape", "set_pass_depth",
    "set_blocking", "set_tile", "set_tile3d", "set_wait_limit", "solve",
    "workspace_size",
]
