"""FP64 CPU oracle for the primal-dual image sweep (test infrastructure only).

This package is the checker, not the product: only the tests, the smoke entry
point and the benchmark's CPU-baseline leg import it.  It shares no code with
the HIP path and the HIP path never imports it.

Problem (the regularised inverse problem of the paper's Section 6, eq. opt,
specialised to an identity forward operator and a total-variation regulariser):

    minimise_f  E(f) = 1/2 ||f - g||^2 + lam * sum_i |(grad f)_i|_2

solved by the first-order primal-dual iteration (Chambolle & Pock, 2011,
Algorithm 1, extrapolation theta = 1).  The dual variable p has one component
per image axis, p[0] along x (the last array axis), p[1] along y, p[2] along z.

Contents
  pdhg      grad / div / projection, one iteration, the stopping rule,
            energies and the duality gap, the quadratic (Tikhonov-gradient)
            variant, the plain solve (a batch is solved image by image)
  unrolled  K unrolled iterations with per-iteration (lam, tau, sigma) and the
            reverse-mode adjoint of that unrolled map
  tomo      the tomographic data term: discrete Radon transform and its
            adjoint backprojection, the primal-dual iteration for
            1/2 ||A f - g||^2 + TV or Tikhonov regulariser, energies, ||A||^2,
            the regularised FBP and the backprojection slice theorem
  logpolar  the log-polar backprojection (Andersson's convolution formula,
            the four-step algorithm of the paper's Section 5)

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, exact finite algorithms or brute force (see the test
files); the centre plateau of a single disc is pinned only approximately, and so are
the tomographic operators' agreement with continuous line integrals and with
the point-source backprojection (their exact pins are the geometric ones).
"""
from .pdhg import (  # noqa: F401
    grad, div, project_ball, pdhg_iteration, primal_energy, dual_energy,
    gap_density, energy_gap, solve, quadratic_iteration,
    step_bound, init_state, run_fixed, prox_data,
)
from .unrolled import (  # noqa: F401
    unrolled_forward, unrolled_backward, unrolled_forward_batch,
    unrolled_backward_batch,
)
