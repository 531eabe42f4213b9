"""Plausible mistakes planted in the FP64 oracle must each fail a pin (CPU).

Each case takes one oracle function's source, replaces one exact snippet
(a sign, an index, a dropped term, a swapped operand or weight), compiles
the mutant in a copy of the module's namespace and installs it, with
pytest's monkeypatch, wherever the original is looked up: the oracle
package, its submodules, and so every pin and every oracle function that
calls it.  The pins named for the case are then run in turn; at least one
must fail.  A mutant that every pin accepts is a hole in the pins.

The snippet must occur exactly once in the source, so a case cannot turn
into a silent no-op when the oracle is edited.
"""
import inspect
import textwrap

import pytest

import oracle
import oracle.logpolar as logpolar
import oracle.pdhg as pdhg
import oracle.tomo as tomo
import oracle.unrolled as unrolled
import test_oracle_logpolar as T_lp
import test_oracle_operators as T_ops
import test_oracle_solver as T_sol
import test_oracle_tomo as T_tomo
import test_oracle_unrolled as T_unr

MODULES = (oracle, pdhg, tomo, unrolled, logpolar)


def mutant(module, name, old, new):
    src = textwrap.dedent(inspect.getsource(getattr(module, name)))
    assert old != new and src.count(old) == 1, (name, old)
    ns = dict(vars(module))
    exec(compile(src.replace(old, new), f"<mutant of {name}>", "exec"), ns)
    return ns[name]


def pin(fn, *args):
    return (f"{fn.__name__}{args if args else ''}", lambda: fn(*args))


OPS_ADJ = pin(T_ops.test_adjointness, (5, 3))
OPS_GRAD = pin(T_ops.test_grad_matches_explicit_matrix, (5, 3))
TRAJ = [pin(T_sol.test_trajectory_in_the_cosine_basis, 1.0),
        pin(T_sol.test_trajectory_in_the_cosine_basis, 0.5)]
TOMO_TRAJ = [pin(T_tomo.test_trajectory_with_two_orthogonal_projections, r, t)
             for r in ("tv", "tikhonov") for t in (1.0, 0.5)]
ADJ = pin(T_tomo.test_adjoint_pair, 37, 53, 30, 41)
MOMENTS = pin(T_tomo.test_mass_and_first_moment_of_every_projection, 37, 53, 30)
LINES = pin(T_tomo.test_line_sums_at_0_and_90_degrees)
FIRST = pin(T_tomo.test_first_iteration_closed_form)
BST_BP = pin(T_tomo.test_bst_equals_the_backprojection_up_to_the_origin_constant)

# (case, module, function, snippet, replacement, pins)
CASES = [
    # --- denoising operators and proximal maps -------------------------------
    ("grad-sign", pdhg, "grad", "f[tuple(hi)] - f[tuple(lo)]",
     "f[tuple(lo)] - f[tuple(hi)]", [OPS_GRAD]),
    ("grad-axes-swapped", pdhg, "grad", "ax = nd - 1 - c", "ax = c",
     [pin(T_ops.test_component_convention)]),
    ("div-last-entry-sign", pdhg, "div", "out[sl(n - 1, n)] -=",
     "out[sl(n - 1, n)] +=", [OPS_ADJ]),
    ("div-interior-reversed", pdhg, "div", "pc[sl(1, n - 1)] - pc[sl(0, n - 2)]",
     "pc[sl(0, n - 2)] - pc[sl(1, n - 1)]", [OPS_ADJ]),
    ("step-bound-index", pdhg, "step_bound", "(n - 1)", "n",
     [pin(T_ops.test_step_bound_dense_eigs, (3, 5))]),
    ("ball-radius-squared", pdhg, "project_ball", "lam / safe", "lam * lam / safe",
     [pin(T_ops.test_projection_is_nearest_point)]),
    ("ball-strict-tie", pdhg, "project_ball", "nrm <= lam", "nrm < lam",
     [pin(T_ops.test_projection_ties_and_zero_weight)]),
    ("data-prox-weight", pdhg, "prox_data", "(v + tau * g)", "(v + g)",
     [pin(T_ops.test_data_prox_minimises)]),
    # --- denoising iteration -------------------------------------------------
    ("no-extrapolation", pdhg, "pdhg_iteration", "fbar = f + theta * (f - f_prev)",
     "fbar = f", TRAJ),
    ("extrapolation-sign", pdhg, "pdhg_iteration", "theta * (f - f_prev)",
     "theta * (f_prev - f)", TRAJ),
    ("primal-step-old-dual", pdhg, "pdhg_iteration", "div(p_new)", "div(p)", TRAJ),
    ("dual-step-unextrapolated", pdhg, "pdhg_iteration", "grad(fbar)", "grad(f)", TRAJ),
    ("primal-step-sign", pdhg, "pdhg_iteration", "f + tau * div(p_new)",
     "f - tau * div(p_new)", TRAJ),
    ("initial-previous-iterate", pdhg, "init_state", "g.copy(), g.copy()",
     "g.copy(), 0.0 * g", TRAJ),
    ("quadratic-dual-prox", pdhg, "quadratic_iteration", "(1.0 + sigma / lam)",
     "(1.0 + lam / sigma)", [pin(T_sol.test_quadratic_variant_matches_cosine_filter)]),
    # --- energies and the gap ------------------------------------------------
    ("primal-energy-half", pdhg, "primal_energy", "0.5 * np.sum", "np.sum",
     [pin(T_ops.test_gap_density_identity)]),
    ("dual-energy-sign", pdhg, "dual_energy", "- np.sum(g * d)", "+ np.sum(g * d)",
     [pin(T_ops.test_gap_density_identity)]),
    ("gap-density-sign", pdhg, "gap_density", "- np.sum(gf * p, axis=0)",
     "+ np.sum(gf * p, axis=0)", [pin(T_ops.test_gap_density_identity)]),
    # --- unrolled adjoint ----------------------------------------------------
    ("adjoint-extrapolation", unrolled, "unrolled_backward", "(1.0 + theta) * w",
     "theta * w", [pin(T_unr.test_finite_differences_3d)]),
    ("adjoint-lam-gradient-mask", unrolled, "unrolled_backward",
     "np.sum(np.where(inside, 0.0, ns))", "np.sum(ns)",
     [pin(T_unr.test_one_iteration_closed_form), pin(T_unr.test_finite_differences_3d)]),
    ("adjoint-tangent-projection", unrolled, "unrolled_backward", "(s - n * ns[None])",
     "s", [pin(T_unr.test_finite_differences_3d)]),
    ("adjoint-data-gradient", unrolled, "unrolled_backward", "gbar += tau * alpha",
     "gbar += alpha", [pin(T_unr.test_one_iteration_closed_form)]),
    ("adjoint-tau-gradient", unrolled, "unrolled_backward", "(d + g - fn)",
     "(d - g + fn)", [pin(T_unr.test_one_iteration_closed_form)]),
    # --- tomography geometry and operators -----------------------------------
    ("angles-full-turn", tomo, "angles", "(math.pi / n_angles)",
     "(2.0 * math.pi / n_angles)", [LINES]),
    ("pixel-centres-unshifted", tomo, "pixel_centres", "+ 0.5 - W / 2.0", "- W / 2.0",
     [LINES]),
    ("detector-unshifted", tomo, "detector", "+ 0.5 - n_det / 2.0", "- n_det / 2.0",
     [MOMENTS]),
    ("project-cos-sin-swapped", tomo, "project", "x * math.cos(th) + y * math.sin(th)",
     "x * math.sin(th) + y * math.cos(th)", [LINES]),
    ("project-weights-swapped", tomo, "project", "((i0, 1.0 - w), (i0 + 1, w))",
     "((i0, w), (i0 + 1, 1.0 - w))", [MOMENTS]),
    ("project-detector-origin", tomo, "project", "t0 = 0.5 - n_det / 2.0",
     "t0 = -n_det / 2.0", [ADJ]),
    ("backproject-weights-swapped", tomo, "backproject",
     "(1.0 - w) * ext[lo] + w * ext[hi]", "w * ext[lo] + (1.0 - w) * ext[hi]", [ADJ]),
    ("backproject-cos-sin-swapped", tomo, "backproject",
     "x * math.cos(th) + y * math.sin(th)", "x * math.sin(th) + y * math.cos(th)", [ADJ]),
    ("project-entry-hat-width", tomo, "project_at", "1.0 - np.abs(u - t[i])",
     "1.0 - 0.5 * np.abs(u - t[i])",
     [pin(T_tomo.test_single_entries_match_the_full_operators)]),
    ("backproject-entry-centre", tomo, "backproject_at", "x = b + 0.5 - W / 2.0",
     "x = b - W / 2.0",
     [pin(T_tomo.test_single_entries_match_the_full_operators)]),
    ("energy-data-half", tomo, "energy", "data = 0.5 *", "data = 1.0 *",
     [pin(T_tomo.test_energy_terms)]),
    # --- tomography iteration ------------------------------------------------
    ("tomo-no-extrapolation", tomo, "iteration", "fbar = f + theta * (f - fp)",
     "fbar = f", TOMO_TRAJ),
    ("tomo-residual-prox", tomo, "iteration", "/ (1.0 + sigma_r)", "", [FIRST]),
    ("tomo-stale-residual", tomo, "iteration", "backproject(r_new, H, W)",
     "backproject(r, H, W)", [FIRST]),
    ("tomo-primal-step-old-dual", tomo, "iteration", "tau * div(p_new)", "tau * div(p)",
     TOMO_TRAJ),
    ("tomo-dual-step-unextrapolated", tomo, "iteration", "grad(fbar)", "grad(f)",
     TOMO_TRAJ),
    ("tomo-tv-sign", tomo, "iteration", "+ tau * div(p_new)", "- tau * div(p_new)",
     TOMO_TRAJ),
    ("tomo-tikhonov-prox", tomo, "iteration", "(1.0 + tau * lam)", "(1.0 + lam)",
     [FIRST]),
    # --- filtered backprojection ---------------------------------------------
    ("fbp-response", tomo, "fbp_response", "nu / (1.0 + lam * nu)",
     "nu / (1.0 + lam * nu * nu)",
     [pin(T_tomo.test_regularised_fbp_approximates_the_tikhonov_solution)]),
    ("fbp-angle-step", tomo, "fbp", "(math.pi / n_angles)", "(1.0 / n_angles)",
     [pin(T_tomo.test_fbp_reconstructs_the_phantom)]),
    ("fbp-padding", tomo, "fbp_length", "2 * n_det", "n_det",
     [pin(T_tomo.test_ramp_filter_impulse_response)]),
    # --- backprojection slice theorem ----------------------------------------
    ("bst-dft-sign", tomo, "bst_spectra", "np.exp(-2j", "np.exp(2j",
     [pin(T_tomo.test_bst_spectra_are_the_dft_of_the_projections)]),
    ("bst-origin-rule", tomo, "bst_spectra", "float(M)", "0.0",
     [pin(T_tomo.test_bst_spectra_are_the_dft_of_the_projections), BST_BP]),
    ("bst-negative-angle-half", tomo, "bst_cartesian", "nu = np.where(neg, -rho, rho)",
     "nu = rho", [BST_BP]),
    ("bst-angle-weights-swapped", tomo, "bst_cartesian",
     "(1.0 - wa) * radial(k0, nu) + wa * radial(k1",
     "wa * radial(k0, nu) + (1.0 - wa) * radial(k1",
     [pin(T_tomo.test_bst_interpolation_is_exact_for_bilinear_spectra), BST_BP]),
    ("bst-radial-weights-swapped", tomo, "bst_cartesian",
     "(1.0 - wr) * p0 + wr * p1", "wr * p0 + (1.0 - wr) * p1",
     [pin(T_tomo.test_bst_interpolation_is_exact_for_radial_affine_spectra)]),
    ("bst-band-limit", tomo, "bst_cartesian", "rho <= 0.5", "rho <= 0.25",
     [pin(T_tomo.test_bst_interpolation_is_exact_for_radial_affine_spectra)]),
    ("bst-inverse-scale", tomo, "bst", "/ (Q * Q)", "/ Q",
     [pin(T_tomo.test_bst_of_a_disc_at_its_centre)]),
    ("bst-inverse-mirrored", tomo, "bst", "np.outer(f, x))", "np.outer(f, -x))",
     [BST_BP]),
    ("fbp-bst-kernel", tomo, "bst_spectra", "1.0 / (1.0 + lam * np.abs(nu))",
     "1.0 / (1.0 + lam * nu * nu)",
     [pin(T_tomo.test_fbp_through_the_bst_matches_the_exact_backprojection)]),
    ("fbp-bst-dc", tomo, "bst_spectra", "1.0 / (1.0 + lam * np.abs(nu))",
     "np.where(nu == 0.0, 0.0, 1.0 / (1.0 + lam * np.abs(nu)))",
     [pin(T_tomo.test_fbp_through_the_bst_keeps_the_mass_and_reconstructs)]),
    ("bst-kernel-squared", tomo, "bst_spectra",
     "1.0 / np.where(nu == 0.0, 1.0, np.abs(nu))", "1.0 / np.where(nu == 0.0, 1.0, nu * nu)",
     [pin(T_tomo.test_bst_spectra_of_a_disc_follow_example_ii, None)]),
    ("bst-dft-sign-example-ii", tomo, "bst_spectra", "np.exp(-2j", "np.exp(2j",
     [pin(T_tomo.test_bst_spectra_of_a_disc_follow_example_ii, 2.5)]),
    ("bst-inverse-scale-slice", tomo, "bst", "/ (Q * Q)", "/ (2 * Q * Q)",
     [pin(T_tomo.test_bst_slice_of_a_disc_follows_the_analytic_backprojection)]),
    ("detector-cell-edges", tomo, "detector", "+ 0.5 - n_det / 2.0", "- n_det / 2.0",
     [pin(T_tomo.test_sinogram_mesh_follows_the_table_of_symbols)]),
    ("angles-over-two-pi", tomo, "angles", "(math.pi / n_angles)", "(2.0 * math.pi / n_angles)",
     [pin(T_tomo.test_sinogram_mesh_follows_the_table_of_symbols)]),
    ("bst-at-axes-swapped", tomo, "bst_at", "x = np.asarray(cols", "x = np.asarray(rows",
     [pin(T_tomo.test_sampled_bst_equals_the_whole_image, None)]),
    ("bst-at-conjugate", tomo, "bst_at", "np.exp(2j * np.pi * np.outer(y, f))",
     "np.exp(-2j * np.pi * np.outer(y, f))",
     [pin(T_tomo.test_sampled_bst_equals_the_whole_image, None)]),
    # --- log-polar backprojection ------------------------------------------------
    ("lp-mesh-first-form", logpolar, "mesh", "math.log(0.5 / R)", "math.log(1.0 / R)",
     [pin(T_lp.test_mesh_matches_the_papers_example)]),
    ("lp-mesh-step", logpolar, "mesh", "ds = 2.0 / n_det", "ds = 1.0 / n_det",
     [pin(T_lp.test_mesh_steps_and_ends, 128, 128, 185)]),
    ("lp-mesh-no-corners", logpolar, "mesh", "max(0.0, math.log(r_max / R))", "0.0",
     [pin(T_lp.test_mesh_steps_and_ends, 64, 100, 64)]),
    ("lp-conv-no-padding", logpolar, "conv_length", "2 * m.n_rho - 1", "m.n_rho",
     [pin(T_lp.test_convolution_equals_the_direct_sum)]),
    ("lp-step1-sides-swapped", logpolar, "to_logpolar",
     "(j, 1.0) if j < n_angles else (j - n_angles, -1.0)",
     "(j, -1.0) if j < n_angles else (j - n_angles, 1.0)",
     [pin(T_lp.test_step1_is_exact_for_linear_projections)]),
    ("lp-step1-bin-origin", logpolar, "to_logpolar", "n_det / 2.0 - 0.5", "n_det / 2.0",
     [pin(T_lp.test_step1_is_exact_for_linear_projections)]),
    ("lp-step1-no-zero-beyond", logpolar, "to_logpolar",
     "np.concatenate(([0.0], s[k], [0.0]))", "np.concatenate(([s[k, 0]], s[k], [s[k, -1]]))",
     [pin(T_lp.test_step1_is_exact_for_linear_projections)]),
    ("lp-kernel-root", logpolar, "kernel", "root = -np.log(c[pos])", "root = 1.0 - c[pos]",
     [pin(T_lp.test_kernel_has_unit_mass_at_the_root)]),
    ("lp-kernel-height", logpolar, "kernel", "return out / m.drho", "return out",
     [pin(T_lp.test_kernel_has_unit_mass_at_the_root)]),
    ("lp-kernel-box", logpolar, "kernel",
     "np.maximum(0.0, 1.0 - np.abs(a[None, :] - root[:, None]) / m.drho)",
     "(np.abs(a[None, :] - root[:, None]) <= m.drho).astype(float)",
     [pin(T_lp.test_kernel_has_unit_mass_at_the_root)]),
    ("lp-conv-angle-weight", logpolar, "convolve", "m.drho * m.dphi * out", "m.drho * out",
     [pin(T_lp.test_convolution_equals_the_direct_sum)]),
    ("lp-conv-correlation", logpolar, "convolve", "np.fft.ifft2(G * Kf)",
     "np.fft.ifft2(G * np.conj(Kf))",
     [pin(T_lp.test_convolution_equals_the_direct_sum)]),
    ("lp-cartesian-axes", logpolar, "to_cartesian", "np.arctan2(Y, X)", "np.arctan2(X, Y)",
     [pin(T_lp.test_cartesian_step_is_exact_for_bilinear_data)]),
    ("lp-cartesian-first-node", logpolar, "to_cartesian", "(m.rho0 + m.drho)", "m.rho0",
     [pin(T_lp.test_cartesian_step_is_exact_for_bilinear_data)]),
    ("lp-cartesian-weights", logpolar, "to_cartesian",
     "(1 - wu) * bL[j0, i0] + wu * bL[j0, i0 + 1]",
     "wu * bL[j0, i0] + (1 - wu) * bL[j0, i0 + 1]",
     [pin(T_lp.test_cartesian_step_is_exact_for_bilinear_data)]),
    ("lp-whole-method-angle-mirror", logpolar, "to_logpolar",
     "ext = np.concatenate(([0.0], s[k], [0.0]))",
     "ext = np.concatenate(([0.0], s[(n_angles - k) % n_angles], [0.0]))",
     [pin(T_lp.test_rotation_by_one_angle_step_shifts_the_result),
      pin(T_lp.test_equals_the_backprojection_without_the_lines_through_the_origin)]),
]


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
@pytest.mark.parametrize("case,module,name,old,new,pins", CASES,
                         ids=[c[0] for c in CASES])
def test_planted_mistake_fails_a_pin(monkeypatch, case, module, name, old, new, pins):
    orig = getattr(module, name)
    bad = mutant(module, name, old, new)
    for m in MODULES:
        if getattr(m, name, None) is orig:
            monkeypatch.setattr(m, name, bad)
    passed = []
    for label, run in pins:
        try:
            run()
        except AssertionError:
            return
        passed.append(label)
    pytest.fail(f"{case}: every pin accepted the mutant: {passed}")


def test_every_pin_passes_on_the_oracle_as_written():
    """The same calls on the unmodified oracle pass, so a case above is
    caught by the mistake it plants, not by a pin that always fails."""
    seen = {}
    for case in CASES:
        for label, run in case[5]:
            seen.setdefault(label, run)
    for label, run in seen.items():
        run()
