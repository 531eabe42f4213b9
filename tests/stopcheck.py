"""Guard for exact stopping-iteration parity.

The stopping iteration is an integer decided by a floating-point comparison,
relative gap <= gap_tol, made once every check interval.  The device decides it
on float32 iterates, the oracle on float64 ones.  Both must give the same
iteration whenever rounding cannot flip the comparison at the two checks that
decide it: the last check that fails and the first that passes.  The guard
measures, at each of those checks, how far the oracle's relative gap of the
device's own iterate lies from the oracle's relative gap of its float64 iterate,
and requires the float64 relative gap to lie farther than twice that from
gap_tol.  When the guard holds, the stopping iterations must be equal.
"""
import numpy as np

import oracle


def deciding_checks(ref, check_every):
    k = ref["iters"]
    return [kk for kk in (k - check_every, k) if kk >= 0]


def assert_stop_guard(ref, g64, lam, tol, check_every, device_state_at):
    """ref: oracle.solve(..., return_history=True); device_state_at(k) returns
    the device's (f^k, p^k) as float32 arrays."""
    hist = {h[0]: h for h in ref["history"]}
    for k in deciding_checks(ref, check_every):
        _, P, _, gap = hist[k]
        f, p = device_state_at(k)
        Pd, _, gd = oracle.energy_gap(np.asarray(f, np.float64),
                                      np.asarray(p, np.float64), g64, lam)
        r_ref, r_dev = gap / P, gd / Pd
        err = abs(r_dev - r_ref)
        print(f"stop guard k={k}: rel gap {r_ref:.6e} (device iterate "
              f"{r_dev:.6e}), tol {tol:.3e}", flush=True)
        assert abs(r_ref - tol) > 2.0 * err, (
            f"check {k}: the oracle's relative gap {r_ref:.6e} lies within twice "
            f"the float32 discrepancy {err:.2e} of gap_tol {tol:.3e}; pick "
            f"another case")
