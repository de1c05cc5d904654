"""Planted mistakes in the CPU oracle must trip at least one pin.

Each mutation is a plausible error (a dropped term, an overwrite instead of an
accumulation, a transposed operand, a sign, a loop order, a wrong scaling); it
is switched on inside the oracle library, on the CPU, and the pins of
``pins.py`` are re-evaluated.  This shows the pins are not vacuous.
"""
import numpy as np
import pytest

import oracle
import pins
from pins import PIN_TOL

MUTATIONS = {
    1: "Riccati update drops the K' St term",
    2: "backward sweep overwrites instead of accumulating (children)",
    3: "backward sweep uses Lambda instead of Lambda'",
    4: "forward sweep drops the dynamics offset c_j",
    5: "forward-backward step with the wrong sign (T = y + lambda R)",
    6: "FBE with +lambda/2 ||R||^2",
    7: "L-BFGS two-loop run in the wrong order",
    8: "preconditioning by pi instead of sqrt(pi)",
}


def failing_pins(prob):
    fails = []

    def chk(name, val, tol):
        if not (val < tol):
            fails.append(name)

    chk("kkt_affine", pins.pin_kkt_affine(prob), PIN_TOL["kkt_affine"])
    chk("kkt_homogeneous", pins.pin_kkt_homogeneous(prob), PIN_TOL["kkt_homogeneous"])
    chk("grad_fd", pins.pin_grad_fd(prob), PIN_TOL["grad_fd"])
    chk("precond_map", pins.pin_precond_map(prob), PIN_TOL["precond_map"])
    pb, fac = oracle.factor(prob)
    L = oracle.power_iteration(pb, fac, True, 500)
    if np.isfinite(L) and L > 0:
        chk("fbe_conj", pins.pin_fbe_conjugate(prob, 0.9 / L, True), PIN_TOL["fbe_conj"])
    sec, dense = pins.pin_lbfgs()
    chk("lbfgs_secant", sec, PIN_TOL["lbfgs_secant"])
    chk("lbfgs_dense", dense, PIN_TOL["lbfgs_dense"])
    if not fails:
        perr, gap, res, cert = pins.pin_solve(prob, "nama", True)
        chk("solve_primal", perr, PIN_TOL["solve_primal"])
        chk("solve_dual_gap", gap, PIN_TOL["solve_dual_gap"])
    return fails


@pytest.fixture(autouse=True)
def _reset():
    oracle.build(force=False)
    oracle.set_mutation(0)
    yield
    oracle.set_mutation(0)


def test_no_mutation_passes_every_pin():
    assert failing_pins(pins.ragged_cross()) == []


@pytest.mark.parametrize("k", sorted(MUTATIONS))
def test_mutation_is_caught(k):
    prob = pins.ragged_cross()
    oracle.set_mutation(k)
    try:
        with np.errstate(all="ignore"):
            fails = failing_pins(prob)
    except (ArithmeticError, np.linalg.LinAlgError):
        fails = ["raised"]
    finally:
        oracle.set_mutation(0)
    assert fails, f"mutation {k} ({MUTATIONS[k]}) passed every pin"


# Mistakes in the accelerated gradient, the soft-row prox, the backtracking
# and the non-finite test, each caught by the pin written for that part.
def _targeted():
    import test_oracle_methods as tm
    return {
        9: ("GPAD momentum theta (theta_prev - 1) instead of theta (1/theta_prev - 1)",
            lambda: tm.test_gpad_equals_textbook_fista_on_the_dense_dual("tiny")),
        10: ("Huber prox with the threshold dropped from the shrink factor",
             lambda: tm.test_soft_prox_by_scalar_minimisation("tiny_soft")),
        11: ("lambda halved without emptying the L-BFGS buffer",
             lambda: tm.test_halving_empties_the_lbfgs_buffer("nama")),
        12: ("residual norm skips NaN entries and GPAD checks only that norm",
             lambda: tm.test_step_above_two_over_L_is_never_reported_solved("tight_tiny", "gpad")),
    }


@pytest.mark.parametrize("k", [9, 10, 11, 12])
def test_targeted_mutation_is_caught(k):
    desc, pin = _targeted()[k]
    pin()                                   # passes on the correct oracle
    oracle.set_mutation(k)
    try:
        with np.errstate(all="ignore"), pytest.raises(AssertionError):
            pin()
    finally:
        oracle.set_mutation(0)
