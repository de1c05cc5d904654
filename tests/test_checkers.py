"""CPU checks of the checkers the GPU tests rely on (no GPU)."""
import numpy as np
import pytest

import oracle
from gpu_cases import SWEEP_CASES, case, inner_kkt_residual, row_scale


@pytest.mark.parametrize("name", SWEEP_CASES)
def test_inner_kkt_residual_accepts_oracle_and_rejects_perturbation(name):
    prob = case(name)
    pb, fac = oracle.factor(prob)
    rng = np.random.default_rng(1)
    for homogeneous in (False, True):
        y = row_scale(prob) * rng.standard_normal(pb.m)
        x, u = oracle.sweep(pb, fac, y, homogeneous=homogeneous)
        dyn, stat = inner_kkt_residual(prob, y, x, u, prob.x0, homogeneous)
        assert dyn < 1e-11 and stat < 1e-11, (dyn, stat)
        u2 = u.copy()
        u2[-1, 0] += 1e-6 * max(1.0, np.abs(u).max())
        assert max(inner_kkt_residual(prob, y, x, u2, prob.x0, homogeneous)) > 1e-9
