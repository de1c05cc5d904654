"""The 64-right-hand-side sweep on the matrix cores (dual_grad with nrhs >= 64)
against single-vector sweeps of the same right-hand sides and against the CPU
oracle, on single trees of every width class and on a batched handle."""
import numpy as np
import pytest

import oracle
import treegen
from gpu_cases import TOL_GRAD, case, row_scale

pytestmark = pytest.mark.gpu

PANEL_CASES = ["tiny", "odd_ragged", "cfg1_shape", "cfg4_shape", "mid_width", "cfg3_shape", "capped",
               "single_path", "no_chain", "wide"]


@pytest.fixture(scope="module")
def st():
    import torch
    from paper_2107_01745_amd import stotree
    assert torch.cuda.is_available()
    stotree.lib()
    return stotree


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _many(st, tf, x0, y, homogeneous, nrhs):
    import torch
    x = torch.full((nrhs * tf.x_len,), np.nan, dtype=torch.float64, device="cuda:0")
    u = torch.full((nrhs * tf.u_len,), np.nan, dtype=torch.float64, device="cuda:0")
    st.dual_grad(tf, x0, y, homogeneous, x, u, nrhs=nrhs)
    torch.cuda.synchronize()
    return x.cpu().numpy().reshape(nrhs, tf.x_len), u.cpu().numpy().reshape(nrhs, tf.u_len)


@pytest.mark.parametrize("name", PANEL_CASES)
@pytest.mark.parametrize("homogeneous", [False, True])
def test_panel_matches_single_sweeps_and_oracle(st, name, homogeneous):
    import torch
    prob = case(name)
    tf = st.tree_factor(prob, precondition=True)
    nrhs = 67                      # one panel of 64, then a pair and a single
    rng = np.random.default_rng(len(name) * 7 + homogeneous)
    Y = rng.standard_normal((nrhs, tf.m))
    X0 = rng.uniform(-2, 2, (nrhs, prob.nx))
    xm, um = _many(st, tf, _t(X0), _t(Y), homogeneous, nrhs)
    scale = max(1.0, np.abs(xm).max())
    for k in range(nrhs):
        xs, us = _many(st, tf, _t(X0[k]), _t(Y[k]), homogeneous, 1)
        assert np.abs(xm[k] - xs[0]).max() <= 1e-12 * scale, (name, k)
        assert np.abs(um[k] - us[0]).max() <= 1e-12 * scale, (name, k)
    pb, fac = oracle.factor(prob)
    for k in (0, 31, 63, 66):
        xo, uo = oracle.sweep(pb, fac, row_scale(prob) * Y[k], homogeneous=homogeneous, x0=X0[k])
        s = max(1.0, np.abs(xo).max())
        assert np.abs(xm[k].reshape(xo.shape) - xo).max() / s < TOL_GRAD, (name, k)
        assert np.abs(um[k].reshape(uo.shape) - uo).max() / s < TOL_GRAD, (name, k)
    tf.free()


def test_panel_on_batched_handle(st):
    probs = [case(n) for n in ("odd_ragged", "capped", "cfg3_shape", "mid_width")]
    probs += treegen.draw_batch_instances(4, seed=5, scale=0.03, N_range=(5, 8))
    tf = st.tree_factor_batch(probs, precondition=True)
    rng = np.random.default_rng(9)
    Y = rng.standard_normal((64, tf.m))
    X0 = rng.uniform(-2, 2, (64, tf.x0_len))
    xm, um = _many(st, tf, _t(X0), _t(Y), False, 64)
    for k in (0, 17, 63):
        xs, us = _many(st, tf, _t(X0[k]), _t(Y[k]), False, 1)
        s = max(1.0, np.abs(xs).max())
        assert np.abs(xm[k] - xs[0]).max() <= 1e-12 * s and np.abs(um[k] - us[0]).max() <= 1e-12 * s, k
    tf.free()
