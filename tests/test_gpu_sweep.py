"""GPU parity of the factor step and the sweeps (Algorithms 3 and 4) through
the C ABI, against the CPU oracle element by element, and at the full size of
the large-tree workload against the inner problem's optimality conditions."""
import numpy as np
import pytest

import oracle
import treegen
from gpu_cases import SWEEP_CASES, TOL_GRAD, case, inner_kkt_residual, row_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def st():
    import torch
    from paper_2107_01745_amd import stotree
    assert torch.cuda.is_available()
    stotree.lib()
    return stotree


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _run(st, tf, x0, y, homogeneous, nrhs=1):
    import torch
    x = torch.full((nrhs, tf.V, tf.nx), np.nan, dtype=torch.float64, device="cuda:0")
    u = torch.full((nrhs, tf.Vnl, tf.nu), np.nan, dtype=torch.float64, device="cuda:0")
    st.dual_grad(tf, None if x0 is None else _dev(x0), _dev(y), homogeneous, x, u, nrhs=nrhs)
    torch.cuda.synchronize()
    return x.cpu().numpy(), u.cpu().numpy()


def _relerr(a, b):
    return np.abs(a - b).max() / max(1.0, np.abs(b).max())


@pytest.mark.parametrize("precondition", [True, False])
@pytest.mark.parametrize("name", SWEEP_CASES)
def test_dual_grad_matches_oracle(st, name, precondition):
    prob = case(name)
    print(f"case {name} precondition={precondition}", flush=True)
    tf = st.tree_factor(prob, precondition=precondition)
    assert tf.m == prob.m
    pb, fac = oracle.factor(prob)
    rng = np.random.default_rng(17)
    sc = row_scale(prob, precondition)
    for homogeneous in (False, True):
        ybar = rng.standard_normal(tf.m)
        x, u = _run(st, tf, prob.x0, ybar, homogeneous)
        xo, uo = oracle.sweep(pb, fac, sc * ybar, homogeneous=homogeneous)
        assert _relerr(x[0], xo) < TOL_GRAD, (name, homogeneous, _relerr(x[0], xo))
        assert _relerr(u[0], uo) < TOL_GRAD, (name, homogeneous, _relerr(u[0], uo))
    tf.free()


# 64-lane chains (64 < nx + nu <= 128) whose row products end on every
# remainder of the backward batch depth: nx mod 6 (the [A B] rows) and
# ceil(nu / 2) mod 6 (the paired rows of the nu x nu and nu x nx products)
CHAIN_SHAPES = [(36, 30), (37, 33), (38, 37), (39, 29), (40, 32), (41, 35), (42, 27)]


@pytest.mark.parametrize("nx,nu", CHAIN_SHAPES)
def test_wide_chain_batch_remainders(st, nx, nu):
    prob = treegen.draw_problem(treegen.uniform_tree([2, 1, 1, 1, 1, 1]), nx, nu, np.random.default_rng(nx))
    print(f"chain shape nx={nx} nu={nu}", flush=True)
    tf = st.tree_factor(prob, precondition=True)
    pb, fac = oracle.factor(prob)
    rng = np.random.default_rng(nu)
    sc = row_scale(prob, True)
    for homogeneous in (False, True):
        ybar = rng.standard_normal(tf.m)
        x, u = _run(st, tf, prob.x0, ybar, homogeneous)
        xo, uo = oracle.sweep(pb, fac, sc * ybar, homogeneous=homogeneous)
        assert _relerr(x[0], xo) < TOL_GRAD, (nx, nu, homogeneous, _relerr(x[0], xo))
        assert _relerr(u[0], uo) < TOL_GRAD, (nx, nu, homogeneous, _relerr(u[0], uo))
    tf.free()


@pytest.mark.parametrize("nrhs", [2, 3, 5])
@pytest.mark.parametrize("name", ["odd_ragged", "fanout"])
def test_dual_grad_several_rhs(st, name, nrhs):
    prob = case(name)
    tf = st.tree_factor(prob, precondition=True)
    pb, fac = oracle.factor(prob)
    rng = np.random.default_rng(nrhs)
    sc = row_scale(prob)
    Y = rng.standard_normal((nrhs, tf.m))
    X0 = rng.uniform(-1, 1, (nrhs, tf.nx))
    for homogeneous in (False, True):
        x, u = _run(st, tf, X0, Y, homogeneous, nrhs=nrhs)
        for k in range(nrhs):
            xo, uo = oracle.sweep(pb, fac, sc * Y[k], homogeneous=homogeneous, x0=X0[k])
            assert _relerr(x[k], xo) < TOL_GRAD
            assert _relerr(u[k], uo) < TOL_GRAD
    tf.free()


def test_zero_dual_edge_case(st):
    """y = 0 gives the unconstrained LQR-tree solution; homogeneous gives 0."""
    prob = case("tiny")
    tf = st.tree_factor(prob, precondition=True)
    pb, fac = oracle.factor(prob)
    x, u = _run(st, tf, prob.x0, np.zeros(tf.m), False)
    xo, uo = oracle.sweep(pb, fac, np.zeros(tf.m))
    assert _relerr(x[0], xo) < TOL_GRAD and _relerr(u[0], uo) < TOL_GRAD
    x, u = _run(st, tf, None, np.zeros(tf.m), True)
    assert np.abs(x).max() == 0.0 and np.abs(u).max() == 0.0
    tf.free()


def test_deterministic_repeat(st):
    prob = case("large_blocks")
    tf = st.tree_factor(prob, precondition=True)
    y = np.random.default_rng(2).standard_normal(tf.m)
    a = _run(st, tf, prob.x0, y, False)
    b = _run(st, tf, prob.x0, y, False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    tf.free()


def test_not_positive_definite_is_reported(st):
    """An indefinite R makes the first Cholesky pivot of the factor step fail."""
    import dataclasses
    prob = case("tiny")
    bad = dataclasses.replace(prob, R=-100.0 * prob.R)
    with pytest.raises(st.StotreeError) as ei:
        st.tree_factor(bad)
    assert ei.value.code == -3


def test_large_tree_full_size_kkt(st):
    """Large tree at full size (62,805 nodes, nx=50, nu=30): the GPU x(y)
    satisfies the dynamics and the stationarity conditions of the inner
    problem at a random dual; x-hat(r) likewise for the homogeneous problem."""
    prob = treegen.make_workload("large")
    print("large tree generated", flush=True)
    tf = st.tree_factor(prob, precondition=True)
    rng = np.random.default_rng(5)
    sc = row_scale(prob)
    for homogeneous in (False, True):
        ybar = rng.standard_normal(tf.m)
        x, u = _run(st, tf, prob.x0, ybar, homogeneous)
        dyn, stat = inner_kkt_residual(prob, sc * ybar, x[0], u[0], prob.x0, homogeneous)
        print(f"homogeneous={homogeneous}: dynamics {dyn:.2e}, stationarity {stat:.2e}", flush=True)
        assert dyn < TOL_GRAD and stat < TOL_GRAD
        # the stages above s* in other launch forms (per stage with 8
        # wavefronts a node, first stages fused): equal to rounding
        for knobs in ((8, 1, 8, 0, 16), (8, 1, 8, 3, 16), (8, 1, 16, 3, 16), (8, 1, 8, 4, 16)):
            st.sweep_schedule(tf, knobs)
            for _ in range(2):
                xk, uk = _run(st, tf, prob.x0, ybar, homogeneous)
                s = np.abs(x[0]).max()
                assert np.abs(xk[0] - x[0]).max() <= 1e-12 * s, knobs
                assert np.abs(uk[0] - u[0]).max() <= 1e-12 * s, knobs
            print(f"schedule {knobs}: equal to rounding", flush=True)
        st.sweep_schedule(tf, (8, 1, 16, 0, 16))
    tf.free()
