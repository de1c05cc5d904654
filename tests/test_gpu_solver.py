"""GPU parity of the device-resident MINFBE / NAMA solvers and the power
iteration, through the C ABI, against the CPU oracle."""
import numpy as np
import pytest

import oracle
import pins
from gpu_cases import TOL_PRIMAL, TOL_RES, case, with_tight_boxes

pytestmark = pytest.mark.gpu


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


def solver_cases():
    return {
        "tight_tiny": pins.tight_tiny,
        "ragged_cross": pins.ragged_cross,
        "warm_tight": lambda: with_tight_boxes(case("warm_blocks"), 3.0, 0.4),
        # degenerate shapes with binding input bounds
        "scalar_tight": lambda: with_tight_boxes(case("scalar"), 2.0, 0.3),
        "scalar_chain_tight": lambda: with_tight_boxes(case("scalar_chain"), 2.0, 0.3),
        "one_stage_tight": lambda: with_tight_boxes(case("one_stage"), 2.0, 0.05),
        "single_input_tight": lambda: with_tight_boxes(case("single_input"), 5.0, 0.6),
    }


def _gpu_solve(st, tf, prob, method, lam, y0=None, **kw):
    import torch
    y = _t(np.zeros(tf.m) if y0 is None else y0)
    x = torch.zeros(tf.V, tf.nx, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(tf.Vnl, tf.nu, dtype=torch.float64, device="cuda:0")
    fn = st.minfbe_solve if method == "minfbe" else st.nama_solve
    rc, info = fn(tf, _t(prob.x0), y, x, u, st.make_opts(lam=lam, **kw))
    torch.cuda.synchronize()
    return rc, info, y.cpu().numpy(), x.cpu().numpy(), u.cpu().numpy()


@pytest.mark.parametrize("method", ["minfbe", "nama"])
@pytest.mark.parametrize("name", ["tight_tiny", "ragged_cross", "warm_tight", "scalar_tight", "scalar_chain_tight",
                                  "one_stage_tight", "single_input_tight"])
def test_solution_matches_oracle(st, method, name):
    prob = solver_cases()[name]()
    print(f"{method} {name}", flush=True)
    pb, fac = oracle.factor(prob)
    L = oracle.power_iteration(pb, fac, True, 500)
    lam = 1.0 / (1.1 * L)
    ref = oracle.solve(pb, fac, method, lam, eps=1e-10, max_iter=5000)
    assert ref["status"] == 0
    tf = st.tree_factor(prob, precondition=True)
    rc, info, y, x, u = _gpu_solve(st, tf, prob, method, lam, eps=1e-8, max_iter=5000)
    print(info, flush=True)
    assert rc == 0 and info["status"] == 0
    assert info["res_scaled_inf"] <= 1e-8
    # the oracle recomputes the residual at the GPU's dual
    ev = oracle.evaluate(pb, fac, y, lam, True)
    assert np.abs(ev["R"]).max() <= TOL_RES
    scale = max(1.0, np.abs(ref["x"]).max(), np.abs(ref["u"]).max())
    assert np.abs(x - ref["x"]).max() / scale < TOL_PRIMAL
    assert np.abs(u - ref["u"]).max() / scale < TOL_PRIMAL
    # x returned is x(y) at the returned y
    assert np.abs(x - ev["x"]).max() / scale < 1e-9
    tf.free()


@pytest.mark.parametrize("method", ["minfbe", "nama"])
def test_first_iterations_match_oracle(st, method):
    """Same step decisions in the first iterations give the same iterates."""
    prob = pins.tight_tiny()
    pb, fac = oracle.factor(prob)
    L = oracle.power_iteration(pb, fac, True, 500)
    lam = 1.0 / (1.1 * L)
    tf = st.tree_factor(prob, precondition=True)
    for iters in (1, 2, 3):
        ref = oracle.solve(pb, fac, method, lam, eps=1e-14, max_iter=iters)
        rc, info, y, x, u = _gpu_solve(st, tf, prob, method, lam, eps=1e-14, max_iter=iters)
        assert rc == 1 and info["iters"] == iters
        assert info["ls_trials"] == ref["ls_trials"]
        assert np.abs(y - ref["y"]).max() <= 1e-9 * max(1.0, np.abs(ref["y"]).max())
    tf.free()


def test_lipschitz_matches_oracle_power_iteration(st):
    prob = case("odd_ragged")
    pb, fac = oracle.factor(prob)
    tf = st.tree_factor(prob, precondition=True)
    Lg = st.dual_lipschitz(tf, 300)
    Lo = oracle.power_iteration(pb, fac, True, 300, v0=np.ones(pb.m))
    assert abs(Lg - Lo) <= 1e-9 * Lo
    tf.free()


def test_max_iter_reports_not_converged(st):
    prob = pins.tight_tiny()
    tf = st.tree_factor(prob, precondition=True)
    rc, info, *_ = _gpu_solve(st, tf, prob, "nama", 0.0, eps=1e-15, max_iter=2)
    assert rc == 1 and info["iters"] == 2 and info["status"] == 1
    tf.free()


def test_warm_start_at_solution_stops_immediately(st):
    prob = pins.tight_tiny()
    pb, fac = oracle.factor(prob)
    L = oracle.power_iteration(pb, fac, True, 500)
    lam = 1.0 / (1.1 * L)
    ref = oracle.solve(pb, fac, "nama", lam, eps=1e-11)
    tf = st.tree_factor(prob, precondition=True)
    rc, info, y, x, u = _gpu_solve(st, tf, prob, "nama", lam, y0=ref["y"], eps=1e-8)
    assert rc == 0 and info["iters"] == 0
    tf.free()


@pytest.mark.parametrize("method", ["minfbe", "nama"])
def test_tiny_workload_as_specified(st, method):
    import treegen
    prob = treegen.make_workload("tiny")
    tf = st.tree_factor(prob, precondition=True)
    rc, info, y, x, u = _gpu_solve(st, tf, prob, method, 0.0, eps=1e-6)
    assert rc == 0 and info["res_scaled_inf"] <= 1e-6
    pb, fac = oracle.factor(prob)
    ev = oracle.evaluate(pb, fac, y, info["lam"], True)
    assert np.abs(ev["R"]).max() <= TOL_RES
    tf.free()


def test_large_tree_solves_full_size(st):
    """The large tree at full size with abs(u) <= 0.1 (the benchmark's solve),
    NAMA and MINFBE from a cold start to a 1e-6 residual on the GPU; the CPU
    oracle, factored independently, recomputes the residual at the GPU's final
    dual (<= 1e-6) and x(y) there (the GPU's returned primal)."""
    import dataclasses
    import treegen
    prob = treegen.make_workload("large")
    tight = dataclasses.replace(prob, umin=np.full_like(prob.umin, -0.1), umax=np.full_like(prob.umax, 0.1))
    print("large tree generated", flush=True)
    tf = st.tree_factor(tight, precondition=True)
    lam = 1.0 / (1.1 * st.dual_lipschitz(tf, 100))
    sols = {}
    for method in ("nama", "minfbe"):
        rc, info, y, x, u = _gpu_solve(st, tf, tight, method, lam, eps=1e-6, max_iter=2000)
        print(f"{method}: rc {rc}, iterations {info['iters']}, residual {info['res_scaled_inf']:.2e}", flush=True)
        assert rc == 0 and info["res_scaled_inf"] <= 1e-6
        sols[method] = (y, x, u)
    tf.free()
    pb, fac = oracle.factor(tight)
    print("oracle factored", flush=True)
    for method, (y, x, u) in sols.items():
        ev = oracle.evaluate(pb, fac, y, lam, True)
        res = np.abs(ev["R"]).max()
        scale = max(1.0, np.abs(ev["x"]).max())
        print(f"{method}: oracle residual {res:.2e}", flush=True)
        assert res <= TOL_RES
        assert np.abs(x - ev["x"]).max() / scale < 1e-9 and np.abs(u - ev["u"]).max() / scale < 1e-9
