"""The 64-right-hand-side sweep on the matrix cores (dual_grad with nrhs >= 64)
against single-vector sweeps of the same right-hand sides and against the CPU
oracle, on single trees of every width class and on a batched handle."""
import numpy as np
import pytest

import oracle
import treegen
from gpu_cases import TOL_GRAD, case, row_scale

pytestmark = pytest.mark.gpu

PANEL_CASES = ["tiny", "odd_ragged", "large_blocks", "shared_blocks", "panel_wide", "mid_width", "warm_blocks", "capped",
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
    probs = [case(n) for n in ("odd_ragged", "capped", "warm_blocks", "mid_width")]
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


def _shared_base():
    """A small tree whose boxes bind (checked feasible for every x0 drawn)."""
    base = treegen.draw_problem(treegen.uniform_tree([3, 2, 1, 1]), 6, 3, np.random.default_rng(8))
    return treegen.with_boxes(base, 5.0, 0.3)


@pytest.mark.parametrize("count,pmin", [(64, 16), (64, 65), (3, 16)])
def test_shared_handle_sweeps_match_solo(st, count, pmin):
    """count instances sharing one factor copy (panels across instances when
    count is a multiple of 64) against each instance's own handle."""
    import dataclasses
    import torch
    base = case("shared_blocks") if count == 64 else case("odd_ragged")
    tf = st.tree_factor_shared(base, count, precondition=True)
    assert tf.ninst == count and tf.m == count * base.m
    st.sweep_schedule(tf, (8, 1, 16, 0, pmin))   # 65 > count: the copies on lane groups
    rng = np.random.default_rng(count)
    X0 = rng.uniform(-2, 2, (count, base.nx))
    Y = rng.standard_normal(tf.m)
    for homogeneous in (False, True):
        xs, us = _many(st, tf, _t(X0.ravel()), _t(Y), homogeneous, 1)
        tf1 = st.tree_factor(base, precondition=True)
        for k in (0, 1, count // 2, count - 1):
            d = tf.instances[k]
            x1, u1 = _many(st, tf1, _t(X0[k]), _t(Y[d["y_off"]:d["y_off"] + d["m"]]), homogeneous, 1)
            s = max(1.0, np.abs(x1).max())
            assert np.abs(xs[0][d["x_off"]:d["x_off"] + d["V"] * d["nx"]] - x1[0]).max() <= 1e-12 * s, k
            assert np.abs(us[0][d["u_off"]:d["u_off"] + d["Vnl"] * d["nu"]] - u1[0]).max() <= 1e-12 * s, k
        tf1.free()
    tf.free()


@pytest.mark.parametrize("method", ["nama", "minfbe"])
def test_shared_handle_solves_match_oracle(st, method):
    """64 instances that differ only in x0, solved together (every sweep a
    64-instance panel), against the oracle's solution of each."""
    import dataclasses
    import torch
    base = _shared_base()
    rng = np.random.default_rng(21)
    X0 = rng.uniform(-1.5, 1.5, (64, base.nx))
    tf = st.tree_factor_shared(base, 64, precondition=True)
    pb, fac = oracle.factor(base)
    lam = 1.0 / (1.1 * oracle.power_iteration(pb, fac, True, 300))
    y = _t(np.zeros(tf.m))
    x = torch.zeros(tf.x_len, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(tf.u_len, dtype=torch.float64, device="cuda:0")
    fn = st.nama_solve if method == "nama" else st.minfbe_solve
    rc, agg = fn(tf, _t(X0.ravel()), y, x, u, st.make_opts(lam=lam, eps=1e-8, max_iter=3000))
    torch.cuda.synchronize()
    assert rc == 0, agg
    infos = st.solve_info_batch(tf)
    xh, uh = x.cpu().numpy(), u.cpu().numpy()
    for k in (0, 5, 33, 63):
        assert infos[k]["status"] == 0 and infos[k]["res_scaled_inf"] <= 1e-8, infos[k]
        p = dataclasses.replace(base, x0=X0[k])
        pk, fk = oracle.factor(p)
        ref = oracle.solve(pk, fk, method, lam, eps=1e-10, max_iter=5000)
        assert ref["status"] == 0
        d = tf.instances[k]
        xb = xh[d["x_off"]:d["x_off"] + d["V"] * d["nx"]].reshape(d["V"], d["nx"])
        ub = uh[d["u_off"]:d["u_off"] + d["Vnl"] * d["nu"]].reshape(d["Vnl"], d["nu"])
        s = max(1.0, np.abs(ref["x"]).max())
        assert np.abs(xb - ref["x"]).max() / s < 1e-6 and np.abs(ub - ref["u"]).max() / s < 1e-6, k
    tf.free()


@pytest.mark.parametrize("count", [64, 3])
def test_shared_handle_with_own_disturbances(st, count):
    """Copies that differ in x0 and in the disturbances c (affine terms from
    the kept value-function Hessians) against each copy factored on its own."""
    import dataclasses
    base = _shared_base() if count == 64 else case("odd_ragged")
    draws = treegen.draw_warm_instances(base, count, seed=30 + count)
    C = np.stack([p.c for p in draws])
    tf = st.tree_factor_shared(base, count, precondition=True, c=C)
    rng = np.random.default_rng(count + 1)
    Y = rng.standard_normal(tf.m)
    X0 = np.stack([p.x0 for p in draws])
    for homogeneous in (False, True):
        xs, us = _many(st, tf, _t(X0.ravel()), _t(Y), homogeneous, 1)
        for k in (0, 1, count // 2, count - 1):
            d = tf.instances[k]
            tf1 = st.tree_factor(draws[k], precondition=True)
            x1, u1 = _many(st, tf1, _t(X0[k]), _t(Y[d["y_off"]:d["y_off"] + d["m"]]), homogeneous, 1)
            tf1.free()
            s = max(1.0, np.abs(x1).max())
            assert np.abs(xs[0][d["x_off"]:d["x_off"] + d["V"] * d["nx"]] - x1[0]).max() <= 1e-11 * s, k
            assert np.abs(us[0][d["u_off"]:d["u_off"] + d["Vnl"] * d["nu"]] - u1[0]).max() <= 1e-11 * s, k
    tf.free()


@pytest.mark.parametrize("method", ["nama", "minfbe"])
def test_shared_handle_with_own_disturbances_solves(st, method):
    """64 copies with their own x0 and c solved together (panels) against the
    oracle solution of each copy."""
    import torch
    base = _shared_base()
    draws = treegen.draw_warm_instances(base, 64, seed=77, x0_range=1.5)
    pb, fac = oracle.factor(base)
    lam = 1.0 / (1.1 * oracle.power_iteration(pb, fac, True, 300))
    tf = st.tree_factor_shared(base, 64, precondition=True, c=np.stack([p.c for p in draws]))
    y = _t(np.zeros(tf.m))
    x = torch.zeros(tf.x_len, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(tf.u_len, dtype=torch.float64, device="cuda:0")
    fn = st.nama_solve if method == "nama" else st.minfbe_solve
    rc, agg = fn(tf, _t(np.concatenate([p.x0 for p in draws])), y, x, u,
                 st.make_opts(lam=lam, eps=1e-8, max_iter=3000))
    infos = st.solve_info_batch(tf)
    xh = x.cpu().numpy()
    checked = 0
    for k in (0, 9, 40, 63):
        pk, fk = oracle.factor(draws[k])
        ref = oracle.solve(pk, fk, method, lam, eps=1e-10, max_iter=5000)
        if ref["status"] != 0:
            continue          # a draw without a feasible point: nothing to compare
        assert infos[k]["status"] == 0 and infos[k]["res_scaled_inf"] <= 1e-8, infos[k]
        d = tf.instances[k]
        xb = xh[d["x_off"]:d["x_off"] + d["V"] * d["nx"]].reshape(d["V"], d["nx"])
        s = max(1.0, np.abs(ref["x"]).max())
        assert np.abs(xb - ref["x"]).max() / s < 1e-6, k
        checked += 1
    assert checked >= 3
    tf.free()


def test_many_rhs_on_shared_handle_off_panels(st):
    """dual_grad with 64 right-hand sides on a shared handle whose copies are
    not swept as panels (3 copies): every copy of every right-hand side
    against its own single sweep."""
    base = case("odd_ragged")
    tf = st.tree_factor_shared(base, 3, precondition=True)
    rng = np.random.default_rng(41)
    Y = rng.standard_normal((64, tf.m))
    X0 = rng.uniform(-2, 2, (64, tf.x0_len))
    xm, um = _many(st, tf, _t(X0), _t(Y), False, 64)
    tf1 = st.tree_factor(base, precondition=True)
    for r in (0, 30, 63):
        for k in range(3):
            d = tf.instances[k]
            x1, u1 = _many(st, tf1, _t(X0[r, k * base.nx:(k + 1) * base.nx]),
                           _t(Y[r, d["y_off"]:d["y_off"] + d["m"]]), False, 1)
            s = max(1.0, np.abs(x1).max())
            assert np.abs(xm[r, d["x_off"]:d["x_off"] + d["V"] * d["nx"]] - x1[0]).max() <= 1e-12 * s, (r, k)
            assert np.abs(um[r, d["u_off"]:d["u_off"] + d["Vnl"] * d["nu"]] - u1[0]).max() <= 1e-12 * s, (r, k)
    tf1.free()
    tf.free()


def test_shared_handle_route_switch_keeps_solutions(st):
    """The same 64 copies solved with panels until every copy has finished
    (panel minimum 1), with the default switch to lane groups for the last 15
    unfinished copies, and on lane groups only (65): every copy converges,
    and iterations and solutions agree (the routes differ in rounding only)."""
    import torch
    base = _shared_base()
    rng = np.random.default_rng(23)
    X0 = rng.uniform(-1.5, 1.5, (64, base.nx))
    pb, fac = oracle.factor(base)
    lam = 1.0 / (1.1 * oracle.power_iteration(pb, fac, True, 300))
    out = {}
    for pmin in (1, 16, 65):
        tf = st.tree_factor_shared(base, 64, precondition=True)
        st.sweep_schedule(tf, (8, 1, 16, 0, pmin))
        y = _t(np.zeros(tf.m))
        x = torch.zeros(tf.x_len, dtype=torch.float64, device="cuda:0")
        u = torch.zeros(tf.u_len, dtype=torch.float64, device="cuda:0")
        rc, _ = st.nama_solve(tf, _t(X0.ravel()), y, x, u, st.make_opts(lam=lam, eps=1e-8, max_iter=3000))
        infos = st.solve_info_batch(tf)
        assert rc == 0 and all(i["status"] == 0 and i["res_scaled_inf"] <= 1e-8 for i in infos), pmin
        out[pmin] = (x.cpu().numpy(), np.array([i["iters"] for i in infos]))
        tf.free()
    its = out[1][1]
    assert its.max() > its.min()          # the copies finish at different iterations
    s = max(1.0, np.abs(out[1][0]).max())
    for pmin in (16, 65):
        assert abs(out[pmin][1].mean() - its.mean()) <= 1.0, (pmin, out[pmin][1], its)
        assert np.abs(out[pmin][0] - out[1][0]).max() / s < 1e-6, pmin


def test_two_panels_finishing_apart(st):
    """128 copies (two panels) kept on the matrix cores throughout (panel
    minimum 1): the second panel's copies start far from the first's, so one
    panel finishes while the other still iterates and its sweeps are skipped;
    every copy matches the same copies solved on lane groups only."""
    import torch
    base = _shared_base()
    rng = np.random.default_rng(31)
    X0 = np.concatenate([rng.uniform(-0.2, 0.2, (64, base.nx)), rng.uniform(-1.5, 1.5, (64, base.nx))])
    pb, fac = oracle.factor(base)
    lam = 1.0 / (1.1 * oracle.power_iteration(pb, fac, True, 300))
    out = {}
    for pmin in (1, 129):
        tf = st.tree_factor_shared(base, 128, precondition=True)
        st.sweep_schedule(tf, (8, 1, 16, 0, pmin))
        y = _t(np.zeros(tf.m))
        x = torch.zeros(tf.x_len, dtype=torch.float64, device="cuda:0")
        u = torch.zeros(tf.u_len, dtype=torch.float64, device="cuda:0")
        rc, _ = st.nama_solve(tf, _t(X0.ravel()), y, x, u, st.make_opts(lam=lam, eps=1e-8, max_iter=3000))
        infos = st.solve_info_batch(tf)
        assert rc == 0 and all(i["status"] == 0 and i["res_scaled_inf"] <= 1e-8 for i in infos), pmin
        out[pmin] = (x.cpu().numpy(), np.array([i["iters"] for i in infos]))
        tf.free()
    its = out[1][1]
    assert its[:64].max() < its[64:].max()      # the first panel finishes first
    s = max(1.0, np.abs(out[129][0]).max())
    assert np.abs(out[1][0] - out[129][0]).max() / s < 1e-6
    assert abs(its.mean() - out[129][1].mean()) <= 1.0


def test_shared_tree_full_size_kkt(st):
    """The shared tree at full size (234,837 nodes, nx=64, nu=32), 64 copies
    with their own x0 swept as one panel per right-hand side on the matrix
    cores, as the benchmark times it: the x(y) of copies 0 and 63 satisfies the
    dynamics and stationarity of the inner problem at random duals (drawn on
    the device; only the checked copies come back)."""
    import dataclasses
    import torch
    from gpu_cases import inner_kkt_residual
    prob = treegen.make_workload("shared")
    print("shared tree generated", flush=True)
    tf = st.tree_factor_shared(prob, 64, precondition=True)
    rng = np.random.default_rng(13)
    X0 = rng.uniform(-3, 3, (64, prob.nx))
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(13)
    y = torch.randn(tf.m, dtype=torch.float64, device="cuda:0", generator=gen)
    x = torch.empty(tf.x_len, dtype=torch.float64, device="cuda:0")
    u = torch.empty(tf.u_len, dtype=torch.float64, device="cuda:0")
    st.dual_grad(tf, _t(X0.ravel()), y, False, x, u)
    torch.cuda.synchronize()
    print("panel sweep done", flush=True)
    sc = row_scale(prob)
    for k in (0, 63):
        d = tf.instances[k]
        xb = x[d["x_off"]:d["x_off"] + d["V"] * d["nx"]].cpu().numpy().reshape(d["V"], d["nx"])
        ub = u[d["u_off"]:d["u_off"] + d["Vnl"] * d["nu"]].cpu().numpy().reshape(d["Vnl"], d["nu"])
        yb = sc * y[d["y_off"]:d["y_off"] + d["m"]].cpu().numpy()
        dyn, stat = inner_kkt_residual(dataclasses.replace(prob, x0=X0[k]), yb, xb, ub, X0[k])
        print(f"copy {k}: dynamics {dyn:.2e}, stationarity {stat:.2e}", flush=True)
        assert dyn < TOL_GRAD and stat < TOL_GRAD, k
    tf.free()


def test_graph_replay_of_panel_sweep(st):
    """A shared handle's dual_grad (one 64-copy panel per right-hand side on
    the matrix cores) recorded as a HIP graph: replays with new duals at the
    bound address, and eager work in between, equal eager sweeps bit for bit."""
    import torch
    base = case("shared_blocks")
    tf = st.tree_factor_shared(base, 64, precondition=True)
    rng = np.random.default_rng(19)
    x0 = _t(rng.uniform(-2, 2, 64 * base.nx))
    y = _t(rng.standard_normal(tf.m))
    x = torch.zeros(tf.x_len, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(tf.u_len, dtype=torch.float64, device="cuda:0")
    g = st.SweepGraph(tf, x0, y, False, x, u)
    for rep in range(4):
        y.copy_(_t(rng.standard_normal(tf.m)))
        x.fill_(np.nan)
        u.fill_(np.nan)
        g.launch()
        torch.cuda.synchronize()
        xe, ue = _many(st, tf, x0, y, False, 1)
        assert np.array_equal(x.cpu().numpy(), xe[0]) and np.array_equal(u.cpu().numpy(), ue[0]), rep
    g.free()
    tf.free()
