"""GPU parity of batched handles (forests of uneven trees) through the C ABI:
every instance of a batched sweep against the CPU oracle, batched solves
against the oracle and against solo solves of each instance."""
import numpy as np
import pytest

import oracle
import pins
import treegen
from gpu_cases import TOL_GRAD, TOL_PRIMAL, TOL_RES, case, row_scale, with_tight_boxes

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


def forest_cases():
    probs = [case(n) for n in ("odd_ragged", "capped", "single_path", "no_chain", "tiny", "warm_blocks")]
    probs += treegen.draw_batch_instances(6, seed=77, scale=0.05, N_range=(6, 12))
    return probs


def _split(tf, b, y=None, x=None, u=None, x0=None):
    d = tf.instances[b]
    out = []
    if y is not None:
        out.append(y[d["y_off"]:d["y_off"] + d["m"]])
    if x is not None:
        out.append(x[d["x_off"]:d["x_off"] + d["V"] * d["nx"]].reshape(d["V"], d["nx"]))
    if u is not None:
        out.append(u[d["u_off"]:d["u_off"] + d["Vnl"] * d["nu"]].reshape(d["Vnl"], d["nu"]))
    if x0 is not None:
        out.append(x0[d["x0_off"]:d["x0_off"] + d["nx"]])
    return out


@pytest.mark.parametrize("precondition", [True, False])
def test_batched_dual_grad_matches_oracle(st, precondition):
    import torch
    probs = forest_cases()
    tf = st.tree_factor_batch(probs, precondition=precondition)
    assert tf.ninst == len(probs)
    rng = np.random.default_rng(3)
    y = rng.standard_normal(tf.m)
    x0 = np.concatenate([p.x0 for p in probs])
    for homogeneous in (False, True):
        x = torch.full((tf.x_len,), np.nan, dtype=torch.float64, device="cuda:0")
        u = torch.full((tf.u_len,), np.nan, dtype=torch.float64, device="cuda:0")
        st.dual_grad(tf, _t(x0), _t(y), homogeneous, x, u)
        torch.cuda.synchronize()
        xh, uh = x.cpu().numpy(), u.cpu().numpy()
        for b, p in enumerate(probs):
            yb, xb, ub = _split(tf, b, y=y, x=xh, u=uh)
            pb, fac = oracle.factor(p)
            xo, uo = oracle.sweep(pb, fac, row_scale(p, precondition) * yb, homogeneous=homogeneous)
            scale = max(1.0, np.abs(xo).max())
            assert np.abs(xb - xo).max() / scale < TOL_GRAD, (b, homogeneous)
            assert np.abs(ub - uo).max() / scale < TOL_GRAD, (b, homogeneous)
    tf.free()


def test_batched_lipschitz_per_instance(st):
    probs = forest_cases()[:5]
    tf = st.tree_factor_batch(probs, precondition=True)
    L = st.dual_lipschitz(tf, 300)
    for b, p in enumerate(probs):
        pb, fac = oracle.factor(p)
        Lo = oracle.power_iteration(pb, fac, True, 300, v0=np.ones(pb.m))
        assert abs(L[b] - Lo) <= 1e-9 * Lo
    tf.free()


def solver_forest():
    return [pins.tight_tiny(), pins.ragged_cross(), with_tight_boxes(case("warm_blocks"), 3.0, 0.4),
            pins.tight_tiny(seed=40)]


@pytest.mark.parametrize("method", ["nama", "minfbe"])
def test_batched_solve_matches_oracle_and_solo(st, method):
    import torch
    probs = solver_forest()
    tf = st.tree_factor_batch(probs, precondition=True)
    y = _t(np.zeros(tf.m))
    x = torch.zeros(tf.x_len, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(tf.u_len, dtype=torch.float64, device="cuda:0")
    x0 = np.concatenate([p.x0 for p in probs])
    fn = st.nama_solve if method == "nama" else st.minfbe_solve
    rc, agg = fn(tf, _t(x0), y, x, u, st.make_opts(lam=0.0, eps=1e-8, max_iter=3000))
    torch.cuda.synchronize()
    assert rc == 0, agg
    infos = st.solve_info_batch(tf)
    yh, xh, uh = y.cpu().numpy(), x.cpu().numpy(), u.cpu().numpy()
    for b, p in enumerate(probs):
        yb, xb, ub = _split(tf, b, y=yh, x=xh, u=uh)
        info = infos[b]
        assert info["status"] == 0 and info["res_scaled_inf"] <= 1e-8, info
        pb, fac = oracle.factor(p)
        lam = info["lam"]
        ev = oracle.evaluate(pb, fac, yb, lam, True)
        assert np.abs(ev["R"]).max() <= TOL_RES
        ref = oracle.solve(pb, fac, method, lam, eps=1e-10, max_iter=5000)
        scale = max(1.0, np.abs(ref["x"]).max())
        assert np.abs(xb - ref["x"]).max() / scale < TOL_PRIMAL
        assert np.abs(ub - ref["u"]).max() / scale < TOL_PRIMAL
        # the same instance solved alone takes the same path
        tf1 = st.tree_factor(p, precondition=True)
        y1 = _t(np.zeros(tf1.m))
        x1 = torch.zeros(tf1.V, tf1.nx, dtype=torch.float64, device="cuda:0")
        u1 = torch.zeros(tf1.Vnl, tf1.nu, dtype=torch.float64, device="cuda:0")
        rc1, info1 = fn(tf1, _t(p.x0), y1, x1, u1, st.make_opts(lam=lam, eps=1e-8, max_iter=3000))
        torch.cuda.synchronize()
        assert rc1 == 0
        assert abs(info1["iters"] - info["iters"]) <= 2, (info1["iters"], info["iters"])
        assert np.abs(x1.cpu().numpy() - xb).max() / scale < TOL_PRIMAL
        tf1.free()
    tf.free()


def test_batch_instances_stop_independently(st):
    """An instance that starts at its solution stops at iteration 0 while the
    others keep iterating."""
    import torch
    probs = solver_forest()[:2]
    p0 = probs[0]
    pb, fac = oracle.factor(p0)
    L = oracle.power_iteration(pb, fac, True, 500)
    lam = 1.0 / (1.1 * L)
    ref = oracle.solve(pb, fac, "nama", lam, eps=1e-12)
    tf = st.tree_factor_batch(probs, precondition=True)
    y0 = np.zeros(tf.m)
    d0 = tf.instances[0]
    y0[d0["y_off"]:d0["y_off"] + d0["m"]] = ref["y"]
    y = _t(y0)
    x = torch.zeros(tf.x_len, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(tf.u_len, dtype=torch.float64, device="cuda:0")
    x0 = np.concatenate([p.x0 for p in probs])
    rc, agg = st.nama_solve(tf, _t(x0), y, x, u, st.make_opts(lam=lam, eps=1e-8))
    infos = st.solve_info_batch(tf)
    assert rc == 0 and infos[0]["iters"] == 0 and infos[1]["iters"] > 0
    tf.free()


@pytest.mark.parametrize("method", ["nama", "minfbe"])
def test_polling_interval_changes_no_iterate(st, method):
    """Polling the stop counter every 5 iterations instead of every one
    changes no bit of the result: finished instances are skipped on the
    device, so the extra iterations the host enqueues do nothing."""
    import torch
    probs = solver_forest()
    lams = []
    for p in probs:
        pb, fac = oracle.factor(p)
        lams.append(1.0 / (1.1 * oracle.power_iteration(pb, fac, True, 300)))
    lam = min(lams)
    tf = st.tree_factor_batch(probs, precondition=True)
    x0 = _t(np.concatenate([p.x0 for p in probs]))
    out = []
    for every in (1, 5):
        y = _t(np.zeros(tf.m))
        x = torch.zeros(tf.x_len, dtype=torch.float64, device="cuda:0")
        u = torch.zeros(tf.u_len, dtype=torch.float64, device="cuda:0")
        fn = st.nama_solve if method == "nama" else st.minfbe_solve
        rc, _ = fn(tf, x0, y, x, u, st.make_opts(lam=lam, eps=1e-8, check_every=every))
        assert rc == 0
        out.append((y.cpu().numpy(), x.cpu().numpy(), [i["iters"] for i in st.solve_info_batch(tf)]))
    assert out[0][2] == out[1][2] and len(set(out[0][2])) > 1      # instances stop at different iterations
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    tf.free()


@pytest.mark.parametrize("trunk", [3, 4])
def test_fused_trunk_solves_skip_finished_instances(st, trunk):
    """Batched NAMA with each instance's first stages in one launch per
    direction (trunk modes 3, 4): instances stop at different iterations and
    are then skipped inside the fused launches, whose workgroups wait on one
    another; polling every 1 or 5 iterations changes no bit, and every
    instance's dual meets the tolerance in the oracle's residual."""
    import torch
    probs = solver_forest()
    lams = []
    for p in probs:
        pb, fac = oracle.factor(p)
        lams.append(1.0 / (1.1 * oracle.power_iteration(pb, fac, True, 300)))
    lam = min(lams)
    tf = st.tree_factor_batch(probs, precondition=True)
    st.sweep_schedule(tf, (8, 1, 8, trunk, 16))
    x0 = _t(np.concatenate([p.x0 for p in probs]))
    out = []
    for every in (1, 5):
        y = _t(np.zeros(tf.m))
        x = torch.zeros(tf.x_len, dtype=torch.float64, device="cuda:0")
        u = torch.zeros(tf.u_len, dtype=torch.float64, device="cuda:0")
        rc, _ = st.nama_solve(tf, x0, y, x, u, st.make_opts(lam=lam, eps=1e-8, check_every=every))
        assert rc == 0
        out.append((y.cpu().numpy(), x.cpu().numpy(), [i["iters"] for i in st.solve_info_batch(tf)]))
    assert out[0][2] == out[1][2] and len(set(out[0][2])) > 1
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    for b, p in enumerate(probs):
        (yb,) = _split(tf, b, y=out[0][0])
        pb, fac = oracle.factor(p)
        ev = oracle.evaluate(pb, fac, yb, lam, True)
        assert np.abs(ev["R"]).max() <= 2e-8, b
    tf.free()


def test_uneven_batch_full_size_kkt(st):
    """The uneven batch at full size (256 trees, about 2.2M nodes), in the
    benchmark's launch configuration (autotuned schedule, one graph replay):
    the x(y) of sampled instances (the smallest, the largest and two more)
    satisfies the dynamics and stationarity of each instance's inner problem
    at a random dual."""
    import torch
    from gpu_cases import inner_kkt_residual
    probs = treegen.draw_batch_instances(256)
    print("uneven batch generated", flush=True)
    tf = st.tree_factor_batch(probs, precondition=True)
    rec = st.sweep_autotune(tf, nrhs=1, reps=3)
    print(f"schedule {rec['knobs']}", flush=True)
    rng = np.random.default_rng(17)
    ybar = rng.standard_normal(tf.m)
    x0 = _t(np.concatenate([p.x0 for p in probs]))
    y = _t(ybar)
    x = torch.full((tf.x_len,), np.nan, dtype=torch.float64, device="cuda:0")
    u = torch.full((tf.u_len,), np.nan, dtype=torch.float64, device="cuda:0")
    graph = st.SweepGraph(tf, x0, y, False, x, u)
    graph.launch()
    torch.cuda.synchronize()
    xh, uh = x.cpu().numpy(), u.cpu().numpy()
    sizes = [p.tree.V for p in probs]
    for b in sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 200}):
        p, d = probs[b], tf.instances[b]
        xb = xh[d["x_off"]:d["x_off"] + d["V"] * d["nx"]].reshape(d["V"], d["nx"])
        ub = uh[d["u_off"]:d["u_off"] + d["Vnl"] * d["nu"]].reshape(d["Vnl"], d["nu"])
        yb = row_scale(p) * ybar[d["y_off"]:d["y_off"] + d["m"]]
        dyn, stat = inner_kkt_residual(p, yb, xb, ub, p.x0)
        print(f"instance {b} (V={d['V']}, nx={d['nx']}): dynamics {dyn:.2e}, stationarity {stat:.2e}", flush=True)
        assert dyn < TOL_GRAD and stat < TOL_GRAD, b
    graph.free()
    tf.free()
