"""GPU parity, through the C ABI, of GPAD, the line-search trace (value by
value), both lambda-backtracking tests, the infeasibility test, soft rows
and the general constraint map, against the CPU oracle."""
import numpy as np
import pytest

import oracle
import pins
import treegen
from gpu_cases import TOL_GRAD, TOL_PRIMAL, TOL_RES

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


def _solve(st, tf, prob, method, lam, y0=None, trace_iters=0, **kw):
    import torch
    y = _t(np.zeros(tf.m) if y0 is None else y0)
    x = torch.zeros(tf.V, tf.nx, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(tf.Vnl, tf.nu, dtype=torch.float64, device="cuda:0")
    tr = None
    if trace_iters:
        tr = torch.full((1, trace_iters, st.TRACE_COLS), np.nan, dtype=torch.float64, device="cuda:0")
    fn = {"minfbe": st.minfbe_solve, "nama": st.nama_solve, "gpad": st.gpad_solve}[method]
    rc, info = fn(tf, _t(prob.x0), y, x, u, st.make_opts(lam=lam, trace=tr, **kw))
    torch.cuda.synchronize()
    out = dict(rc=rc, info=info, y=y.cpu().numpy(), x=x.cpu().numpy(), u=u.cpu().numpy())
    if tr is not None:
        out["trace"] = tr.cpu().numpy()[0]
    return out


def _robust_prefix(tr_o, nu_max, tol):
    """Updates whose step decision is fixed by the mathematics: every trial
    up to the accepted one has |phi(w) - phi(y)| above the rounding level
    tol.  Near convergence the changes of the FBE fall to rounding level and
    the decision (and from there the trajectory) may differ legitimately."""
    n = 0
    for row in tr_o:
        acc = int(row[2])
        last = acc if acc >= 0 else nu_max
        d = row[oracle.TRACE_PHI:oracle.TRACE_PHI + last + 1]
        if not np.all(np.abs(d) > tol):
            break
        n += 1
    return n


def _setup(prob):
    pb, fac = oracle.factor(prob)
    L = oracle.power_iteration(pb, fac, True, 600)
    return pb, fac, L


def _cases():
    return {"tight_tiny": pins.tight_tiny, "ragged_cross": pins.ragged_cross,
            "general": pins.general_map, "tiny_soft": lambda: pins.soft_rows(pins.tight_tiny()),
            "general_soft": lambda: pins.soft_rows(pins.general_map()), "general_noleaf": pins.general_map_noleaf}


# ---------------------------------- GPAD ----------------------------------- #
@pytest.mark.parametrize("name", ["tight_tiny", "ragged_cross", "general", "tiny_soft"])
def test_gpad_iterates_match_oracle(st, name):
    """GPAD has no line search: its iterates are a fixed sequence, compared
    element by element after K updates."""
    prob = _cases()[name]()
    print(f"gpad {name}", flush=True)
    pb, fac, L = _setup(prob)
    lam = 1.0 / L
    tf = st.tree_factor(prob, precondition=True)
    for K in (0, 1, 5, 30):
        g = _solve(st, tf, prob, "gpad", lam, eps=0.0, max_iter=K, div_window=-1)
        ref = oracle.solve(pb, fac, "gpad", lam, eps=0.0, max_iter=K, div_window=0)
        assert g["info"]["iters"] == K == ref["iters"]
        scale = max(1.0, np.abs(ref["y"]).max())
        assert np.abs(g["y"] - ref["y"]).max() / scale < TOL_GRAD, (K, np.abs(g["y"] - ref["y"]).max())
        assert np.abs(g["x"] - ref["x"]).max() / max(1.0, np.abs(ref["x"]).max()) < TOL_GRAD
    tf.free()


@pytest.mark.parametrize("name", ["tight_tiny", "general_soft"])
def test_gpad_solve_reaches_tolerance(st, name):
    prob = _cases()[name]()
    pb, fac, L = _setup(prob)
    lam = 1.0 / L
    tf = st.tree_factor(prob, precondition=True)
    g = _solve(st, tf, prob, "gpad", lam, eps=1e-7, max_iter=20000)
    assert g["rc"] == 0
    ref = oracle.solve(pb, fac, "gpad", lam, eps=1e-7, max_iter=20000)
    assert ref["status"] == 0 and g["info"]["iters"] == ref["iters"]
    ev = oracle.evaluate(pb, fac, g["y"], lam, True)
    assert np.abs(ev["R"]).max() <= 1e-7 * (1 + 1e-6)
    tf.free()


# ---------------------------- line-search trace ----------------------------- #
@pytest.mark.parametrize("method", ["minfbe", "nama"])
@pytest.mark.parametrize("name,nu_max", [("tight_tiny", 10), ("ragged_cross", 10), ("tight_tiny", 0),
                                         ("ragged_cross", 1), ("tiny_soft", 10), ("general", 10)])
def test_line_search_trace_matches_oracle(st, method, name, nu_max):
    """Every trial's change of the FBE, as the GPU accumulates it row by row
    from the tau-independent quantities, against the oracle's direct
    phi(w) - phi(y) (one affine sweep per trial), and identical accepted
    steps, over the first updates; nu_max = 0 and 1 exercise the tau = 0
    fallback."""
    prob = _cases()[name]()
    print(f"trace {method} {name} nu_max={nu_max}", flush=True)
    pb, fac, L = _setup(prob)
    lam = 1.0 / (1.1 * L)
    K = 12
    ref = oracle.solve(pb, fac, method, lam, eps=0.0, max_iter=K, nu_max=nu_max, trace_iters=K, div_window=0)
    tf = st.tree_factor(prob, precondition=True)
    g = _solve(st, tf, prob, method, lam, eps=0.0, max_iter=K, nu_max=nu_max, trace_iters=K, div_window=-1)
    tr_g, tr_o = g["trace"], ref["trace"]
    phis = [abs(oracle.evaluate(pb, fac, np.zeros(pb.m), lam, True)["phi"]), abs(ref["phi"])]
    tol = 1e-9 * max(1.0, *phis)
    n = _robust_prefix(tr_o, nu_max, tol)
    assert n >= 5, n
    fallback = 0
    for k in range(n):
        assert tr_g[k, 2] == tr_o[k, 2], (k, tr_g[k, 2], tr_o[k, 2])          # accepted nu
        assert tr_g[k, 4] == tr_o[k, 4]                                      # pairs used
        assert abs(tr_g[k, 0] - tr_o[k, 0]) <= 1e-15 * tr_o[k, 0]           # lambda
        assert abs(tr_g[k, 1] - tr_o[k, 1]) <= 1e-9 * max(1.0, tr_o[k, 1])  # ||R||_inf
        dg = tr_g[k, st.TRACE_PHI:st.TRACE_PHI + nu_max + 1]
        do = tr_o[k, oracle.TRACE_PHI:oracle.TRACE_PHI + nu_max + 1]
        assert np.abs(dg - do).max() <= tol, (k, dg, do)
        fallback += tr_g[k, 2] < 0
    if nu_max == 0:
        assert fallback > 0
    tf.free()


# ------------------------------- backtracking ------------------------------- #
def _rounding_horizon(pb, fac, method, lam0, ref, seeds=(0, 1), **kw):
    """First update at which the oracle's own step decisions change when the
    starting dual point moves by 1e-14: past it, rounding differences alone
    (amplified along directions where the dual is flat) can change a
    line-search decision, so two correct implementations may legitimately
    take different paths to the same solution."""
    h = ref["iters"]
    for seed in seeds:
        y0 = np.random.default_rng(seed).standard_normal(pb.m) * 1e-14
        q = oracle.solve(pb, fac, method, lam0, y0=y0, **kw)
        m = min(ref["iters"], q["iters"], len(ref["trace"]))
        d = np.nonzero(ref["trace"][:m, 2] != q["trace"][:m, 2])[0]
        h = min(h, int(d[0]) if len(d) else m)
    return h


@pytest.mark.parametrize("name", ["tight_tiny", "general_soft", "general_noleaf"])
@pytest.mark.parametrize("method", ["minfbe", "nama"])
@pytest.mark.parametrize("rule,param", [(1, 0.1), (2, 0.4)])
def test_backtracking_matches_oracle(st, name, method, rule, param):
    prob = _cases()[name]()
    print(f"backtrack {name} {method} rule {rule}", flush=True)
    pb, fac, L = _setup(prob)
    lam0 = 64.0 / (1.1 * L)
    kw = dict(eps=1e-9, max_iter=3000, backtrack=rule, bt_param=param, trace_iters=400)
    ref = oracle.solve(pb, fac, method, lam0, **kw)
    tf = st.tree_factor(prob, precondition=True)
    g = _solve(st, tf, prob, method, lam0, **kw)
    assert ref["status"] == 0 and g["rc"] == 0
    # the lambda sequence and the step decisions agree while the decisions
    # are above rounding level and stable under rounding-size perturbations
    n = min(_robust_prefix(ref["trace"][:ref["iters"]], 10, 1e-9 * max(1.0, abs(ref["phi"]))),
            _rounding_horizon(pb, fac, method, lam0, ref, **kw))
    assert n >= 5, n
    assert np.array_equal(g["trace"][:n, 0], ref["trace"][:n, 0])
    assert np.array_equal(g["trace"][:n, 2], ref["trace"][:n, 2])
    assert np.array_equal(g["trace"][:n, 4], ref["trace"][:n, 4])
    b = g["info"]["backtracks"]
    assert b >= 1 and g["info"]["lam"] == lam0 * 0.5 ** b
    if ref["trace"][n - 1, 0] == ref["lambda_final"]:
        # every halving happened inside that prefix
        assert b == ref["backtracks"]
        assert g["info"]["lam"] == pytest.approx(ref["lambda_final"], rel=1e-15)
    else:
        # later halvings follow the GPU's own path: a halving needs
        # lambda L above the rule's threshold, so lambda stays above half of it
        thr = (1.0 - param) if rule == 1 else param
        assert b >= int(round(np.log2(lam0 / ref["trace"][n - 1, 0])))
        assert thr / (2 * L) * (1 - 1e-9) < g["info"]["lam"]
    scale = max(1.0, np.abs(ref["x"]).max(), np.abs(ref["u"]).max())
    assert np.abs(g["x"] - ref["x"]).max() / scale < TOL_PRIMAL
    tf.free()


def test_backtracking_from_lambda_zero(st):
    """lambda = 0 with backtracking starts from a 5-iteration power estimate
    and still converges to the oracle's solution."""
    prob = pins.ragged_cross()
    pb, fac, L = _setup(prob)
    tf = st.tree_factor(prob, precondition=True)
    for method in ("minfbe", "nama"):
        g = _solve(st, tf, prob, method, 0.0, eps=1e-9, max_iter=3000, backtrack=2, bt_param=0.45)
        assert g["rc"] == 0
        ev = oracle.evaluate(pb, fac, g["y"], g["info"]["lam"], True)
        assert np.abs(ev["R"]).max() <= 1e-9 * (1 + 1e-6)
        assert g["info"]["lam"] > 0.45 / (2 * L)
    tf.free()


# ---------------------------- infeasibility test ---------------------------- #
@pytest.mark.parametrize("method", ["minfbe", "nama", "gpad"])
def test_infeasible_problem_reports_diverged(st, method):
    prob = treegen.with_boxes(pins.tight_tiny(), xbox=0.05, ubox=0.05)
    pb, fac, L = _setup(prob)
    lam = 1.0 / (1.1 * L)
    ref = oracle.solve(pb, fac, method, lam, eps=1e-9, max_iter=2000, div_window=50)
    assert ref["status"] == -6
    tf = st.tree_factor(prob, precondition=True)
    import torch
    y = _t(np.zeros(tf.m))
    x = torch.zeros(tf.V, tf.nx, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(tf.Vnl, tf.nu, dtype=torch.float64, device="cuda:0")
    fn = {"minfbe": st.minfbe_solve, "nama": st.nama_solve, "gpad": st.gpad_solve}[method]
    with pytest.raises(st.StotreeError) as ei:
        fn(tf, _t(prob.x0), y, x, u, st.make_opts(lam=lam, eps=1e-9, max_iter=2000, div_window=50))
    assert ei.value.code == -6
    info = st.solve_info_batch(tf)[0]
    assert info["status"] == -6 and info["iters"] == ref["iters"]
    tf.free()


@pytest.mark.parametrize("method", ["minfbe", "nama", "gpad"])
def test_step_above_two_over_L_reports_numeric_error(st, method):
    """lambda fixed by the host at 4/L and 16/L, no backtracking: the device
    stops with ERR_NUMERIC, as the oracle does, and never reports a solve."""
    import torch
    prob = pins.tight_tiny()
    pb, fac, L = _setup(prob)
    tf = st.tree_factor(prob, precondition=True)
    fn = {"minfbe": st.minfbe_solve, "nama": st.nama_solve, "gpad": st.gpad_solve}[method]
    for scale in (4.0, 16.0):
        print(f"lambda {scale}/L {method}", flush=True)
        ref = oracle.solve(pb, fac, method, scale / L, eps=1e-9, max_iter=2000)
        assert ref["status"] == -5
        y = _t(np.zeros(tf.m))
        x = torch.zeros(tf.V, tf.nx, dtype=torch.float64, device="cuda:0")
        u = torch.zeros(tf.Vnl, tf.nu, dtype=torch.float64, device="cuda:0")
        with pytest.raises(st.StotreeError) as ei:
            fn(tf, _t(prob.x0), y, x, u, st.make_opts(lam=scale / L, eps=1e-9, max_iter=2000))
        assert ei.value.code == -5
        info = st.solve_info_batch(tf)[0]
        assert info["status"] == -5 and info["iters"] < 2000
    tf.free()


def test_weakly_separated_infeasible_batch_is_flagged(st):
    """The LP-infeasible draws whose objective falls by only 3.9e-4 to 1.1e-3
    of ||d|| ||R|| along the run-off direction, in one handle with a
    feasible instance: both methods flag each of them within a window of
    the oracle (the windows are 50 updates apart and the paths differ by
    rounding) and solve the feasible one.  The draw whose fall is within a
    factor 1.5 of the bound may be flagged or run to the limit, since a
    rounding-level difference can move one window across the bound; it is
    never reported solved."""
    import torch
    good = pins.tight_tiny()
    cases = list(pins.WEAK_INFEASIBLE) + [pins.NEAR_BOUND_INFEASIBLE]
    probs = [pins.reduced_uneven_boxed(*c) for c in cases] + [good]
    tf = st.tree_factor_batch(probs, precondition=True)
    x0 = _t(np.concatenate([p.x0 for p in probs]))
    for method in ("minfbe", "nama"):
        print(f"weak infeasible batch {method}", flush=True)
        y = _t(np.zeros(tf.m))
        x = torch.zeros(tf.x_len, dtype=torch.float64, device="cuda:0")
        u = torch.zeros(tf.u_len, dtype=torch.float64, device="cuda:0")
        fn = {"minfbe": st.minfbe_solve, "nama": st.nama_solve}[method]
        with pytest.raises(st.StotreeError) as ei:
            fn(tf, x0, y, x, u, st.make_opts(eps=1e-6, max_iter=3000, div_window=50))
        assert ei.value.code == -6
        infos = st.solve_info_batch(tf)
        assert infos[-1]["status"] == 0
        for c, p, info in zip(cases, probs[:-1], infos[:-1]):
            if c == pins.NEAR_BOUND_INFEASIBLE:
                assert info["status"] in (-6, 1), (c, info["status"])
                continue
            pb, fac = oracle.factor(p)
            ref = oracle.solve(pb, fac, method, info["lam"], eps=1e-6, max_iter=3000, div_window=50)
            assert ref["status"] == -6 and info["status"] == -6, (c, ref["status"], info["status"])
            assert abs(info["iters"] - ref["iters"]) <= 50, (c, info["iters"], ref["iters"])
    tf.free()


def test_batch_stops_only_the_infeasible_instance(st):
    good = pins.tight_tiny()
    bad = treegen.with_boxes(pins.tight_tiny(), xbox=0.05, ubox=0.05)
    tf = st.tree_factor_batch([good, bad, good], precondition=True)
    import torch
    x0 = _t(np.concatenate([good.x0, bad.x0, good.x0]))
    y = _t(np.zeros(tf.m))
    x = torch.zeros(tf.x_len, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(tf.u_len, dtype=torch.float64, device="cuda:0")
    with pytest.raises(st.StotreeError) as ei:
        st.nama_solve(tf, x0, y, x, u, st.make_opts(eps=1e-9, max_iter=2000))
    assert ei.value.code == -6
    infos = st.solve_info_batch(tf)
    assert [i["status"] for i in infos] == [0, -6, 0]
    tf.free()


# ------------------------ soft rows and constraint maps ---------------------- #
@pytest.mark.parametrize("name", ["general", "general_soft", "tiny_soft", "general_noleaf"])
def test_mapped_dual_grad_matches_oracle(st, name):
    import torch
    prob = _cases()[name]()
    pb, fac = oracle.factor(prob)
    tf = st.tree_factor(prob, precondition=True)
    assert tf.m == prob.m
    sc = pins.row_scale(prob)
    rng = np.random.default_rng(3)
    for homogeneous in (False, True):
        yb = rng.standard_normal((2, tf.m))
        x = torch.zeros(2, tf.V, tf.nx, dtype=torch.float64, device="cuda:0")
        u = torch.zeros(2, tf.Vnl, tf.nu, dtype=torch.float64, device="cuda:0")
        st.dual_grad(tf, _t(np.tile(prob.x0, 2)), _t(yb), homogeneous, x, u, nrhs=2)
        torch.cuda.synchronize()
        for k in range(2):
            xo, uo = oracle.sweep(pb, fac, oracle.apply_Ht(pb, sc * yb[k]), homogeneous=homogeneous)
            assert np.abs(x[k].cpu().numpy() - xo).max() <= TOL_GRAD * max(1.0, np.abs(xo).max())
            assert np.abs(u[k].cpu().numpy() - uo).max() <= TOL_GRAD * max(1.0, np.abs(uo).max())
    tf.free()


@pytest.mark.parametrize("method", ["minfbe", "nama", "gpad"])
@pytest.mark.parametrize("name", ["general", "general_soft", "tiny_soft", "general_noleaf"])
def test_mapped_and_soft_solves_match_oracle(st, method, name):
    prob = _cases()[name]()
    print(f"{method} {name}", flush=True)
    pb, fac, L = _setup(prob)
    lam = (1.0 if method == "gpad" else 1.0 / 1.1) / L
    ref = oracle.solve(pb, fac, method, lam, eps=1e-10, max_iter=100000)   # GPAD: 63,000 on general_noleaf
    assert ref["status"] == 0
    tf = st.tree_factor(prob, precondition=True)
    g = _solve(st, tf, prob, method, lam, eps=1e-8, max_iter=100000)
    assert g["rc"] == 0
    ev = oracle.evaluate(pb, fac, g["y"], lam, True)
    assert np.abs(ev["R"]).max() <= TOL_RES
    scale = max(1.0, np.abs(ref["x"]).max(), np.abs(ref["u"]).max())
    assert np.abs(g["x"] - ref["x"]).max() / scale < TOL_PRIMAL
    assert np.abs(g["u"] - ref["u"]).max() / scale < TOL_PRIMAL
    tf.free()


def test_batch_mixing_mapped_and_box_instances(st):
    """One handle with a mapped, a soft and a plain instance: each solves to
    its own oracle solution."""
    import torch
    probs = [pins.general_map(), pins.soft_rows(pins.tight_tiny()), pins.ragged_cross()]
    tf = st.tree_factor_batch(probs, precondition=True)
    lams = []
    for p in probs:
        pb, fac, L = _setup(p)
        lams.append(1.0 / (1.1 * L))
    lam = min(lams)
    x0 = _t(np.concatenate([p.x0 for p in probs]))
    y = _t(np.zeros(tf.m))
    x = torch.zeros(tf.x_len, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(tf.u_len, dtype=torch.float64, device="cuda:0")
    rc, info = st.nama_solve(tf, x0, y, x, u, st.make_opts(lam=lam, eps=1e-8, max_iter=5000))
    assert rc == 0
    yv = y.cpu().numpy()
    for b, p in enumerate(probs):
        d = tf.instances[b]
        pb, fac = oracle.factor(p)
        ev = oracle.evaluate(pb, fac, yv[d["y_off"]:d["y_off"] + d["m"]], lam, True)
        assert np.abs(ev["R"]).max() <= TOL_RES
    tf.free()
