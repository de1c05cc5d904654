"""The CPU oracle pinned to the mathematics (no GPU).

Each test compares the oracle with something other than itself: a dense KKT
solve of the inner problem (Sec. III-D), exact central differences of the dual
function, the dense Hessian's symmetry/spectrum, the conjugate form of the FBE
(Sec. III-A), the forward-backward decrease, a dense interior-point solution
and brute-force active-set enumeration of the whole problem (Sec. II), the
discrete algebraic Riccati equation (scipy) for a single path, and the dense
inverse-BFGS recursion.
"""
import dataclasses

import numpy as np
import pytest
import scipy.linalg

import oracle
import treegen
from dense import DenseQP, active_set_bruteforce, ipm
import pins
from pins import PIN_TOL


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)
    oracle.set_mutation(0)
    yield
    oracle.set_mutation(0)


PROBLEMS = {"tiny": pins.tight_tiny, "ragged": pins.ragged_cross,
            "tiny_workload": lambda: treegen.make_workload("tiny")}


def test_tree_invariants():
    trees = [treegen.uniform_tree(treegen.WORKLOAD_SHAPES[k]["branching"]) for k in ("tiny", "large", "warm")]
    trees += [pins.ragged_cross().tree, treegen.capped_tree(12, 37, 3), treegen.capped_tree(10, 1024, 2)]
    for t in trees:
        V, N = t.V, t.N
        assert t.stage_ptr[0] == 0 and t.anc[0] == -1
        for s in range(N + 1):
            a, b = t.stage_ptr[s], t.stage_ptr[s + 1]
            assert abs(t.prob[a:b].sum() - 1.0) < 1e-12
        for i in range(t.Vnl):
            kids = np.arange(t.child_ptr[i], t.child_ptr[i + 1])
            assert kids.size >= 1
            assert (t.anc[kids] == i).all()
        assert t.child_ptr[t.Vnl] == V
        # leaves all at stage N
        assert t.stage_ptr[N] == t.Vnl
    t1 = treegen.uniform_tree(treegen.WORKLOAD_SHAPES["large"]["branching"])
    assert (t1.V, t1.Vnl, t1.Vl) == (62805, 58709, 4096)
    t = treegen.capped_tree(12, 37, 3)
    sizes = np.diff(t.stage_ptr)
    assert list(sizes[:5]) == [1, 3, 9, 27, 37] and (sizes[4:] == 37).all()


@pytest.mark.parametrize("name", ["tiny", "ragged", "tiny_workload"])
def test_sweep_matches_dense_kkt(name):
    assert pins.pin_kkt_affine(PROBLEMS[name]()) < PIN_TOL["kkt_affine"]


@pytest.mark.parametrize("name", ["tiny", "ragged"])
def test_hom_sweep_matches_dense_kkt(name):
    assert pins.pin_kkt_homogeneous(PROBLEMS[name]()) < PIN_TOL["kkt_homogeneous"]


def test_sweep_is_affine_in_y():
    prob = pins.ragged_cross()
    pb, fac = oracle.factor(prob)
    rng = np.random.default_rng(9)
    y, r = rng.standard_normal(pb.m), rng.standard_normal(pb.m)
    x1, u1 = oracle.sweep(pb, fac, y)
    x2, u2 = oracle.sweep(pb, fac, y + r)
    xh, uh = oracle.sweep(pb, fac, r, homogeneous=True)
    assert np.abs(x2 - x1 - xh).max() < 1e-12 * max(1, np.abs(xh).max())
    assert np.abs(u2 - u1 - uh).max() < 1e-12 * max(1, np.abs(uh).max())


@pytest.mark.parametrize("name", ["tiny", "ragged"])
def test_gradient_central_differences(name):
    assert pins.pin_grad_fd(PROBLEMS[name]()) < PIN_TOL["grad_fd"]


@pytest.mark.parametrize("name", ["tiny", "ragged"])
def test_hessian_symmetric_psd_and_power_iteration(name):
    prob = PROBLEMS[name]()
    sym, psd, lmax = pins.pin_hessian(prob)
    assert sym < PIN_TOL["hess_sym"] and psd < PIN_TOL["hess_psd"]
    pb, fac = oracle.factor(prob)
    L = oracle.power_iteration(pb, fac, False, 2000)
    assert abs(L - lmax) / lmax < 1e-6


def test_precondition_is_diagonal_similarity():
    assert pins.pin_precond_map(pins.ragged_cross()) < PIN_TOL["precond_map"]


def test_single_path_is_dare_lqr():
    """A one-scenario tree with time-invariant data and terminal weight equal to
    the DARE solution keeps the stationary LQR gain at every stage."""
    rng = np.random.default_rng(21)
    nx, nu, N = 5, 3, 40
    tree = treegen.uniform_tree([1] * N)
    pr = treegen.draw_problem(tree, nx, nu, rng)
    A1, B1 = pr.A[1].copy(), pr.B[1].copy()
    Q1 = np.diag(rng.uniform(0.5, 2.0, nx))
    R1 = np.diag(rng.uniform(0.1, 1.0, nu))
    Pd = scipy.linalg.solve_discrete_are(A1, B1, Q1, R1)
    Kd = -np.linalg.solve(R1 + B1.T @ Pd @ B1, B1.T @ Pd @ A1)
    pr = dataclasses.replace(pr, A=np.broadcast_to(A1, pr.A.shape).copy(),
                             B=np.broadcast_to(B1, pr.B.shape).copy(),
                             Q=np.broadcast_to(Q1, pr.Q.shape).copy(),
                             R=np.broadcast_to(R1, pr.R.shape).copy(),
                             P=Pd[None].copy())
    pb, fac = oracle.factor(pr)
    assert np.abs(fac.K - Kd[None]).max() < 1e-9 * max(1, np.abs(Kd).max())
    assert np.abs(fac.Pcal - 2 * Pd[None]).max() < 1e-9 * np.abs(Pd).max()


def test_identical_children_collapse_to_single_path():
    """Siblings with identical data and zero duals follow the single path."""
    rng = np.random.default_rng(33)
    nx, nu, N = 3, 2, 4
    path = treegen.draw_problem(treegen.uniform_tree([1] * N), nx, nu, rng)
    tree = treegen.uniform_tree([3, 2, 1, 1])
    stage_of = np.repeat(np.arange(N + 1), np.diff(tree.stage_ptr))
    pr = treegen.draw_problem(tree, nx, nu, rng)
    pr = dataclasses.replace(pr, A=path.A[stage_of], B=path.B[stage_of], c=path.c[stage_of],
                             x0=path.x0)
    pb, fac = oracle.factor(pr)
    x, u = oracle.sweep(pb, fac, np.zeros(pb.m))
    pbp, facp = oracle.factor(path)
    xp, up = oracle.sweep(pbp, facp, np.zeros(pbp.m))
    for i in range(tree.V):
        assert np.abs(x[i] - xp[stage_of[i]]).max() < 1e-12 * max(1, np.abs(xp).max())
    for i in range(tree.Vnl):
        assert np.abs(u[i] - up[stage_of[i]]).max() < 1e-12 * max(1, np.abs(up).max())


@pytest.mark.parametrize("precondition", [False, True])
def test_fbe_conjugate_form_and_fb_decrease(precondition):
    prob = pins.ragged_cross()
    pb, fac = oracle.factor(prob)
    L = oracle.power_iteration(pb, fac, precondition, 2000)
    lam = 0.9 / L
    assert pins.pin_fbe_conjugate(prob, lam, precondition) < PIN_TOL["fbe_conj"]
    assert pins.pin_fb_decrease(prob, lam, L, precondition) < PIN_TOL["fb_decrease"]


@pytest.mark.parametrize("method", ["minfbe", "nama"])
@pytest.mark.parametrize("precondition", [False, True])
@pytest.mark.parametrize("name", ["tiny", "ragged"])
def test_solve_matches_interior_point(method, precondition, name):
    perr, gap, res, cert = pins.pin_solve(PROBLEMS[name](), method, precondition)
    assert max(cert.values()) < 1e-9, cert
    assert res["status"] == 0
    assert perr < PIN_TOL["solve_primal"], perr
    assert gap < PIN_TOL["solve_dual_gap"], gap


def test_solution_satisfies_termination_meaning():
    """||z - Hx||_inf <= eps and dist(y, normal cone at z) <= lambda eps."""
    prob = pins.tight_tiny()
    pb, fac = oracle.factor(prob)
    L = oracle.power_iteration(pb, fac, True, 400)
    lam, eps = 1 / (1.1 * L), 1e-7
    res = oracle.solve(pb, fac, "nama", lam, eps=eps, precondition=True)
    ev = oracle.evaluate(pb, fac, res["y"], lam, True)
    z, Hbx, yb = ev["z"], ev["Hbx"], res["y"]
    assert np.abs(z - Hbx).max() <= eps
    s = pins.row_scale(prob)
    lo, hi = pins.box_rows(prob)
    lo, hi = s * lo, s * hi
    dist = np.where(z >= hi, np.maximum(0, -yb), np.where(z <= lo, np.maximum(0, yb), np.abs(yb)))
    assert dist.max() <= lam * eps * (1 + 1e-9)


def test_bruteforce_active_sets_tiny():
    """nx = nu = 1, N = 2: exhaustive active-set enumeration of the QP."""
    rng = np.random.default_rng(6)
    tree = treegen.uniform_tree([2, 1])
    pr = treegen.draw_problem(tree, 1, 1, rng, xbox=0.6, ubox=0.4)
    pr = dataclasses.replace(pr, x0=np.array([1.0]))
    assert pins.feasible(pr)
    dq = DenseQP(pr)
    best = active_set_bruteforce(dq.G, dq.g, dq.E, dq.e, dq.lb, dq.ub)
    assert best is not None
    Xb, _ = best
    # the brute force must bind something, or the test proves little
    assert np.any(np.isclose(Xb, dq.lb) | np.isclose(Xb, dq.ub))
    pb, fac = oracle.factor(pr)
    L = oracle.power_iteration(pb, fac, True, 500)
    for method in ("minfbe", "nama"):
        res = oracle.solve(pb, fac, method, 1 / (1.1 * L), eps=1e-10, precondition=True)
        xd, ud = dq.split(Xb)
        assert np.abs(res["x"] - xd).max() < 1e-7
        assert np.abs(res["u"] - ud).max() < 1e-7


def test_ipm_certificate_vs_bruteforce():
    """The interior-point reference itself agrees with brute force."""
    rng = np.random.default_rng(12)
    pr = treegen.draw_problem(treegen.uniform_tree([2, 1]), 1, 1, rng, xbox=0.6, ubox=0.4)
    pr = dataclasses.replace(pr, x0=np.array([1.0]))
    assert pins.feasible(pr)
    dq = DenseQP(pr)
    Xb, _ = active_set_bruteforce(dq.G, dq.g, dq.E, dq.e, dq.lb, dq.ub)
    X, *_ , cert = ipm(dq.G, dq.g, dq.E, dq.e, dq.lb, dq.ub)
    assert np.abs(X - Xb).max() < 1e-8


def test_lbfgs_secant_and_dense_recursion():
    sec, dense = pins.pin_lbfgs()
    assert sec < PIN_TOL["lbfgs_secant"] and dense < PIN_TOL["lbfgs_dense"]
    # empty buffer: d = -g
    g = np.arange(5.0)
    assert np.array_equal(oracle.lbfgs_direction([], [], g), -g)


def test_minfbe_and_nama_agree_with_each_other_on_tiny_workload():
    prob = pins.tight_tiny(seed=3)
    pb, fac = oracle.factor(prob)
    L = oracle.power_iteration(pb, fac, True, 400)
    a = oracle.solve(pb, fac, "minfbe", 1 / (1.1 * L), eps=1e-9)
    b = oracle.solve(pb, fac, "nama", 1 / (1.1 * L), eps=1e-9)
    assert a["status"] == 0 and b["status"] == 0
    assert np.abs(a["x"] - b["x"]).max() < 1e-6
    # NAMA needs no Hessian-vector products
    assert b["sweeps_hom"] == 0 and a["sweeps_hom"] > 0


def test_threaded_oracle_is_bitwise_the_sequential_one():
    """The node-parallel loops keep every node's summation order."""
    prob = pins.ragged_cross()
    rng = np.random.default_rng(2)
    y = rng.standard_normal(prob.m)
    out = []
    for n in (1, 4):
        oracle.set_threads(n)
        try:
            pb, fac = oracle.factor(prob)
            x, u = oracle.sweep(pb, fac, y)
            xh, uh = oracle.sweep(pb, fac, y, homogeneous=True)
            out.append((fac.K.copy(), fac.Pcal.copy(), x, u, xh, uh))
        finally:
            oracle.set_threads(1)
    for a, b in zip(*out):
        assert np.array_equal(a, b)
