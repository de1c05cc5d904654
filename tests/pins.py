"""Pins of the CPU oracle against the mathematics (shared by the pin tests and
the planted-mistake tests).  Each pin returns an error measure; the tolerance
lives beside it in ``PIN_TOL``.

The references here come from the problem statement (dense QP, dense KKT,
interior point, closed forms, library routines), never from the oracle's own
recursion.
"""
from __future__ import annotations

import numpy as np

import oracle
import treegen
from dense import DenseQP, ipm

PIN_TOL = {
    "kkt_affine": 1e-10,
    "kkt_homogeneous": 1e-10,
    "grad_fd": 1e-9,
    "hess_sym": 1e-11,
    "hess_psd": 1e-11,
    "fbe_conj": 1e-10,
    "fb_decrease": 1e-12,
    "precond_map": 1e-12,
    "solve_primal": 1e-6,
    "solve_dual_gap": 1e-7,
    "lbfgs_secant": 1e-10,
    "lbfgs_dense": 1e-10,
}


def feasible(prob) -> bool:
    """LP feasibility of the whole problem (Sec. II assumes it; the generator
    does not guarantee it, so test instances are certified).  Covers a
    general constraint map and soft rows (through the slack form)."""
    from scipy.optimize import linprog
    from dense import soft_qp
    G, g, k, E, e, lb, ub, n, dq = soft_qp(prob)
    bounds = list(zip(np.where(np.isfinite(lb), lb, None), np.where(np.isfinite(ub), ub, None)))
    return linprog(np.zeros(G.shape[0]), A_eq=E, b_eq=e, bounds=bounds).status == 0


def tight_tiny(seed=7):
    """Tiny-workload shape with boxes tight enough that constraints bind; the first
    LP-feasible draw at or after ``seed``."""
    for s in range(seed, seed + 200):
        pr = treegen.draw_problem(treegen.uniform_tree([2, 2, 2, 1, 1]), 4, 2,
                                  np.random.default_rng(s), xbox=2.0, ubox=0.3,
                                  x0_range=1.5)
        if feasible(pr):
            return pr
    raise RuntimeError("no feasible draw")


def ragged_cross(seed=11):
    """Uneven tree with the optional S, q, r, p terms."""
    rng = np.random.default_rng(seed)
    counts, n = [], 1
    for _ in range(4):
        ct = rng.integers(1, 4, size=n)
        counts.append(ct.tolist())
        n = int(ct.sum())
    tree = treegen.tree_from_counts(counts)
    pr = treegen.draw_problem(tree, 3, 2, rng, xbox=2.0, ubox=0.5, cross_terms=True)
    assert feasible(pr)
    return pr


def row_scale(prob):
    """sqrt(pi) of the owning node for every dual row (the preconditioning of
    Sec. III-E), built from the layout of the problem statement."""
    t = prob.tree
    sc = []
    for i in range(t.V):
        w = prob.nc if i < t.Vnl else prob.ncN
        sc += [np.sqrt(t.prob[i])] * w
    return np.array(sc)


def general_map(seed=13, nc=3, ncN=2):
    """Tiny-shape problem bounded through a general constraint map
    z_i = F x_i + G u_i (|z| <= 0.8) and z_j = FN x_j (|z| <= 1.5): the first
    LP-feasible draw at or after ``seed``."""
    for s in range(seed, seed + 200):
        rng = np.random.default_rng(s)
        pr = treegen.draw_problem(treegen.uniform_tree([2, 2, 2, 1, 1]), 4, 2, rng, x0_range=1.5)
        F = rng.standard_normal((nc, pr.nx)) * 0.5
        G = rng.standard_normal((nc, pr.nu))
        FN = rng.standard_normal((ncN, pr.nx)) * 0.5
        pr = treegen.with_constraint_map(pr, F, G, FN, -0.8, 0.8, -1.5, 1.5)
        if feasible(pr):
            return pr
    raise RuntimeError("no feasible draw")


def general_map_noleaf(seed=13):
    """A constraint map with no leaf rows (ncN = 0): z_i = F x_i + G u_i,
    |z| <= 0.3, with a weak state coupling (F ~ 0.15 N(0, 1)).  A strong
    coupling with no leaf rows can force an unstable closed loop: feasible,
    but with primal costs near 1e6 and dual optima near 1e7."""
    rng = np.random.default_rng(seed)
    pr = treegen.draw_problem(treegen.uniform_tree([2, 2, 2, 1, 1]), 4, 2, rng, x0_range=1.5)
    F = rng.standard_normal((2, pr.nx)) * 0.15
    G = rng.standard_normal((2, pr.nu))
    pr = treegen.with_constraint_map(pr, F, G, np.zeros((0, pr.nx)), -0.3, 0.3, -1.5, 1.5)
    assert feasible(pr)
    return pr


# Reduced uneven-batch draws (scale 0.02, nx 4..10, N 5..10) with |u| <= 0.1
# that an LP proves infeasible and whose separating direction is weak in the
# norms of the infeasibility test: along the null direction the iterates run
# off on, the dual objective falls by only 3.9e-4 to 1.1e-3 of ||d|| ||R||.
WEAK_INFEASIBLE = ((0, 0), (5, 5), (25, 1), (27, 5))
# such a draw whose fall under NAMA (1.5e-4) is within a factor 1.5 of the
# bound, and one whose fall (8.4e-5) is below it
NEAR_BOUND_INFEASIBLE = (11, 0)
WEAKER_INFEASIBLE = (7, 5)


def reduced_uneven_boxed(seed, b):
    """Instance b of a reduced uneven batch (``seed``) with |u| <= 0.1,
    certified infeasible by an LP."""
    p = treegen.draw_batch_instances(8, seed=seed, scale=0.02, nx_range=(4, 10), N_range=(5, 10))[b]
    pr = treegen.with_boxes(p, ubox=0.1)
    assert not feasible(pr)
    return pr


def soft_rows(prob, seed=17, frac=0.5):
    """``prob`` with about ``frac`` of its finite rows made soft: weights
    U[0.5, 3], half of them with a Huber threshold U[0.05, 0.5], and every
    input row of the first non-leaf stage turned into an l1 penalty on u
    (bounds [0, 0])."""
    import dataclasses
    rng = np.random.default_rng(seed)
    lo, hi = box_rows(prob) if prob.F is None else (prob.zmin.copy(), prob.zmax.copy())
    m = prob.m
    wgt = np.full(m, np.inf)
    hub = np.zeros(m)
    fin = np.isfinite(lo) | np.isfinite(hi)
    pick = fin & (rng.random(m) < frac)
    wgt[pick] = rng.uniform(0.5, 3.0, pick.sum())
    hub[pick] = np.where(rng.random(pick.sum()) < 0.5, 0.0, rng.uniform(0.05, 0.5, pick.sum()))
    out = prob
    if prob.F is None:
        umin, umax = prob.umin.copy(), prob.umax.copy()
        umin[0], umax[0] = 0.0, 0.0
        out = dataclasses.replace(prob, umin=umin, umax=umax)
        nx, nu = prob.nx, prob.nu
        rows = nx + np.arange(nu)           # node 0's input rows
        wgt[rows] = 1.5
        hub[rows] = 0.0
    return treegen.with_soft_rows(out, wgt, hub)


def box_rows(prob):
    if prob.F is not None:
        return prob.zmin.copy(), prob.zmax.copy()
    t = prob.tree
    lo, hi = [], []
    for i in range(t.V):
        lo += list(prob.xmin[i])
        hi += list(prob.xmax[i])
        if i < t.Vnl:
            lo += list(prob.umin[i])
            hi += list(prob.umax[i])
    return np.array(lo), np.array(hi)


def hx_dense(dq, x, u):
    """H x in the dual layout from the split primal."""
    out = []
    for i in range(dq.V):
        out += list(x[i])
        if i < dq.Vnl:
            out += list(u[i])
    return np.array(out)


def fhat_dense(dq, y, x, u):
    """f-hat(y) = -f(x(y)) - <y, H x(y)>, with f from the dense objective."""
    X = np.concatenate([u.ravel(), x[1:].ravel()])
    return -(dq.objective(X)) - y @ hx_dense(dq, x, u)


# ------------------------------- the pins -------------------------------- #
def pin_kkt_affine(prob, seed=0):
    pb, fac = oracle.factor(prob)
    dq = DenseQP(prob)
    rng = np.random.default_rng(seed)
    err = 0.0
    for _ in range(3):
        y = rng.standard_normal(pb.m)
        x, u = oracle.sweep(pb, fac, y)
        xd, ud = dq.inner(y)
        scale = max(1.0, np.abs(xd).max(), np.abs(ud).max())
        err = max(err, np.abs(x - xd).max() / scale, np.abs(u - ud).max() / scale)
    return err


def pin_kkt_homogeneous(prob, seed=1):
    pb, fac = oracle.factor(prob)
    dq = DenseQP(prob)
    rng = np.random.default_rng(seed)
    err = 0.0
    for _ in range(3):
        r = rng.standard_normal(pb.m)
        x, u = oracle.sweep(pb, fac, r, homogeneous=True)
        xd, ud = dq.inner(r, homogeneous=True)
        scale = max(1.0, np.abs(xd).max(), np.abs(ud).max())
        err = max(err, np.abs(x - xd).max() / scale, np.abs(u - ud).max() / scale)
    return err


def pin_grad_fd(prob, seed=2):
    """Central differences of f-hat are exact for a quadratic at any step:
    (f-hat(y+v) - f-hat(y-v))/2 = <grad f-hat(y), v> = -<H x(y), v>."""
    pb, fac = oracle.factor(prob)
    dq = DenseQP(prob)
    rng = np.random.default_rng(seed)
    y = rng.standard_normal(pb.m)
    x, u = oracle.sweep(pb, fac, y)
    grad = -hx_dense(dq, x, u)
    err = 0.0
    for _ in range(4):
        v = rng.standard_normal(pb.m)
        xp, up = oracle.sweep(pb, fac, y + v)
        xm, um = oracle.sweep(pb, fac, y - v)
        fd = 0.5 * (fhat_dense(dq, y + v, xp, up) - fhat_dense(dq, y - v, xm, um))
        err = max(err, abs(fd - grad @ v) / max(1.0, abs(fd)))
    return err


def dense_hessian(pb, fac, precondition):
    """Columns of Hess f-hat = -(Hb x-hat(sc e_k)), from the oracle."""
    M = np.zeros((pb.m, pb.m))
    for k in range(pb.m):
        e = np.zeros(pb.m)
        e[k] = 1.0
        M[:, k] = -oracle.hess_neg(pb, fac, e, precondition)
    return M


def pin_hessian(prob):
    pb, fac = oracle.factor(prob)
    M = dense_hessian(pb, fac, False)
    sym = np.abs(M - M.T).max() / np.abs(M).max()
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    psd = max(0.0, -ev.min()) / ev.max()
    return sym, psd, ev.max()


def pin_precond_map(prob):
    """The scaled Hessian is diag(sqrt pi) Hess diag(sqrt pi)."""
    pb, fac = oracle.factor(prob)
    M = dense_hessian(pb, fac, False)
    Mb = dense_hessian(pb, fac, True)
    s = row_scale(prob)
    return np.abs(Mb - s[:, None] * M * s[None, :]).max() / np.abs(Mb).max()


def pin_fbe_conjugate(prob, lam, precondition, seed=3):
    """phi = f-hat(y) + g*(T) - lam <grad f-hat, R> + lam/2 ||R||^2 with g* the
    support function of the (scaled) box, f-hat from the dense objective."""
    pb, fac = oracle.factor(prob)
    dq = DenseQP(prob)
    rng = np.random.default_rng(seed)
    s = row_scale(prob) if precondition else np.ones(pb.m)
    lo, hi = box_rows(prob)
    lo, hi = s * lo, s * hi
    err = 0.0
    for _ in range(3):
        yb = rng.standard_normal(pb.m)
        yb[~np.isfinite(lo)] = 0.0
        ev = oracle.evaluate(pb, fac, yb, lam, precondition)
        y = s * yb
        fh = fhat_dense(dq, y, ev["x"], ev["u"])
        T, R = ev["T"], ev["R"]
        fin = np.isfinite(lo) & np.isfinite(hi)
        # on rows with infinite bounds the support function is finite only at 0
        gstar = np.sum(np.maximum(T[fin] * lo[fin], T[fin] * hi[fin]))
        inf_rows = np.abs(T[~fin]).max(initial=0.0)
        grad_fhat = -ev["Hbx"]
        phi2 = fh + gstar - lam * grad_fhat @ R + 0.5 * lam * R @ R
        err = max(err, abs(phi2 - ev["phi"]) / max(1.0, abs(phi2)), inf_rows)
    return err


def pin_fb_decrease(prob, lam, L, precondition, seed=4):
    """phi(T(y)) <= phi(y) - (lam/2)(1 - lam L)||R(y)||^2 for lam < 1/L."""
    pb, fac = oracle.factor(prob)
    rng = np.random.default_rng(seed)
    worst = -np.inf
    for _ in range(5):
        yb = rng.standard_normal(pb.m)
        ev = oracle.evaluate(pb, fac, yb, lam, precondition)
        ev2 = oracle.evaluate(pb, fac, ev["T"], lam, precondition)
        bound = ev["phi"] - 0.5 * lam * (1 - lam * L) * ev["R"] @ ev["R"]
        worst = max(worst, (ev2["phi"] - bound) / max(1.0, abs(ev["phi"])))
    return max(0.0, worst)


def reference_solution(prob):
    dq = DenseQP(prob)
    X, nu, ll, lu, cert = ipm(dq.G, dq.g, dq.E, dq.e, dq.lb, dq.ub)
    return dq, X, cert


def pin_solve(prob, method, precondition, eps=1e-9):
    pb, fac = oracle.factor(prob)
    L = oracle.power_iteration(pb, fac, precondition, 400)
    lam = 1.0 / (1.1 * L)
    res = oracle.solve(pb, fac, method, lam, eps=eps, max_iter=5000, precondition=precondition)
    dq, X, cert = reference_solution(prob)
    xd, ud = dq.split(X)
    scale = max(1.0, np.abs(xd).max(), np.abs(ud).max())
    perr = max(np.abs(res["x"] - xd).max(), np.abs(res["u"] - ud).max()) / scale
    opt = dq.objective(X)
    gap = abs(res["phi"] + opt) / max(1.0, abs(opt))
    return perr, gap, res, cert


def pin_lbfgs(seed=5, m=12, cnt=4):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, m))
    Hs = A @ A.T + m * np.eye(m)      # SPD "Hessian": pairs q = Hs s
    S = [rng.standard_normal(m) for _ in range(cnt)]
    Qs = [Hs @ s for s in S]
    # secant identity: B q_newest = s_newest
    d = oracle.lbfgs_direction(S, Qs, Qs[-1])
    sec = np.abs(-d - S[-1]).max() / np.abs(S[-1]).max()
    # dense inverse-BFGS recursion from gamma I
    gamma = S[-1] @ Qs[-1] / (Qs[-1] @ Qs[-1])
    Hk = gamma * np.eye(m)
    for s, q in zip(S, Qs):
        rho = 1.0 / (s @ q)
        V = np.eye(m) - rho * np.outer(q, s)
        Hk = V.T @ Hk @ V + rho * np.outer(s, s)
    g = rng.standard_normal(m)
    d = oracle.lbfgs_direction(S, Qs, g)
    dense = np.abs(d + Hk @ g).max() / np.abs(Hk @ g).max()
    return sec, dense
