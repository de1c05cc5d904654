"""Dense, structure-free references used to pin the oracle.

Everything here is built directly from the problem statement of Sec. II of the
paper (variables, dynamics, costs, boxes), as one dense quadratic program, with
no tree recursion.  It shares nothing with the oracle or the HIP library.

* ``DenseQP``             the whole problem P(p) as  min 1/2 X'GX + g'X + k
                          s.t. E X = e, lb <= X <= ub;
* ``DenseQP.inner``       x(y): the equality-constrained minimiser of
                          f(x) + <y, Hx> (the inner problem of Sec. III-D) by
                          one dense KKT solve;
* ``ipm``                 a primal-dual interior-point method with a KKT
                          certificate for the whole problem;
* ``active_set_bruteforce``  exhaustive enumeration of active sets for tiny
                          problems.
"""
from __future__ import annotations

import itertools

import numpy as np


class DenseQP:
    """Dense form of the problem with variables X = (u_0..u_{Vnl-1}, x_1..x_{V-1})."""

    def __init__(self, prob, x0=None):
        t = prob.tree
        nx, nu, V, Vnl = prob.nx, prob.nu, t.V, t.Vnl
        self.prob, self.nx, self.nu, self.V, self.Vnl = prob, nx, nu, V, Vnl
        p = prob.x0 if x0 is None else np.asarray(x0, dtype=float)
        self.p = p
        nU, nX = Vnl * nu, (V - 1) * nx
        n = nU + nX
        self.n = n

        def ui(i):
            return slice(i * nu, (i + 1) * nu)

        def xi(i):
            assert i >= 1
            return slice(nU + (i - 1) * nx, nU + i * nx)

        self.ui, self.xi = ui, xi
        G = np.zeros((n, n))
        g = np.zeros(n)
        k = 0.0
        for i in range(Vnl):
            pi = t.prob[i]
            Q, R = prob.Q[i], prob.R[i]
            S = prob.S[i] if prob.S is not None else np.zeros((nu, nx))
            q = prob.q[i] if prob.q is not None else np.zeros(nx)
            r = prob.r[i] if prob.r is not None else np.zeros(nu)
            # pi * ([x;u]' [[Q,S'],[S,R]] [x;u] + q'x + r'u)
            G[ui(i), ui(i)] += 2 * pi * R
            g[ui(i)] += pi * r
            if i == 0:
                g[ui(i)] += 2 * pi * S @ p
                k += pi * (p @ Q @ p + q @ p)
            else:
                G[xi(i), xi(i)] += 2 * pi * Q
                G[ui(i), xi(i)] += 2 * pi * S
                G[xi(i), ui(i)] += 2 * pi * S.T
                g[xi(i)] += pi * q
        for j in range(Vnl, V):
            pj = t.prob[j]
            G[xi(j), xi(j)] += 2 * pj * prob.P[j - Vnl]
            if prob.p is not None:
                g[xi(j)] += pj * prob.p[j - Vnl]
        self.G, self.g, self.k = G, g, k
        # dynamics  x_j - A_j x_i - B_j u_i = c_j
        E = np.zeros(((V - 1) * nx, n))
        e = np.zeros((V - 1) * nx)
        for j in range(1, V):
            i = t.anc[j]
            rows = slice((j - 1) * nx, j * nx)
            E[rows, xi(j)] = np.eye(nx)
            E[rows, ui(i)] = -prob.B[j]
            e[rows] = prob.c[j]
            if i == 0:
                e[rows] += prob.A[j] @ p
            else:
                E[rows, xi(i)] = -prob.A[j]
        self.E, self.e = E, e
        lb = np.empty(n)
        ub = np.empty(n)
        for i in range(Vnl):
            lb[ui(i)] = prob.umin[i]
            ub[ui(i)] = prob.umax[i]
        for j in range(1, V):
            lb[xi(j)] = prob.xmin[j]
            ub[xi(j)] = prob.xmax[j]
        self.lb, self.ub = lb, ub

    # -- dual-vector layout (non-leaf: x rows then u rows; leaves: x rows) --
    def dual_blocks(self):
        nx, nu, Vnl = self.nx, self.nu, self.Vnl
        out, o = [], 0
        for i in range(self.V):
            w = nx + nu if i < Vnl else nx
            out.append((i, o))
            o += w
        return out, o

    def split(self, X):
        """X -> (x [V][nx] with x_0 = p, u [Vnl][nu])."""
        x = np.zeros((self.V, self.nx))
        u = np.zeros((self.Vnl, self.nu))
        x[0] = self.p
        for i in range(self.Vnl):
            u[i] = X[self.ui(i)]
        for j in range(1, self.V):
            x[j] = X[self.xi(j)]
        return x, u

    def H_linear(self, y):
        """(h, hconst): <y, H x> = h' X + hconst for the stacked variables
        (y in the constraint layout; the map of ``constraint_matrix``)."""
        Hd, hcv = constraint_matrix(self)
        assert y.shape == (Hd.shape[0],)
        return Hd.T @ y, float(hcv @ y)

    def inner(self, y, homogeneous=False):
        """x(y) by a dense KKT solve of min f(X) + <y, HX> s.t. EX = e.

        With ``homogeneous`` the constant data (c, p, the linear cost terms)
        are dropped, which gives the linear part x-hat(y)."""
        h, _ = self.H_linear(np.asarray(y, dtype=float))
        if homogeneous:
            dq = DenseQP._homogeneous(self.prob)
            return dq.inner(y)
        n, me = self.n, self.E.shape[0]
        Kkt = np.zeros((n + me, n + me))
        Kkt[:n, :n] = self.G
        Kkt[:n, n:] = self.E.T
        Kkt[n:, :n] = self.E
        rhs = np.concatenate([-(self.g + h), self.e])
        sol = np.linalg.solve(Kkt, rhs)
        return self.split(sol[:n])

    @staticmethod
    def _homogeneous(prob):
        import dataclasses
        z = dataclasses.replace(prob, c=np.zeros_like(prob.c), q=None, r=None, p=None,
                                x0=np.zeros_like(prob.x0))
        return DenseQP(z)

    def objective(self, X):
        return 0.5 * X @ self.G @ X + self.g @ X + self.k


def ipm(G, g, E, e, lb, ub, tol=1e-12, max_iter=200):
    """Primal-dual interior point (Mehrotra predictor-corrector) for
    min 1/2 X'GX + g'X s.t. EX = e, lb <= X <= ub (infinite bounds allowed).

    Returns (X, nu, lam_l, lam_u, cert) where cert holds the final
    stationarity, primal feasibility and complementarity residuals."""
    n = G.shape[0]
    L = np.where(np.isfinite(lb))[0]
    U = np.where(np.isfinite(ub))[0]
    X = np.zeros(n)
    for ix in range(n):  # start strictly inside the box
        lo, hi = lb[ix], ub[ix]
        if np.isfinite(lo) and np.isfinite(hi):
            X[ix] = 0.5 * (lo + hi)
        elif np.isfinite(lo):
            X[ix] = lo + 1.0
        elif np.isfinite(hi):
            X[ix] = hi - 1.0
    sl = np.maximum(X[L] - lb[L], 1.0)
    su = np.maximum(ub[U] - X[U], 1.0)
    zl = np.ones(L.size)
    zu = np.ones(U.size)
    nu = np.zeros(E.shape[0])
    me = E.shape[0]

    def residuals(X, nu, zl, zu, sl, su):
        rd = G @ X + g - E.T @ nu
        rd[L] -= zl
        rd[U] += zu
        rp = E @ X - e
        rl = X[L] - lb[L] - sl
        ru = ub[U] - X[U] - su
        return rd, rp, rl, ru

    cert = {}
    for _ in range(max_iter):
        rd, rp, rl, ru = residuals(X, nu, zl, zu, sl, su)
        mu = (sl @ zl + su @ zu) / max(1, L.size + U.size)
        cert = dict(stat=np.abs(rd).max(initial=0.0), feas=max(np.abs(rp).max(initial=0.0),
                    np.abs(rl).max(initial=0.0), np.abs(ru).max(initial=0.0)), comp=mu)
        if cert["stat"] < tol and cert["feas"] < tol and mu < tol:
            break

        def solve_dir(rsl, rsu):
            # eliminate slacks and bound multipliers:
            # dzl = (rsl - zl*dsl)/sl with dsl = dX[L] + rl ; etc.
            W = np.zeros(n)
            r1 = -rd.copy()
            W[L] += zl / sl
            r1[L] += (rsl - zl * rl) / sl
            W[U] += zu / su
            r1[U] -= (rsu - zu * ru) / su
            K = np.zeros((n + me, n + me))
            K[:n, :n] = G + np.diag(W)
            K[:n, n:] = -E.T
            K[n:, :n] = E
            sol = np.linalg.solve(K, np.concatenate([r1, -rp]))
            dX, dnu = sol[:n], sol[n:]
            dsl = dX[L] + rl
            dsu = -dX[U] + ru
            dzl = (rsl - zl * dsl) / sl
            dzu = (rsu - zu * dsu) / su
            return dX, dnu, dzl, dzu, dsl, dsu

        def step_len(v, dv):
            neg = dv < 0
            return min(1.0, np.min(-v[neg] / dv[neg])) if neg.any() else 1.0

        # predictor (affine scaling)
        aff = solve_dir(-sl * zl, -su * zu)
        a_p = min(step_len(sl, aff[4]), step_len(su, aff[5]))
        a_d = min(step_len(zl, aff[2]), step_len(zu, aff[3]))
        mu_aff = ((sl + a_p * aff[4]) @ (zl + a_d * aff[2]) +
                  (su + a_p * aff[5]) @ (zu + a_d * aff[3])) / max(1, L.size + U.size)
        sigma = (mu_aff / mu) ** 3 if mu > 0 else 0.0
        # corrector
        cor = solve_dir(-sl * zl - aff[4] * aff[2] + sigma * mu,
                        -su * zu - aff[5] * aff[3] + sigma * mu)
        dX, dnu, dzl, dzu, dsl, dsu = cor
        a_p = 0.99 * min(step_len(sl, dsl), step_len(su, dsu))
        a_d = 0.99 * min(step_len(zl, dzl), step_len(zu, dzu))
        a_p = min(a_p, 1.0)
        a_d = min(a_d, 1.0)
        X = X + a_p * dX
        sl = sl + a_p * dsl
        su = su + a_p * dsu
        nu = nu + a_d * dnu
        zl = zl + a_d * dzl
        zu = zu + a_d * dzu
    lam_l = np.zeros(n)
    lam_u = np.zeros(n)
    lam_l[L] = zl
    lam_u[U] = zu
    return X, nu, lam_l, lam_u, cert


def active_set_bruteforce(G, g, E, e, lb, ub, tol=1e-10):
    """Exhaustive active-set enumeration for tiny QPs: every variable is at its
    lower bound, its upper bound or free; each choice is an equality QP; the
    feasible one whose bound multipliers have the right signs is optimal."""
    n = G.shape[0]
    me = E.shape[0]
    best = None
    for choice in itertools.product((0, 1, 2), repeat=n):  # 0 free, 1 lo, 2 hi
        fixed = [ix for ix in range(n) if choice[ix] != 0]
        if any((choice[ix] == 1 and not np.isfinite(lb[ix])) or
               (choice[ix] == 2 and not np.isfinite(ub[ix])) for ix in fixed):
            continue
        nf = len(fixed)
        F = np.zeros((nf, n))
        fv = np.zeros(nf)
        for r, ix in enumerate(fixed):
            F[r, ix] = 1.0
            fv[r] = lb[ix] if choice[ix] == 1 else ub[ix]
        A = np.vstack([E, F])
        b = np.concatenate([e, fv])
        K = np.zeros((n + me + nf, n + me + nf))
        K[:n, :n] = G
        K[:n, n:] = -A.T
        K[n:, :n] = A
        try:
            sol = np.linalg.solve(K, np.concatenate([-g, b]))
        except np.linalg.LinAlgError:
            continue
        X = sol[:n]
        mult = sol[n + me:]
        if (X < lb - tol).any() or (X > ub + tol).any():
            continue
        ok = True
        for r, ix in enumerate(fixed):
            # stationarity G X + g = E'nu + F'mult: a lower bound pushes up
            # (mult >= 0), an upper bound pushes down (mult <= 0)
            if choice[ix] == 1 and mult[r] < -tol:
                ok = False
            if choice[ix] == 2 and mult[r] > tol:
                ok = False
        if ok:
            obj = 0.5 * X @ G @ X + g @ X
            if best is None or obj < best[1] - 1e-12:
                best = (X, obj)
    return best


# ---------------------- constraint map and soft rows ---------------------- #
def constraint_matrix(dq):
    """The map of Sec. II-B written out densely: z = Hd X + hc in the dual
    (constraint) layout, Hd [m][n], from the problem statement (F, G, FN at
    every node, or the rows (x_i, u_i) and x_j themselves).  x_0 = p is data,
    so the root's state part goes to the constant hc."""
    prob = dq.prob
    nx, nu, V, Vnl = dq.nx, dq.nu, dq.V, dq.Vnl
    if prob.F is None:
        F, G, FN = (np.vstack([np.eye(nx), np.zeros((nu, nx))]),
                    np.vstack([np.zeros((nx, nu)), np.eye(nu)]), np.eye(nx))
    else:
        F, G, FN = prob.F, prob.G, prob.FN
    rows = []
    for i in range(V):
        rows.append(F.shape[0] if i < Vnl else FN.shape[0])
    m = int(sum(rows))
    Hd = np.zeros((m, dq.n))
    hc = np.zeros(m)
    o = 0
    for i in range(V):
        r = rows[i]
        Fi = F if i < Vnl else FN
        if i == 0:
            hc[o:o + r] = Fi @ dq.p
        else:
            Hd[o:o + r, dq.xi(i)] = Fi
        if i < Vnl:
            Hd[o:o + r, dq.ui(i)] = G
        o += r
    return Hd, hc


def row_bounds(prob):
    """Lower / upper bound of every constraint row (dual layout)."""
    if prob.F is not None:
        return np.asarray(prob.zmin, float), np.asarray(prob.zmax, float)
    t = prob.tree
    lo, hi = [], []
    for i in range(t.V):
        lo += list(prob.xmin[i])
        hi += list(prob.xmax[i])
        if i < t.Vnl:
            lo += list(prob.umin[i])
            hi += list(prob.umax[i])
    return np.array(lo), np.array(hi)


def row_prob(prob):
    """Probability of the node owning each constraint row."""
    t = prob.tree
    out = []
    for i in range(t.V):
        r = prob.nc if i < t.Vnl else prob.ncN
        out += [t.prob[i]] * r
    return np.array(out)


def soft_qp(prob):
    """The whole problem with a general constraint map and soft rows as one
    QP for ``ipm``: variables (X, z, slacks) with z = Hd X + hc; a hard row
    bounds z directly; a soft row k (weight w, Huber threshold d, node
    probability pi) costs pi w (e + q^2 / (2 d)) with e, q >= 0 (no q when
    d = 0) and z - hi = e + q + a (a <= 0), z - lo = b - e - q (b >= 0): at
    the optimum e + q is the distance of z to [lo, hi] and the cost its Huber
    function (min of e + q^2/(2d) over e + q >= t is t^2/(2d) for t <= d,
    else t - d/2).  Returns (G, g, k, E, e, lb, ub, n, dq) with n the size of
    X."""
    dq = DenseQP(prob)
    Hd, hc = constraint_matrix(dq)
    lo, hi = row_bounds(prob)
    m, n = Hd.shape
    pi = row_prob(prob)
    wgt = prob.wgt if prob.wgt is not None else np.full(m, np.inf)
    hub = prob.hub if prob.hub is not None else np.zeros(m)
    # every bound sits on the z rows (with the identity map too), so X is free
    lbs, ubs, diag, lin = [-np.inf] * n, [np.inf] * n, [0.0] * n, list(dq.g)

    def new_var(lo_, hi_, quad=0.0, cost=0.0):
        lbs.append(lo_)
        ubs.append(hi_)
        diag.append(quad)
        lin.append(cost)
        return len(lbs) - 1

    eq = []          # (dict var -> coefficient, rhs)
    for r in range(dq.E.shape[0]):
        eq.append(({j: dq.E[r, j] for j in np.nonzero(dq.E[r])[0]}, dq.e[r]))
    for k in range(m):
        soft = np.isfinite(wgt[k])
        z = new_var(-np.inf if soft else lo[k], np.inf if soft else hi[k])
        row = {j: -Hd[k, j] for j in np.nonzero(Hd[k])[0]}
        row[z] = 1.0
        eq.append((row, hc[k]))
        if not soft:
            continue
        w, d = wgt[k] * pi[k], hub[k]
        e = new_var(0.0, np.inf, cost=w)
        q = new_var(0.0, np.inf, quad=w / d) if d > 0 else None
        if np.isfinite(hi[k]):
            a = new_var(-np.inf, 0.0)
            row = {z: 1.0, e: -1.0, a: -1.0}
            if q is not None:
                row[q] = -1.0
            eq.append((row, hi[k]))
        if np.isfinite(lo[k]):
            b = new_var(0.0, np.inf)
            row = {z: 1.0, e: 1.0, b: -1.0}
            if q is not None:
                row[q] = 1.0
            eq.append((row, lo[k]))
    N = len(lbs)
    Gm = np.zeros((N, N))
    Gm[:n, :n] = dq.G
    Gm[np.arange(n, N), np.arange(n, N)] = diag[n:]
    E = np.zeros((len(eq), N))
    ev = np.zeros(len(eq))
    for r, (row, rhs) in enumerate(eq):
        for j, v in row.items():
            E[r, j] = v
        ev[r] = rhs
    return Gm, np.array(lin), dq.k, E, ev, np.array(lbs), np.array(ubs), n, dq


def fista_dense(prob, lam, iters, precondition=True):
    """Textbook FISTA (Beck and Teboulle 2009, the t_k form) on the dual
    min f-hat(y) + g*(y) in the scaled variables, with hard rows only:
    the gradient -Hb x(y) comes from the dense KKT solve of the inner problem
    and the prox of lam g* from the Moreau decomposition
    prox_{lam g*}(v) = v - lam proj_box(v / lam).  Returns the extrapolated
    points y_1 .. y_{iters+1} of that form (y_1 = 0)."""
    dq = DenseQP(prob)
    Hd, hc = constraint_matrix(dq)
    lo, hi = row_bounds(prob)
    s = np.sqrt(row_prob(prob)) if precondition else np.ones(Hd.shape[0])
    n, me = dq.n, dq.E.shape[0]
    K = np.zeros((n + me, n + me))
    K[:n, :n] = dq.G
    K[:n, n:] = dq.E.T
    K[n:, :n] = dq.E
    Kinv = np.linalg.inv(K)

    def grad(yb):
        # x(y) minimises f(X) + <y, Hd X + hc> s.t. EX = e, y = s * yb
        rhs = np.concatenate([-(dq.g + Hd.T @ (s * yb)), dq.e])
        X = (Kinv @ rhs)[:n]
        return -(s * (Hd @ X + hc))

    m = Hd.shape[0]
    yk = np.zeros(m)          # the extrapolated point
    x_prev = np.zeros(m)
    t = 1.0
    out = [yk.copy()]
    for _ in range(iters):
        v = yk - lam * grad(yk)
        x_new = v - lam * np.clip(v / lam, s * lo, s * hi)
        t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        yk = x_new + ((t - 1.0) / t_new) * (x_new - x_prev)
        x_prev, t = x_new, t_new
        out.append(yk.copy())
    return out
