"""Seeded synthetic scenario trees and problem data.

This module only draws inputs: tree shapes, dynamics, costs, boxes, initial
states and dual vectors.  It holds none of the solver's arithmetic, so both
the CPU oracle and the HIP library can be fed from it without sharing any
computation.

Conventions (the problem statement of Sec. II-A/II-B of the paper):

* nodes are numbered stage-major: root is 0, the nodes of stage t are
  ``[stage_ptr[t], stage_ptr[t+1])``, the children of node i are the
  contiguous range ``[child_ptr[i], child_ptr[i+1])`` and all leaves sit at
  stage N, numbered last;
* ``prob[i]`` is the node probability; the children of a node split their
  parent's probability uniformly, so every stage sums to one;
* dynamics ``x_j = A_j x_i + B_j u_i + c_j`` live on the child j of i
  (``A[0]``, ``B[0]``, ``c[0]`` are unused and zero);
* costs ``Q, R`` (and optional ``S, q, r``) live on non-leaf nodes, ``P``
  (and optional ``p``) on leaves;
* boxes ``xmin <= x_i <= xmax`` on every node and ``umin <= u_i <= umax`` on
  non-leaf nodes; the root state is data, so its rows carry +-inf.

Draw order for a problem is fixed: G (for A), B, c, then the cost diagonals,
then x0.  Every array is C-contiguous float64 / int32.
"""
from __future__ import annotations

import concurrent.futures as _cf
import dataclasses
import os

import numpy as np

__all__ = [
    "Tree", "Problem", "tree_from_counts", "uniform_tree", "capped_tree",
    "draw_problem", "make_workload", "draw_batch_instances", "random_dual",
    "WORKLOAD_SHAPES",
]


@dataclasses.dataclass
class Tree:
    N: int
    stage_ptr: np.ndarray  # int32 [N+2]
    anc: np.ndarray        # int32 [V], -1 at the root
    child_ptr: np.ndarray  # int32 [Vnl+1]
    prob: np.ndarray       # float64 [V]

    @property
    def V(self) -> int:
        return int(self.stage_ptr[-1])

    @property
    def Vnl(self) -> int:
        return int(self.stage_ptr[self.N])

    @property
    def Vl(self) -> int:
        return self.V - self.Vnl


@dataclasses.dataclass
class Problem:
    tree: Tree
    nx: int
    nu: int
    A: np.ndarray      # [V][nx][nx]
    B: np.ndarray      # [V][nx][nu]
    c: np.ndarray      # [V][nx]
    Q: np.ndarray      # [Vnl][nx][nx]
    R: np.ndarray      # [Vnl][nu][nu]
    P: np.ndarray      # [Vl][nx][nx]
    xmin: np.ndarray   # [V][nx]
    xmax: np.ndarray   # [V][nx]
    umin: np.ndarray   # [Vnl][nu]
    umax: np.ndarray   # [Vnl][nu]
    x0: np.ndarray     # [nx]
    S: np.ndarray | None = None   # [Vnl][nu][nx]
    q: np.ndarray | None = None   # [Vnl][nx]
    r: np.ndarray | None = None   # [Vnl][nu]
    p: np.ndarray | None = None   # [Vl][nx]
    name: str = ""
    # optional constraint map of Sec. II-B, the same at every node:
    # z_i = F x_i + G u_i (non-leaf), z_j = FN x_j (leaf), bounded by
    # zmin <= z <= zmax in the dual layout; F None: the rows (x_i, u_i), x_j
    F: np.ndarray | None = None      # [nc][nx]
    G: np.ndarray | None = None      # [nc][nu]
    FN: np.ndarray | None = None     # [ncN][nx]
    zmin: np.ndarray | None = None   # [m]
    zmax: np.ndarray | None = None   # [m]
    # optional soft rows (dual layout): row k of node i costs
    # pi_i wgt[k] huber_{hub[k]}(dist(z_k, [lo_k, hi_k])); wgt = inf: hard
    wgt: np.ndarray | None = None    # [m]
    hub: np.ndarray | None = None    # [m]

    @property
    def nc(self) -> int:
        return self.nx + self.nu if self.F is None else int(self.F.shape[0])

    @property
    def ncN(self) -> int:
        return self.nx if self.F is None else int(self.FN.shape[0])

    @property
    def m_xu(self) -> int:
        """Length of the (x, u) layout: (nx+nu) rows per non-leaf node, nx per leaf."""
        t = self.tree
        return t.Vnl * (self.nx + self.nu) + t.Vl * self.nx

    @property
    def m(self) -> int:
        """Dual dimension: the constraint rows, nc per non-leaf node and ncN
        per leaf ((nx+nu) and nx without a constraint map)."""
        t = self.tree
        return t.Vnl * self.nc + t.Vl * self.ncN


def tree_from_counts(counts: list) -> Tree:
    """Build a tree from per-stage child counts.

    ``counts[t]`` lists the number of children of each node of stage t, in
    node order; the children of a stage are numbered contiguously in parent
    order.  Children split the parent's probability uniformly.
    """
    N = len(counts)
    sizes = [1]
    for t in range(N):
        ct = np.asarray(counts[t], dtype=np.int64)
        if ct.shape != (sizes[-1],):
            raise ValueError(f"stage {t}: expected {sizes[-1]} counts, got {ct.shape}")
        if (ct < 1).any():
            raise ValueError("every non-leaf node needs at least one child")
        sizes.append(int(ct.sum()))
    stage_ptr = np.zeros(N + 2, dtype=np.int64)
    stage_ptr[1:] = np.cumsum(sizes)
    V = int(stage_ptr[-1])
    Vnl = int(stage_ptr[N])
    anc = np.full(V, -1, dtype=np.int64)
    child_ptr = np.zeros(Vnl + 1, dtype=np.int64)
    prob = np.zeros(V)
    prob[0] = 1.0
    for t in range(N):
        ct = np.asarray(counts[t], dtype=np.int64)
        parents = np.arange(stage_ptr[t], stage_ptr[t + 1])
        first = stage_ptr[t + 1] + np.concatenate([[0], np.cumsum(ct)[:-1]])
        child_ptr[parents] = first
        kids_parent = np.repeat(parents, ct)
        anc[stage_ptr[t + 1]:stage_ptr[t + 2]] = kids_parent
        prob[stage_ptr[t + 1]:stage_ptr[t + 2]] = np.repeat(prob[parents] / ct, ct)
    child_ptr[Vnl] = V
    return Tree(N=N, stage_ptr=stage_ptr.astype(np.int32), anc=anc.astype(np.int32),
                child_ptr=child_ptr.astype(np.int32), prob=prob)


def uniform_tree(branching: list) -> Tree:
    """Every node of stage t has ``branching[t]`` children (t = 0..N-1)."""
    counts, n = [], 1
    for b in branching:
        counts.append([int(b)] * n)
        n *= int(b)
    return tree_from_counts(counts)


def capped_tree(N: int, scenarios: int, b0: int) -> Tree:
    """Stage sizes n_{t+1} = min(b0 * n_t, S); at the stage where the cap bites
    the children are split as evenly as possible (the first ``S mod n_t``
    parents get one more), and from there on every node has one child."""
    counts, n = [], 1
    for _ in range(N):
        if n >= scenarios:
            ct = [1] * n
        elif b0 * n <= scenarios:
            ct = [b0] * n
        else:
            base, extra = divmod(scenarios, n)
            ct = [base + 1] * extra + [base] * (n - extra)
        counts.append(ct)
        n = sum(ct)
    return tree_from_counts(counts)


def _spectral_radius(G: np.ndarray, threads: int | None = None) -> np.ndarray:
    """Batched spectral radius, split over threads for large stacks."""
    if G.shape[0] == 0:
        return np.zeros(0)
    nthreads = min(16, os.cpu_count() or 1) if threads is None else threads
    if G.shape[0] < 512 or nthreads == 1:
        return np.abs(np.linalg.eigvals(G)).max(axis=-1)
    chunks = np.array_split(np.arange(G.shape[0]), nthreads * 4)
    out = np.empty(G.shape[0])

    def work(ix):
        out[ix] = np.abs(np.linalg.eigvals(G[ix])).max(axis=-1)

    with _cf.ThreadPoolExecutor(nthreads) as ex:
        list(ex.map(work, chunks))
    return out


def draw_problem(tree: Tree, nx: int, nu: int, rng: np.random.Generator, *,
                 rho: float = 0.95, c_std: float = 0.1,
                 qdiag=None, rdiag=None, xbox: float = 5.0, ubox: float = 1.0,
                 x0_range: float = 2.0, cross_terms: bool = False,
                 name: str = "", threads: int | None = None) -> Problem:
    """Draw dynamics, costs, boxes and x0 for a tree.

    A_j = rho * G / spectral_radius(G) with G ~ N(0,1), B_j ~ N(0,1),
    c_j ~ N(0, c_std^2).  ``qdiag``/``rdiag`` are either None (Q = I,
    R = 0.1 I) or a pair (lo, hi) for per-node diagonals ~ U[lo, hi].  With
    ``cross_terms`` the optional S, q, r, p terms are drawn too (S small
    enough that the joint cost block stays positive semidefinite).
    """
    V, Vnl, Vl = tree.V, tree.Vnl, tree.Vl
    A = np.zeros((V, nx, nx))
    B = np.zeros((V, nx, nu))
    c = np.zeros((V, nx))
    G = rng.standard_normal((V - 1, nx, nx))
    A[1:] = rho * G / _spectral_radius(G, threads)[:, None, None]
    del G
    B[1:] = rng.standard_normal((V - 1, nx, nu))
    c[1:] = c_std * rng.standard_normal((V - 1, nx))
    if qdiag is None:
        Q = np.broadcast_to(np.eye(nx), (Vnl, nx, nx)).copy()
    else:
        Q = np.zeros((Vnl, nx, nx))
        Q[:, np.arange(nx), np.arange(nx)] = rng.uniform(qdiag[0], qdiag[1], (Vnl, nx))
    if rdiag is None:
        R = np.broadcast_to(0.1 * np.eye(nu), (Vnl, nu, nu)).copy()
    else:
        R = np.zeros((Vnl, nu, nu))
        R[:, np.arange(nu), np.arange(nu)] = rng.uniform(rdiag[0], rdiag[1], (Vnl, nu))
    P = np.broadcast_to(np.eye(nx), (Vl, nx, nx)).copy()
    S = q = r = p = None
    if cross_terms:
        # |S| small relative to Q = I and R: the joint block stays PSD when
        # ||S||_2^2 <= lambda_min(Q) * lambda_min(R).
        lamR = np.linalg.eigvalsh(R)[:, :1]
        lamQ = np.linalg.eigvalsh(Q)[:, :1]
        S = rng.standard_normal((Vnl, nu, nx))
        nrm = np.linalg.norm(S, ord=2, axis=(1, 2))
        S *= (0.9 * np.sqrt(lamR[:, 0] * lamQ[:, 0]) / nrm)[:, None, None]
        q = rng.standard_normal((Vnl, nx))
        r = rng.standard_normal((Vnl, nu))
        p = rng.standard_normal((Vl, nx))
    xmin = np.full((V, nx), -xbox)
    xmax = np.full((V, nx), xbox)
    xmin[0] = -np.inf
    xmax[0] = np.inf
    umin = np.full((Vnl, nu), -ubox)
    umax = np.full((Vnl, nu), ubox)
    x0 = rng.uniform(-x0_range, x0_range, nx)
    return Problem(tree=tree, nx=nx, nu=nu, A=A, B=B, c=c, Q=Q, R=R, P=P,
                   xmin=xmin, xmax=xmax, umin=umin, umax=umax, x0=x0,
                   S=S, q=q, r=r, p=p, name=name)


# Shapes of the single-tree workloads (the uneven batch draws one tree per
# instance, draw_batch_instances):
#   tiny    nx=4,  nu=2,  N=5,  branching 2 at stages 0-2 (8 scenarios)
#   large   nx=50, nu=30, N=20, branching 4 at stages 0-5 (4096 scenarios)
#   warm    nx=20, nu=10, N=15, branching 3 at stages 0-4 (243 scenarios)
#   shared  nx=64, nu=32, N=20, branching 4 at stages 0-6 (16384 scenarios)
WORKLOAD_SHAPES = {
    "tiny": dict(nx=4, nu=2, branching=[2, 2, 2, 1, 1], seed=1000),
    "large": dict(nx=50, nu=30, branching=[4] * 6 + [1] * 14, seed=1001),
    "warm": dict(nx=20, nu=10, branching=[3] * 5 + [1] * 10, seed=1003),
    "shared": dict(nx=64, nu=32, branching=[4] * 7 + [1] * 13, seed=1004),
}


def make_workload(name: str, seed: int | None = None) -> Problem:
    """One of the single-tree workloads of WORKLOAD_SHAPES (its own default seed)."""
    if name not in WORKLOAD_SHAPES:
        raise ValueError(f"{name!r} is not a single-tree workload")
    sh = WORKLOAD_SHAPES[name]
    rng = np.random.default_rng(sh["seed"] if seed is None else seed)
    tree = uniform_tree(sh["branching"])
    kw = {}
    if name == "large":
        kw = dict(qdiag=(0.5, 2.0), rdiag=(0.05, 0.5))
    if name in ("warm", "shared"):
        kw = dict(x0_range=3.0)
    return draw_problem(tree, sh["nx"], sh["nu"], rng, name=name, **kw)


def draw_batch_instances(count: int = 256, seed: int = 1002, *,
                         nx_range=(8, 32), N_range=(10, 30),
                         S_range=(16, 1024), b0_range=(2, 8),
                         scale: float = 1.0) -> list:
    """Uneven batch of independent instances (the uneven-batch workload).

    Per instance: nx ~ U{nx_range}, nu = nx // 2, N ~ U{N_range},
    scenarios S ~ U{S_range} (times ``scale``, for reduced test sizes),
    first-stage branching b0 ~ U{b0_range}; the tree follows ``capped_tree``.
    The sizes come from ``default_rng(seed)`` in instance order; instance b's
    matrices and vectors from its own ``default_rng([seed, b])``, so the
    instances are drawn in parallel threads with a result independent of
    the thread count.
    """
    rng = np.random.default_rng(seed)
    shapes = []
    for b in range(count):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        nu = max(1, nx // 2)
        N = int(rng.integers(N_range[0], N_range[1] + 1))
        S = int(rng.integers(S_range[0], S_range[1] + 1))
        S = max(1, int(round(S * scale)))
        b0 = int(rng.integers(b0_range[0], b0_range[1] + 1))
        shapes.append((nx, nu, N, S, b0))

    def one(b):
        nx, nu, N, S, b0 = shapes[b]
        return draw_problem(capped_tree(N, S, b0), nx, nu, np.random.default_rng([seed, b]),
                            name=f"batch[{b}]", threads=1)

    nthreads = min(16, os.cpu_count() or 1)
    if count < 4 or nthreads == 1:
        return [one(b) for b in range(count)]
    with _cf.ThreadPoolExecutor(nthreads) as ex:
        return list(ex.map(one, range(count)))


def random_dual(prob: Problem, rng: np.random.Generator, nrhs: int | None = None,
                scale: float = 1.0) -> np.ndarray:
    """Gaussian dual vector(s) of the problem's dual dimension."""
    shape = (prob.m,) if nrhs is None else (nrhs, prob.m)
    return scale * rng.standard_normal(shape)


def draw_warm_instances(base: Problem, count: int, seed: int, *, x0_range: float = 3.0,
                        c_std: float = 0.1) -> list:
    """Instances of a fixed tree and fixed matrices that differ only in the
    initial state x0 ~ U[-x0_range, x0_range]^nx and the disturbance path
    c_j ~ N(0, c_std^2) (the learned warm start's training and held-out draws)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        x0 = rng.uniform(-x0_range, x0_range, base.nx)
        c = np.zeros_like(base.c)
        c[1:] = c_std * rng.standard_normal(c[1:].shape)
        out.append(dataclasses.replace(base, c=c, x0=x0, name=f"{base.name}-draw{k}"))
    return out


def with_boxes(prob: Problem, xbox: float | None = None, ubox: float | None = None) -> Problem:
    """The same problem with uniform boxes |x| <= xbox (root free), |u| <= ubox."""
    xmin, xmax, umin, umax = prob.xmin, prob.xmax, prob.umin, prob.umax
    if xbox is not None:
        xmin = np.full_like(prob.xmin, -xbox)
        xmax = np.full_like(prob.xmax, xbox)
        xmin[0], xmax[0] = -np.inf, np.inf
    if ubox is not None:
        umin = np.full_like(prob.umin, -ubox)
        umax = np.full_like(prob.umax, ubox)
    return dataclasses.replace(prob, xmin=xmin, xmax=xmax, umin=umin, umax=umax)


def with_constraint_map(prob: Problem, F: np.ndarray, G: np.ndarray, FN: np.ndarray,
                        lo: float | np.ndarray, hi: float | np.ndarray,
                        loN: float | np.ndarray, hiN: float | np.ndarray) -> Problem:
    """The same problem constrained by z_i = F x_i + G u_i in [lo, hi] at every
    non-leaf node and z_j = FN x_j in [loN, hiN] at every leaf (Sec. II-B);
    the box arrays are kept but no longer bound anything."""
    t = prob.tree
    nc, ncN = F.shape[0], FN.shape[0]
    zmin = np.concatenate([np.broadcast_to(lo, (t.Vnl, nc)).ravel(),
                           np.broadcast_to(loN, (t.Vl, ncN)).ravel()]).astype(np.float64)
    zmax = np.concatenate([np.broadcast_to(hi, (t.Vnl, nc)).ravel(),
                           np.broadcast_to(hiN, (t.Vl, ncN)).ravel()]).astype(np.float64)
    return dataclasses.replace(prob, F=np.ascontiguousarray(F, dtype=np.float64),
                               G=np.ascontiguousarray(G, dtype=np.float64),
                               FN=np.ascontiguousarray(FN, dtype=np.float64), zmin=zmin, zmax=zmax,
                               wgt=None, hub=None)


def with_soft_rows(prob: Problem, wgt: np.ndarray, hub: np.ndarray | None = None) -> Problem:
    """Soft rows (dual layout): row k costs pi wgt[k] huber_{hub[k]}(distance of
    z_k to its bounds); wgt[k] = inf keeps row k hard."""
    wgt = np.ascontiguousarray(wgt, dtype=np.float64)
    hub = np.zeros_like(wgt) if hub is None else np.ascontiguousarray(hub, dtype=np.float64)
    assert wgt.shape == (prob.m,) and hub.shape == (prob.m,)
    return dataclasses.replace(prob, wgt=wgt, hub=hub)


# --------------------- spring-mass-damper array (Sec. IV-A) --------------------- #
def spring_mass_dynamics(M: int = 5, mass: float = 5.0, ks: float = 1.0, bd: float = 0.1,
                         Ts: float = 0.5):
    """(A, B) of the array of M masses between two walls: M + 1 springs
    (stiffness ks) and dampers (coefficient bd), M - 1 actuators, the one
    between masses j and j + 1 pushing them apart with force u_j.  State
    (p_1..p_M, v_1..v_M); Newton's law in continuous time, then a
    zero-order hold with sampling time Ts (the exponential of the augmented
    matrix [[Ac, Bc], [0, 0]] Ts)."""
    from scipy.linalg import expm
    T = 2.0 * np.eye(M) - np.eye(M, k=1) - np.eye(M, k=-1)   # wall-to-wall coupling
    Bu = np.zeros((M, M - 1))
    for j in range(M - 1):
        Bu[j, j] = -1.0
        Bu[j + 1, j] = 1.0
    Ac = np.block([[np.zeros((M, M)), np.eye(M)], [-ks / mass * T, -bd / mass * T]])
    Bc = np.vstack([np.zeros((M, M - 1)), Bu / mass])
    n, m = 2 * M, M - 1
    aug = np.zeros((n + m, n + m))
    aug[:n, :n] = Ac
    aug[:n, n:] = Bc
    E = expm(aug * Ts)
    return E[:n, :n].copy(), E[:n, n:].copy()


def markov_tree(N: int, p0=(0.5, 0.5), Pc=((0.1, 0.9), (0.9, 0.1))):
    """Scenario tree of a two-mode Markov chain: every node has one child per
    mode; the root's children take the initial distribution p0, later
    children the transition probabilities Pc[mode of the parent]; child k of
    a node is mode k.  Returns (tree, mode of every node; -1 at the root)."""
    nm = len(p0)
    t = uniform_tree([nm] * N)
    mode = np.full(t.V, -1, dtype=np.int64)
    prob = np.zeros(t.V)
    prob[0] = 1.0
    for i in range(t.Vnl):
        for k, j in enumerate(range(t.child_ptr[i], t.child_ptr[i + 1])):
            mode[j] = k
            prob[j] = prob[i] * (p0[k] if i == 0 else Pc[mode[i]][k])
    return dataclasses.replace(t, prob=prob), mode


def spring_mass_problem(x0: np.ndarray | None = None, *, N: int = 11, M: int = 5,
                        umax: float = 2.0, vmax: float = 5.0, pmax: float = 2.0,
                        c_mode=(0.0, 0.1), seed: int = 1005, x0_pos: float = 1.0,
                        x0_vel: float = 1.0, name: str = "spring") -> Problem:
    """The stochastic optimal control problem of Sec. IV-A: M = 5 masses of
    5 kg, ks = 1 N/m, bd = 0.1 Ns/m, Ts = 0.5 s, horizon N = 11, |u| <= 2 N,
    |v| <= 5 m/s, positions |p| <= pmax (not given in the paper), stage cost
    x'(5 I)x + u'(2 I)u, terminal cost x'(100 I)x, and the disturbance c of
    the two-mode Markov chain (p0 = (0.5, 0.5), transitions [[0.1, 0.9],
    [0.9, 0.1]]): every state entry is c_mode[k] in mode k.  x0 (default:
    positions U[-x0_pos, x0_pos], velocities U[-x0_vel, x0_vel], drawn from
    default_rng(seed))."""
    tree, mode = markov_tree(N)
    A1, B1 = spring_mass_dynamics(M)
    nx, nu = 2 * M, M - 1
    V, Vnl, Vl = tree.V, tree.Vnl, tree.Vl
    A = np.zeros((V, nx, nx))
    B = np.zeros((V, nx, nu))
    c = np.zeros((V, nx))
    A[1:] = A1
    B[1:] = B1
    c[1:] = np.asarray(c_mode)[mode[1:]][:, None]
    Q = np.broadcast_to(5.0 * np.eye(nx), (Vnl, nx, nx)).copy()
    R = np.broadcast_to(2.0 * np.eye(nu), (Vnl, nu, nu)).copy()
    P = np.broadcast_to(100.0 * np.eye(nx), (Vl, nx, nx)).copy()
    lim = np.concatenate([np.full(M, pmax), np.full(M, vmax)])
    xmin = np.broadcast_to(-lim, (V, nx)).copy()
    xmax = np.broadcast_to(lim, (V, nx)).copy()
    xmin[0], xmax[0] = -np.inf, np.inf
    umin = np.full((Vnl, nu), -umax)
    umax_ = np.full((Vnl, nu), umax)
    if x0 is None:
        rng = np.random.default_rng(seed)
        x0 = np.concatenate([rng.uniform(-x0_pos, x0_pos, M), rng.uniform(-x0_vel, x0_vel, M)])
    return Problem(tree=tree, nx=nx, nu=nu, A=A, B=B, c=c, Q=Q, R=R, P=P, xmin=xmin, xmax=xmax,
                   umin=umin, umax=umax_, x0=np.asarray(x0, dtype=np.float64), name=name)


def spring_mass_x0(count: int, seed: int = 1005, *, x0_pos: float = 1.0, x0_vel: float = 1.0,
                   M: int = 5) -> np.ndarray:
    """count initial states, positions U[-x0_pos, x0_pos], velocities
    U[-x0_vel, x0_vel] (the draws of the Sec. IV-A study), [count][2M]."""
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.uniform(-x0_pos, x0_pos, (count, M)),
                           rng.uniform(-x0_vel, x0_vel, (count, M))], axis=1)
