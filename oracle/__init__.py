"""ctypes wrapper of the plain CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product library never imports,
links or calls anything here, and nothing here calls the product library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, FP64)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int), ("nu", C.c_int), ("N", C.c_int), ("V", C.c_int),
                ("Vnl", C.c_int),
                ("stage_ptr", _ip), ("anc", _ip), ("child_ptr", _ip),
                ("prob", _dp), ("A", _dp), ("B", _dp), ("c", _dp),
                ("Q", _dp), ("R", _dp), ("S", _dp), ("q", _dp), ("r", _dp),
                ("P", _dp), ("p", _dp),
                ("xmin", _dp), ("xmax", _dp), ("umin", _dp), ("umax", _dp),
                ("nc", C.c_int), ("ncN", C.c_int), ("F", _dp), ("G", _dp), ("FN", _dp),
                ("zmin", _dp), ("zmax", _dp), ("wgt", _dp), ("hub", _dp)]


class _Factors(C.Structure):
    _fields_ = [("Pcal", _dp), ("K", _dp), ("Phi", _dp), ("D", _dp),
                ("sigma", _dp), ("chat", _dp), ("Theta", _dp), ("Lambda", _dp)]


class _Opts(C.Structure):
    _fields_ = [("lam", C.c_double), ("eps", C.c_double), ("eps_curv", C.c_double),
                ("mem", C.c_int), ("nu_max", C.c_int), ("max_iter", C.c_int),
                ("precondition", C.c_int), ("method", C.c_int), ("backtrack", C.c_int),
                ("div_window", C.c_int), ("bt_param", C.c_double), ("trace", _dp),
                ("trace_iters", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int), ("sweeps_affine", C.c_int), ("sweeps_hom", C.c_int),
                ("ls_trials", C.c_int), ("lbfgs_push", C.c_int), ("lbfgs_skip", C.c_int),
                ("status", C.c_int), ("res_scaled_inf", C.c_double),
                ("res_unscaled_inf", C.c_double), ("phi", C.c_double),
                ("tau_hist", C.c_int * 32), ("backtracks", C.c_int), ("lambda_final", C.c_double)]


TRACE_COLS = 40     # trace row: lambda, ||R||_inf, accepted nu, nu_max, pairs used, dphi[nu]...
TRACE_PHI = 5
METHODS = {"minfbe": 0, "nama": 1, "gpad": 2}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P, F = C.POINTER(_Problem), C.POINTER(_Factors)
        L.or_factor.argtypes = [P, F]
        L.or_factor.restype = C.c_int
        L.or_sweep.argtypes = [P, F, _dp, _dp, C.c_int, _dp, _dp]
        L.or_sweep.restype = None
        L.or_cost.argtypes = [P, _dp, _dp]
        L.or_cost.restype = C.c_double
        L.or_Hx.argtypes = [P, _dp, _dp, _dp]
        L.or_Hx.restype = None
        L.or_dual_dim.argtypes = [P]
        L.or_dual_dim.restype = C.c_int
        L.or_eval.argtypes = [P, F, _dp, C.c_double, C.c_int, _dp,
                              _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_con_dim.argtypes = [P]
        L.or_con_dim.restype = C.c_int
        L.or_apply_H.argtypes = [P, _dp, _dp, _dp]
        L.or_apply_H.restype = None
        L.or_apply_Ht.argtypes = [P, _dp, _dp]
        L.or_apply_Ht.restype = None
        L.or_eval.restype = C.c_double
        L.or_hess_neg.argtypes = [P, F, C.c_int, _dp, _dp]
        L.or_hess_neg.restype = None
        L.or_power_iteration.argtypes = [P, F, C.c_int, C.c_int, _dp]
        L.or_power_iteration.restype = C.c_double
        L.or_lbfgs_direction.argtypes = [C.c_int, C.c_int, C.POINTER(_dp),
                                         C.POINTER(_dp), _dp, _dp]
        L.or_lbfgs_direction.restype = None
        L.or_solve.argtypes = [P, F, _dp, C.POINTER(_Opts), _dp, _dp, _dp, C.POINTER(_Info)]
        L.or_solve.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_threads.restype = None
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads of the node-parallel loops (factor step and sweeps); results
    are the same for any count.  1: plain sequential loops."""
    lib().or_set_threads(int(n))


def set_mutation(k: int) -> None:
    """Plant deliberate mistake number k in the oracle (0 = none); used only by
    the tests that show each pin detects a plausible error."""
    C.c_int.in_dll(lib(), "or_mutation").value = int(k)


def _ptr(a, dtype=np.float64, ctype=_dp):
    if a is None:
        return ctype()
    assert a.dtype == dtype and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(ctype)


class Problem:
    """Holds the ctypes view of a treegen.Problem (arrays kept alive)."""

    def __init__(self, prob):
        self.src = prob
        t = prob.tree
        self.nx, self.nu, self.N, self.V, self.Vnl = prob.nx, prob.nu, t.N, t.V, t.Vnl
        self._keep = {}

        def arr(name, a, dtype=np.float64):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=dtype)
            self._keep[name] = a
            return a

        s = _Problem()
        s.nx, s.nu, s.N, s.V, s.Vnl = self.nx, self.nu, self.N, self.V, self.Vnl
        for name, a, dt, ct in [
                ("stage_ptr", t.stage_ptr, np.int32, _ip), ("anc", t.anc, np.int32, _ip),
                ("child_ptr", t.child_ptr, np.int32, _ip), ("prob", t.prob, np.float64, _dp),
                ("A", prob.A, np.float64, _dp), ("B", prob.B, np.float64, _dp),
                ("c", prob.c, np.float64, _dp), ("Q", prob.Q, np.float64, _dp),
                ("R", prob.R, np.float64, _dp), ("S", prob.S, np.float64, _dp),
                ("q", prob.q, np.float64, _dp), ("r", prob.r, np.float64, _dp),
                ("P", prob.P, np.float64, _dp), ("p", prob.p, np.float64, _dp),
                ("xmin", prob.xmin, np.float64, _dp), ("xmax", prob.xmax, np.float64, _dp),
                ("umin", prob.umin, np.float64, _dp), ("umax", prob.umax, np.float64, _dp)]:
            setattr(s, name, _ptr(arr(name, a, dt), dt, ct))
        if prob.F is not None:
            s.nc, s.ncN = prob.nc, prob.ncN
            for name in ("F", "G", "FN", "zmin", "zmax"):
                setattr(s, name, _ptr(arr(name, getattr(prob, name))))
        if prob.wgt is not None:
            s.wgt = _ptr(arr("wgt", prob.wgt))
            s.hub = _ptr(arr("hub", np.zeros(prob.m) if prob.hub is None else prob.hub))
        self.s = s
        self.m_xu = lib().or_dual_dim(C.byref(s))     # (x, u) layout of the sweeps
        self.m = lib().or_con_dim(C.byref(s))         # constraint (dual) layout
        self.x0 = np.ascontiguousarray(prob.x0, dtype=np.float64)


class Factors:
    def __init__(self, pb: Problem):
        nx, nu, V, Vnl = pb.nx, pb.nu, pb.V, pb.Vnl
        self.Pcal = np.zeros((V, nx, nx))
        self.K = np.zeros((Vnl, nu, nx))
        self.Phi = np.zeros((Vnl, nu, nx + nu))
        self.D = np.zeros((Vnl, nx + nu, nx))
        self.sigma = np.zeros((Vnl, nu))
        self.chat = np.zeros((V, nx))
        self.Theta = np.zeros((V, nu, nx))
        self.Lambda = np.zeros((V, nx, nx))
        s = _Factors()
        for name in ("Pcal", "K", "Phi", "D", "sigma", "chat", "Theta", "Lambda"):
            setattr(s, name, _ptr(getattr(self, name)))
        self.s = s


def as_problem(prob) -> Problem:
    return prob if isinstance(prob, Problem) else Problem(prob)


def factor(prob) -> tuple:
    """Factor step; returns (Problem view, Factors).  Raises on a non-PD Rt."""
    pb = as_problem(prob)
    fac = Factors(pb)
    rc = lib().or_factor(C.byref(pb.s), C.byref(fac.s))
    if rc != 0:
        raise ArithmeticError(f"oracle factor step failed ({rc})")
    return pb, fac


def sweep(pb: Problem, fac: Factors, y, homogeneous=False, x0=None):
    """Algorithm 3 (homogeneous=False) or 4 on the unscaled dual y given in the
    (x, u) layout (length m_xu; the constraint layout maps there by apply_Ht);
    returns (x, u)."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    assert y.shape == (pb.m_xu,)
    p = pb.x0 if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    x = np.zeros((pb.V, pb.nx))
    u = np.zeros((pb.Vnl, pb.nu))
    lib().or_sweep(C.byref(pb.s), C.byref(fac.s), _ptr(y), _ptr(p), int(bool(homogeneous)),
                   _ptr(x), _ptr(u))
    return x, u


def cost(pb: Problem, x, u) -> float:
    return lib().or_cost(C.byref(pb.s), _ptr(np.ascontiguousarray(x)), _ptr(np.ascontiguousarray(u)))


def Hx(pb: Problem, x, u) -> np.ndarray:
    """(x, u) in the (x, u) layout."""
    out = np.zeros(pb.m_xu)
    lib().or_Hx(C.byref(pb.s), _ptr(np.ascontiguousarray(x)), _ptr(np.ascontiguousarray(u)), _ptr(out))
    return out


def apply_H(pb: Problem, x, u) -> np.ndarray:
    """z = H(x, u) in the constraint layout (Sec. II-B)."""
    out = np.zeros(pb.m)
    lib().or_apply_H(C.byref(pb.s), _ptr(np.ascontiguousarray(x)), _ptr(np.ascontiguousarray(u)),
                     _ptr(out))
    return out


def apply_Ht(pb: Problem, y) -> np.ndarray:
    """H' y: constraint-layout dual -> (x, u) layout."""
    out = np.zeros(pb.m_xu)
    lib().or_apply_Ht(C.byref(pb.s), _ptr(np.ascontiguousarray(y, dtype=np.float64)), _ptr(out))
    return out


def evaluate(pb: Problem, fac: Factors, yb, lam: float, precondition: bool = True,
             x0=None, grad=False) -> dict:
    """x, u, Hbx, z, R, T (and grad_phi) at the scaled dual point yb; phi."""
    yb = np.ascontiguousarray(yb, dtype=np.float64)
    p = pb.x0 if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    out = {k: np.zeros(pb.m) for k in ("Hbx", "z", "R", "T")}
    out["x"] = np.zeros((pb.V, pb.nx))
    out["u"] = np.zeros((pb.Vnl, pb.nu))
    gp = np.zeros(pb.m) if grad else None
    extra = np.zeros(2)
    phi = lib().or_eval(C.byref(pb.s), C.byref(fac.s), _ptr(p), float(lam), int(bool(precondition)),
                        _ptr(yb), _ptr(out["x"]), _ptr(out["u"]), _ptr(out["Hbx"]), _ptr(out["z"]),
                        _ptr(out["R"]), _ptr(out["T"]), _ptr(gp), _ptr(extra))
    out["phi"] = phi
    out["fhat"], out["g"] = float(extra[0]), float(extra[1])
    if grad:
        out["grad_phi"] = gp
    return out


def hess_neg(pb: Problem, fac: Factors, v, precondition: bool = True) -> np.ndarray:
    """v -> -Hess(f-hat) v in the (scaled) dual variables."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(pb.m)
    lib().or_hess_neg(C.byref(pb.s), C.byref(fac.s), int(bool(precondition)), _ptr(v), _ptr(out))
    return out


def power_iteration(pb: Problem, fac: Factors, precondition: bool = True, iters: int = 100,
                    v0=None) -> float:
    if v0 is None:
        v0 = np.ones(pb.m)
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    return lib().or_power_iteration(C.byref(pb.s), C.byref(fac.s), int(bool(precondition)),
                                    int(iters), _ptr(v0))


def lbfgs_direction(S: list, Qs: list, g) -> np.ndarray:
    """Two-loop L-BFGS direction -B g for pairs listed oldest first."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    m, cnt = g.shape[0], len(S)
    S = [np.ascontiguousarray(s, dtype=np.float64) for s in S]
    Qs = [np.ascontiguousarray(q, dtype=np.float64) for q in Qs]
    sp = (_dp * max(cnt, 1))(*[s.ctypes.data_as(_dp) for s in S])
    qp = (_dp * max(cnt, 1))(*[q.ctypes.data_as(_dp) for q in Qs])
    d = np.zeros(m)
    lib().or_lbfgs_direction(m, cnt, sp, qp, _ptr(g), _ptr(d))
    return d


def solve(pb: Problem, fac: Factors, method: str, lam: float, *, eps: float = 1e-6,
          mem: int = 5, nu_max: int = 10, max_iter: int = 1000, eps_curv: float = 1e-12,
          precondition: bool = True, y0=None, x0=None, backtrack: int = 0, bt_param: float = 0.0,
          div_window: int = 50, trace_iters: int = 0) -> dict:
    """Algorithm 1 (method='minfbe'), Algorithm 2 ('nama') or GPAD ('gpad');
    backtrack 1 / 2 halves lambda by the two tests of Sec. III-B; with
    trace_iters > 0 the result holds a per-update trace (TRACE_COLS columns,
    every line-search trial evaluated)."""
    trace = np.full((max(trace_iters, 1), TRACE_COLS), np.nan)
    o = _Opts(lam=float(lam), eps=float(eps), eps_curv=float(eps_curv), mem=int(mem),
              nu_max=int(nu_max), max_iter=int(max_iter),
              precondition=int(bool(precondition)), method=METHODS[method],
              backtrack=int(backtrack), div_window=int(div_window), bt_param=float(bt_param),
              trace=_ptr(trace) if trace_iters > 0 else _dp(), trace_iters=int(trace_iters))
    y = np.zeros(pb.m) if y0 is None else np.array(y0, dtype=np.float64, copy=True)
    p = pb.x0 if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    x = np.zeros((pb.V, pb.nx))
    u = np.zeros((pb.Vnl, pb.nu))
    info = _Info()
    st = lib().or_solve(C.byref(pb.s), C.byref(fac.s), _ptr(p), C.byref(o), _ptr(y), _ptr(x),
                        _ptr(u), C.byref(info))
    return dict(status=st, y=y, x=x, u=u, iters=info.iters, sweeps_affine=info.sweeps_affine,
                sweeps_hom=info.sweeps_hom, ls_trials=info.ls_trials,
                lbfgs_push=info.lbfgs_push, lbfgs_skip=info.lbfgs_skip,
                res_scaled_inf=info.res_scaled_inf, res_unscaled_inf=info.res_unscaled_inf,
                phi=info.phi, tau_hist=list(info.tau_hist), backtracks=info.backtracks,
                lambda_final=info.lambda_final, trace=trace[:trace_iters] if trace_iters > 0 else None)
