"""Thin Python binding of libstotree.so (argument marshalling only).

Every function has the name of the C entry point it calls (include/stotree.h).
Device buffers are torch tensors on a ROCm device; the library receives their
raw pointers and the current HIP stream.  There is no fallback: if the
compiled library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstotree.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)

OK, NOT_CONVERGED = 0, 1
ERRORS = {-1: "ERR_ARG", -2: "ERR_TREE", -3: "ERR_NOT_PD", -4: "ERR_BOX", -5: "ERR_NUMERIC",
          -6: "ERR_DIVERGED", -7: "ERR_DEVICE", -8: "ERR_OOM"}


class StotreeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class TreeDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nu", C.c_int32), ("N", C.c_int32), ("num_nodes", C.c_int32),
                ("stage_ptr", _ip), ("ancestor", _ip), ("child_ptr", _ip), ("prob", _dp)]


class ProblemData(C.Structure):
    _fields_ = ([(n, _dp) for n in ("A", "B", "c", "Q", "R", "S", "q", "r", "P", "p",
                                    "xmin", "xmax", "umin", "umax")] +
                [("nc", C.c_int32), ("ncN", C.c_int32)] +
                [(n, _dp) for n in ("F", "G", "FN", "zmin", "zmax", "wgt", "hub")])


class SolverOpts(C.Structure):
    _fields_ = [("lam", C.c_double), ("eps", C.c_double), ("eps_curv", C.c_double),
                ("mem", C.c_int32), ("nu_max", C.c_int32), ("max_iter", C.c_int32),
                ("check_every", C.c_int32), ("backtrack", C.c_int32), ("div_window", C.c_int32),
                ("bt_param", C.c_double), ("trace", C.c_void_p), ("trace_iters", C.c_int32),
                ("reserved", C.c_int32)]


class SolverInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("sweeps_affine", C.c_int32), ("sweeps_hom", C.c_int32),
                ("ls_trials", C.c_int32), ("lbfgs_push", C.c_int32), ("lbfgs_skip", C.c_int32),
                ("status", C.c_int32), ("res_scaled_inf", C.c_double),
                ("res_unscaled_inf", C.c_double), ("lam", C.c_double), ("seconds", C.c_double),
                ("backtracks", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


TRACE_COLS = 40   # solver trace row: lambda, ||R||_inf, accepted nu, nu_max, pairs, dphi[nu]...
TRACE_PHI = 5


EXPORTS = ("tree_factor", "tree_factor_batch", "tree_factors_free", "tree_dims",
           "tree_instance_dims", "dual_grad", "dual_lipschitz", "minfbe_solve", "nama_solve",
           "solve_info_batch", "stotree_timing", "stotree_timing_read", "stotree_last_error",
           "warm_mlp_params", "warm_mlp_work_len", "warm_mlp_forward", "warm_mlp_backward",
           "warm_mse_grad", "warm_adam", "warm_features", "warm_scatter", "warm_targets",
           "dual_select", "tree_factor_shared", "sweep_schedule", "sweep_schedule_get", "sweep_autotune",
           "sweep_graph_create", "sweep_graph_launch", "sweep_graph_free", "dual_grad_noalloc",
           "gpad_solve", "dual_merge", "warm_gather")
PHASES = ("bwd_chain", "bwd_stages", "fwd_stages", "fwd_chain")

_lib = None


def lib():
    """Load the compiled library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2107_01745_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.tree_factor.argtypes = [C.POINTER(TreeDesc), C.POINTER(ProblemData), C.c_int, vp,
                                  C.POINTER(vp)]
        L.tree_factor.restype = C.c_int
        L.tree_factor_batch.argtypes = [C.c_int, C.POINTER(TreeDesc), C.POINTER(ProblemData), C.c_int,
                                        vp, C.POINTER(vp)]
        L.tree_factor_batch.restype = C.c_int
        L.tree_factor_shared.argtypes = [C.POINTER(TreeDesc), C.POINTER(ProblemData), C.c_int, C.c_int, _dp,
                                         vp, C.POINTER(vp)]
        L.tree_factor_shared.restype = C.c_int
        L.tree_instance_dims.argtypes = [vp, C.c_int, C.POINTER(C.c_int64)]
        L.tree_instance_dims.restype = C.c_int
        L.solve_info_batch.argtypes = [vp, C.POINTER(SolverInfo)]
        L.solve_info_batch.restype = C.c_int
        L.tree_factors_free.argtypes = [vp]
        L.tree_factors_free.restype = None
        L.tree_dims.argtypes = [vp, C.POINTER(C.c_int64)]
        L.tree_dims.restype = C.c_int
        for fn in (L.dual_grad, L.dual_grad_noalloc):
            fn.argtypes = [vp, vp, vp, C.c_int, C.c_int, vp, vp, vp]
            fn.restype = C.c_int
        L.dual_lipschitz.argtypes = [vp, C.c_int, _dp, vp]
        L.dual_lipschitz.restype = C.c_int
        for fn in (L.minfbe_solve, L.nama_solve, L.gpad_solve):
            fn.argtypes = [vp, vp, C.POINTER(SolverOpts), vp, vp, vp, C.POINTER(SolverInfo), vp]
            fn.restype = C.c_int
        L.stotree_timing.argtypes = [C.c_int]
        L.stotree_timing.restype = C.c_int
        L.stotree_timing_read.argtypes = [_dp, C.POINTER(C.c_int64)]
        L.stotree_timing_read.restype = C.c_int
        L.stotree_last_error.argtypes = []
        L.stotree_last_error.restype = C.c_char_p
        i32p = C.POINTER(C.c_int32)
        L.sweep_schedule.argtypes = [vp, i32p]
        L.sweep_schedule_get.argtypes = [vp, i32p]
        L.sweep_autotune.argtypes = [vp, C.c_int, C.c_int, i32p, _dp, vp]
        L.sweep_graph_create.argtypes = [vp, vp, vp, C.c_int, C.c_int, vp, vp, C.POINTER(vp)]
        L.sweep_graph_launch.argtypes = [vp, vp]
        for fn in (L.sweep_schedule, L.sweep_schedule_get, L.sweep_autotune, L.sweep_graph_create,
                   L.sweep_graph_launch):
            fn.restype = C.c_int
        L.sweep_graph_free.argtypes = [vp]
        L.sweep_graph_free.restype = None
        _lib = L
    return _lib


def stotree_last_error() -> str:
    return lib().stotree_last_error().decode()


def _check(rc):
    if rc < 0:
        raise StotreeError(rc, stotree_last_error())
    return rc


def _stream(stream):
    """The given HIP stream, else torch's current stream, else the NULL stream."""
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    if not torch.cuda.is_available():
        return C.c_void_p(None)
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    """Raw device pointer of a contiguous float64 torch tensor (or None)."""
    if t is None:
        return None
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), (t.device, t.dtype)
    return C.c_void_p(t.data_ptr())


class TreeFactors:
    """Owns the handle returned by tree_factor / tree_factor_batch.

    Totals: ninst, m (concatenated dual length), n, x_len (sum V nx), u_len
    (sum V_nl nu), x0_len (sum nx), V (total nodes).  ``instances`` lists
    the per-instance sizes and offsets; for a single tree its nx, nu, N, Vnl
    and sstar are also attributes."""

    shared = 1      # tree_factor_shared: the number of copies

    def __init__(self, handle):
        self.handle = handle
        d = tree_dims(handle)
        (self.ninst, self.precondition, self.m, self.n, self.x_len, self.u_len, self.x0_len,
         self.V, self.device_bytes, self.max_width) = [int(v) for v in d]
        self.instances = []
        for b in range(self.ninst):
            out = (C.c_int64 * 12)()
            _check(lib().tree_instance_dims(handle, b, out))
            keys = ("nx", "nu", "N", "V", "Vnl", "m", "n", "sstar", "y_off", "x_off", "u_off", "x0_off")
            self.instances.append(dict(zip(keys, [int(v) for v in out])))
        i0 = self.instances[0]
        self.nx, self.nu, self.N, self.Vnl, self.sstar = i0["nx"], i0["nu"], i0["N"], i0["Vnl"], i0["sstar"]

    def free(self):
        for ref in getattr(self, "_graphs", ()):
            g = ref()
            if g is not None:
                g.free()
        self._graphs = []
        if self.handle:
            lib().tree_factors_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _descs(prob, keep):
    t = prob.tree

    def d(a, dtype=np.float64):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dtype)
        keep.append(a)
        return a.ctypes.data_as(_ip if dtype == np.int32 else _dp)

    td = TreeDesc(nx=prob.nx, nu=prob.nu, N=t.N, num_nodes=t.V,
                  stage_ptr=d(t.stage_ptr, np.int32), ancestor=d(t.anc, np.int32),
                  child_ptr=d(t.child_ptr, np.int32), prob=d(t.prob))
    names = ("A", "B", "c", "Q", "R", "S", "q", "r", "P", "p", "xmin", "xmax", "umin", "umax",
             "F", "G", "FN", "zmin", "zmax", "wgt", "hub")
    pd = ProblemData(**{n: d(getattr(prob, n, None)) for n in names})
    if getattr(prob, "F", None) is not None:
        pd.nc, pd.ncN = int(prob.F.shape[0]), int(prob.FN.shape[0])
    return td, pd


def tree_factor(prob, precondition: bool = True, stream=None) -> TreeFactors:
    """Factor step on a treegen.Problem (host arrays)."""
    keep = []
    td, pd = _descs(prob, keep)
    h = C.c_void_p()
    _check(lib().tree_factor(C.byref(td), C.byref(pd), int(bool(precondition)), _stream(stream),
                             C.byref(h)))
    return TreeFactors(h)


def tree_factor_shared(prob, count: int, precondition: bool = True, c=None, stream=None) -> TreeFactors:
    """Factor step once for ``count`` instances sharing prob's tree and data;
    they differ in x0 (given per call) and, with ``c`` ([count][V][nx] host
    array), in the disturbances."""
    keep = []
    td, pd = _descs(prob, keep)
    cp = None
    if c is not None:
        c = np.ascontiguousarray(c, dtype=np.float64)
        assert c.shape == (count, prob.tree.V, prob.nx), c.shape
        cp = c.ctypes.data_as(_dp)
    h = C.c_void_p()
    _check(lib().tree_factor_shared(C.byref(td), C.byref(pd), int(bool(precondition)), int(count), cp,
                                    _stream(stream), C.byref(h)))
    tf = TreeFactors(h)
    tf.shared = int(count)
    return tf


def tree_factor_batch(probs, precondition: bool = True, stream=None) -> TreeFactors:
    """Factor step on a list of treegen.Problem instances (one handle)."""
    keep = []
    n = len(probs)
    tds, pds = zip(*[_descs(p, keep) for p in probs]) if n else ((), ())
    tarr = (TreeDesc * n)(*tds)
    parr = (ProblemData * n)(*pds)
    h = C.c_void_p()
    _check(lib().tree_factor_batch(n, tarr, parr, int(bool(precondition)), _stream(stream), C.byref(h)))
    return TreeFactors(h)


def tree_dims(handle) -> list:
    out = (C.c_int64 * 10)()
    _check(lib().tree_dims(handle.handle if isinstance(handle, TreeFactors) else handle, out))
    return list(out)


def solve_info_batch(tf: TreeFactors) -> list:
    infos = (SolverInfo * tf.ninst)()
    _check(lib().solve_info_batch(tf.handle, infos))
    return [i.as_dict() for i in infos]


def dual_grad(tf: TreeFactors, x0, y, homogeneous: bool, x, u, nrhs: int = 1, stream=None) -> None:
    """x(y) (Algorithm 3) or x-hat(y) (Algorithm 4) into the device tensors x, u."""
    _check(lib().dual_grad(tf.handle, _ptr(x0), _ptr(y), int(bool(homogeneous)), int(nrhs),
                           _ptr(x), _ptr(u), _stream(stream)))


def dual_grad_noalloc(tf: TreeFactors, x0, y, homogeneous: bool, x, u, nrhs: int = 1, stream=None) -> None:
    """dual_grad with the sweep workspace in the library's static device
    scratch (no device allocation in the call)."""
    _check(lib().dual_grad_noalloc(tf.handle, _ptr(x0), _ptr(y), int(bool(homogeneous)), int(nrhs),
                                   _ptr(x), _ptr(u), _stream(stream)))


def sweep_schedule(tf: TreeFactors, knobs) -> None:
    """Set (group_min, chain_order, trunk_cap, trunk_fused, panel_min) of the
    handle's sweeps."""
    if len(knobs) != 5:
        raise ValueError("sweep_schedule takes 5 knobs")
    k = (C.c_int32 * 5)(*[int(v) for v in knobs])
    _check(lib().sweep_schedule(tf.handle, k))


def sweep_schedule_get(tf: TreeFactors) -> tuple:
    k = (C.c_int32 * 5)()
    _check(lib().sweep_schedule_get(tf.handle, k))
    return tuple(int(v) for v in k)


def forest_signature(tf: TreeFactors, nrhs: int) -> str:
    """Key of the autotuning cache: the sizes of every instance, whether the
    instances are copies of one factored tree, and nrhs."""
    import hashlib
    h = hashlib.sha1()
    for d in tf.instances:
        h.update(repr((d["nx"], d["nu"], d["N"], d["V"], d["Vnl"], d["sstar"])).encode())
    return f"{tf.ninst}x{h.hexdigest()[:16]}:shared{tf.shared}:nrhs{nrhs}:k5"


def sweep_autotune(tf: TreeFactors, nrhs: int = 1, reps: int = 5, cache: str | None = None,
                   stream=None) -> dict:
    """Pick the fastest schedule for this handle (timed on the device) and
    keep it.  With ``cache`` (a JSON file), a schedule stored for the same
    forest signature is applied without timing, and a new one is stored."""
    import json
    key = forest_signature(tf, nrhs)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
        if key in table:
            sweep_schedule(tf, table[key]["knobs"])
            return dict(table[key], cached=True)
    k = (C.c_int32 * 5)()
    ms = C.c_double()
    _check(lib().sweep_autotune(tf.handle, int(nrhs), int(reps), k, C.byref(ms), _stream(stream)))
    rec = {"knobs": [int(v) for v in k], "ms": ms.value}
    if cache:
        table[key] = rec
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(rec, cached=False)


class SweepGraph:
    """A dual_grad call recorded as one HIP graph (pointers bound at creation)."""

    def __init__(self, tf: TreeFactors, x0, y, homogeneous: bool, x, u, nrhs: int = 1):
        h = C.c_void_p()
        _check(lib().sweep_graph_create(tf.handle, _ptr(x0), _ptr(y), int(bool(homogeneous)), int(nrhs),
                                        _ptr(x), _ptr(u), C.byref(h)))
        self.handle = h
        self._keep = (x0, y, x, u)   # the bound buffers must outlive the graph
        import weakref
        if not hasattr(tf, "_graphs"):
            tf._graphs = []
        tf._graphs.append(weakref.ref(self))   # freed with (before) the handle

    def launch(self, stream=None) -> None:
        _check(lib().sweep_graph_launch(self.handle, _stream(stream)))

    def free(self) -> None:
        if self.handle:
            lib().sweep_graph_free(self.handle)
            self.handle = None
            self._keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def dual_lipschitz(tf: TreeFactors, iters: int = 100, stream=None):
    """L of every instance (a float for a single tree, else a list)."""
    L = (C.c_double * tf.ninst)()
    _check(lib().dual_lipschitz(tf.handle, int(iters), L, _stream(stream)))
    return L[0] if tf.ninst == 1 else list(L)


def make_opts(lam=0.0, eps=1e-6, eps_curv=1e-12, mem=5, nu_max=10, max_iter=1000, check_every=1,
              backtrack=0, bt_param=0.0, div_window=0, trace=None, trace_iters=0):
    """solver_opts; trace: a float64 device tensor of [instances][trace_iters][TRACE_COLS]."""
    tp = None
    if trace is not None:
        tp = _ptr(trace)
        trace_iters = int(trace.shape[-2])
    return SolverOpts(lam=lam, eps=eps, eps_curv=eps_curv, mem=mem, nu_max=nu_max,
                      max_iter=max_iter, check_every=check_every, backtrack=backtrack,
                      div_window=div_window, bt_param=bt_param, trace=tp, trace_iters=trace_iters)


def _solve(fn, tf, x0, y, x, u, opts, stream):
    info = SolverInfo()
    rc = fn(tf.handle, _ptr(x0), C.byref(opts), _ptr(y), _ptr(x), _ptr(u), C.byref(info),
            _stream(stream))
    _check(rc)
    return rc, info.as_dict()


def minfbe_solve(tf, x0, y, x, u, opts=None, stream=None):
    """Algorithm 1; y holds the initial dual and receives the last iterate."""
    return _solve(lib().minfbe_solve, tf, x0, y, x, u, opts or make_opts(), stream)


def nama_solve(tf, x0, y, x, u, opts=None, stream=None):
    """Algorithm 2 (two-right-hand-side homogeneous sweep per iteration)."""
    return _solve(lib().nama_solve, tf, x0, y, x, u, opts or make_opts(), stream)


def gpad_solve(tf, x0, y, x, u, opts=None, stream=None):
    """Accelerated dual proximal gradient (one affine sweep per update); y
    receives the last point evaluated."""
    return _solve(lib().gpad_solve, tf, x0, y, x, u, opts or make_opts(), stream)


def stotree_timing(enable: bool) -> None:
    _check(lib().stotree_timing(int(bool(enable))))


def stotree_timing_read() -> dict:
    """{phase: (total_ms, launches)} accumulated since the last read."""
    ms = (C.c_double * 4)()
    cnt = (C.c_int64 * 4)()
    _check(lib().stotree_timing_read(ms, cnt))
    return {PHASES[p]: (ms[p], int(cnt[p])) for p in range(4)}


# ---------------------------- learned warm start ----------------------------
def _warm_sigs(L):
    vp, f32 = C.c_void_p, C.c_float
    L.warm_mlp_params.argtypes = [C.c_int, C.c_int, C.c_int]
    L.warm_mlp_params.restype = C.c_int64
    L.warm_mlp_work_len.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
    L.warm_mlp_work_len.restype = C.c_int64
    L.warm_mlp_forward.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp]
    L.warm_mlp_backward.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp]
    L.warm_mse_grad.argtypes = [C.c_int64, vp, vp, vp, f32, vp, vp, vp, vp]
    L.warm_adam.argtypes = [C.c_int64, vp, vp, vp, vp, f32, f32, f32, f32, C.c_int, vp]
    L.warm_gather.argtypes = [C.c_int64, C.c_int, vp, C.c_int64, vp, vp, vp, vp]
    L.warm_features.argtypes = [vp, vp, f32, vp, vp]
    L.warm_scatter.argtypes = [vp, vp, f32, vp, vp]
    L.warm_targets.argtypes = [vp, vp, f32, vp, vp, vp]
    L.dual_select.argtypes = [vp, vp, C.POINTER(C.c_int32), vp]
    L.dual_merge.argtypes = [vp, vp, vp, C.POINTER(C.c_int32), vp]
    for fn in (L.warm_mlp_forward, L.warm_mlp_backward, L.warm_mse_grad, L.warm_adam, L.warm_features,
               L.warm_scatter, L.warm_targets, L.dual_select, L.dual_merge, L.warm_gather):
        fn.restype = C.c_int


def _wl():
    L = lib()
    if not getattr(L, "_warm_ready", False):
        _warm_sigs(L)
        L._warm_ready = True
    return L


def _fptr(t):
    """Raw device pointer of a contiguous tensor of any dtype."""
    assert t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def warm_mlp_params(din, dh, dout) -> int:
    return int(_wl().warm_mlp_params(din, dh, dout))


def warm_mlp_work_len(rows, din, dh, dout) -> int:
    return int(_wl().warm_mlp_work_len(rows, din, dh, dout))


def warm_mlp_forward(rows, din, dh, dout, params, X, H, Y, stream=None):
    _check(_wl().warm_mlp_forward(rows, din, dh, dout, _fptr(params), _fptr(X), _fptr(H), _fptr(Y),
                                  _stream(stream)))


def warm_mlp_backward(rows, din, dh, dout, params, X, H, dY, grad, work, stream=None):
    _check(_wl().warm_mlp_backward(rows, din, dh, dout, _fptr(params), _fptr(X), _fptr(H), _fptr(dY),
                                   _fptr(grad), _fptr(work), _stream(stream)))


def warm_mse_grad(n, Y, T, mask, inv_count, dY, loss2, part, stream=None):
    _check(_wl().warm_mse_grad(n, _fptr(Y), _fptr(T), _fptr(mask), float(inv_count), _fptr(dY),
                               _fptr(loss2), _fptr(part), _stream(stream)))


def warm_gather(src, idx, dst, bad, stream=None):
    """dst[r] = src[idx[r]] for the rows of float32 matrices (idx int64, bad a
    one-element int32 device flag set on an out-of-range index)."""
    import torch
    assert src.dtype == torch.float32 and dst.dtype == torch.float32 and idx.dtype == torch.int64
    assert bad.dtype == torch.int32 and src.dim() == 2 and dst.dim() == 2 and src.shape[1] == dst.shape[1]
    assert idx.numel() == dst.shape[0]
    _check(_wl().warm_gather(dst.shape[0], dst.shape[1], _fptr(src), src.shape[0], _fptr(idx), _fptr(dst),
                             _fptr(bad), _stream(stream)))


def warm_adam(n, params, grad, m, v, lr, beta1, beta2, eps, step, stream=None):
    _check(_wl().warm_adam(n, _fptr(params), _fptr(grad), _fptr(m), _fptr(v), float(lr), float(beta1),
                           float(beta2), float(eps), int(step), _stream(stream)))


def warm_features(tf, x0, c_scale, X, stream=None):
    _check(_wl().warm_features(tf.handle, _fptr(x0), float(c_scale), _fptr(X), _stream(stream)))


def warm_scatter(tf, Y, y_scale, y, stream=None):
    _check(_wl().warm_scatter(tf.handle, _fptr(Y), float(y_scale), _fptr(y), _stream(stream)))


def warm_targets(tf, y, y_scale, T, mask, stream=None):
    _check(_wl().warm_targets(tf.handle, _fptr(y), float(y_scale), _fptr(T), _fptr(mask), _stream(stream)))


def dual_select(tf, y, keep, stream=None):
    keep = (C.c_int32 * tf.ninst)(*[int(bool(k)) for k in keep])
    _check(_wl().dual_select(tf.handle, _fptr(y), keep, _stream(stream)))


def dual_merge(tf, y, y_other, keep, stream=None):
    """Rows of instances with keep[b] false copied from y_other into y."""
    keep = (C.c_int32 * tf.ninst)(*[int(bool(k)) for k in keep])
    _check(_wl().dual_merge(tf.handle, _fptr(y), _fptr(y_other), keep, _stream(stream)))
