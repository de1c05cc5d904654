"""Learned warm start driver (Python orchestration of the library's kernels).

Data: the batched NAMA solver produces the optimal (preconditioned) duals of
many draws (x0, disturbance path) on one fixed tree.  Training: the MLP's
forward, loss-gradient, backward and Adam kernels (include/stotree.h).
Use: predict a dual per instance and refine it by one solver iteration; keep
it where its residual is below that of one iteration from zero (the cold
start), then solve.
Every arithmetic step runs in the library; this module only moves buffers.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import stotree

C_SCALE = 0.1   # standard deviation of the disturbances: feature normalisation


def _dev():
    return torch.device("cuda:0")


def _primal_buffers(tf):
    """x, u device buffers of a handle, allocated once and kept with it."""
    if getattr(tf, "_xu_buf", None) is None:
        tf._xu_buf = (torch.empty(tf.x_len, dtype=torch.float64, device=_dev()),
                      torch.empty(tf.u_len, dtype=torch.float64, device=_dev()))
    return tf._xu_buf


def solve_batch(probs, lam, *, method="nama", eps=1e-6, max_iter=2000, y0=None, tf=None, mem=5, div_window=0):
    """Batched solve of a list of instances (or, with tf given, of the
    concatenated x0 tensor); returns (tf, y, infos, seconds).  Instances the
    infeasibility test stops keep status ERR_DIVERGED in their record."""
    own = tf is None
    if own:
        tf = stotree.tree_factor_batch(probs, precondition=True)
    x0 = _x0_of(probs)
    y = torch.zeros(tf.m, dtype=torch.float64, device=_dev()) if y0 is None else y0
    x, u = _primal_buffers(tf)
    fn = stotree.nama_solve if method == "nama" else stotree.minfbe_solve
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        fn(tf, x0, y, x, u, stotree.make_opts(lam=lam, eps=eps, max_iter=max_iter, mem=mem, div_window=div_window))
    except stotree.StotreeError as e:
        if e.code != -6:
            raise
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    return tf, y, stotree.solve_info_batch(tf), sec


class WarmStartMLP:
    """Node-wise MLP din -> dh -> dh -> nx+nu with parameters on the GPU."""

    def __init__(self, nx, nu, N, dh=128, seed=0):
        self.nx, self.nu, self.N, self.dh = nx, nu, N, dh
        self.din, self.dout = 3 * nx + N + 1, nx + nu
        n = stotree.warm_mlp_params(self.din, dh, self.dout)
        rng = np.random.default_rng(seed)
        p = np.zeros(n, dtype=np.float32)
        k = 0
        for fan_in, fan_out in ((self.din, dh), (dh, dh), (dh, self.dout)):
            lim = np.sqrt(6.0 / fan_in)            # He-uniform for ReLU layers
            p[k:k + fan_in * fan_out] = rng.uniform(-lim, lim, fan_in * fan_out)
            k += fan_in * fan_out + fan_out        # biases start at zero
        self.params = torch.tensor(p, device=_dev())
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step = 0
        self.y_scale = 1.0

    def features(self, tf, x0):
        X = torch.empty(tf.V, self.din, dtype=torch.float32, device=_dev())
        stotree.warm_features(tf, x0, C_SCALE, X)
        return X

    def targets(self, tf, y):
        T = torch.empty(tf.V, self.dout, dtype=torch.float32, device=_dev())
        M = torch.empty_like(T)
        stotree.warm_targets(tf, y, self.y_scale, T, M)
        return T, M

    def forward(self, X):
        rows = X.shape[0]
        H = torch.empty(rows, 2 * self.dh, dtype=torch.float32, device=_dev())
        Y = torch.empty(rows, self.dout, dtype=torch.float32, device=_dev())
        stotree.warm_mlp_forward(rows, self.din, self.dh, self.dout, self.params, X, H, Y)
        return H, Y

    def predict(self, tf, x0, y_out, chunk_rows=1 << 20):
        """Predicted dual of every instance of tf into y_out (the network runs
        over chunks of rows, so its activations stay small)."""
        X = self.features(tf, x0)
        rows = X.shape[0]
        Y = torch.empty(rows, self.dout, dtype=torch.float32, device=_dev())
        H = torch.empty(min(rows, chunk_rows), 2 * self.dh, dtype=torch.float32, device=_dev())
        for r0 in range(0, rows, chunk_rows):
            n = min(chunk_rows, rows - r0)
            stotree.warm_mlp_forward(n, self.din, self.dh, self.dout, self.params, X[r0:r0 + n], H, Y[r0:r0 + n])
        del X, H
        stotree.warm_scatter(tf, Y, self.y_scale, y_out)

    def fit(self, X, T, M, *, epochs=30, batch_rows=65536, lr=1e-3, seed=0, log=None):
        """Adam on the masked squared error over shuffled minibatches; the
        minibatch rows are gathered and the masked count formed by the
        library's kernels, and the host reads the losses once per epoch."""
        batch_rows = min(batch_rows, X.shape[0])
        rows = X.shape[0]
        work = torch.empty(stotree.warm_mlp_work_len(batch_rows, self.din, self.dh, self.dout),
                           dtype=torch.float32, device=_dev())
        H = torch.empty(batch_rows, 2 * self.dh, dtype=torch.float32, device=_dev())
        Y = torch.empty(batch_rows, self.dout, dtype=torch.float32, device=_dev())
        dY = torch.empty_like(Y)
        Xb = torch.empty(batch_rows, self.din, dtype=torch.float32, device=_dev())
        Tb = torch.empty(batch_rows, self.dout, dtype=torch.float32, device=_dev())
        Mb = torch.empty_like(Tb)
        nb = rows // batch_rows
        losses = torch.zeros(nb, 2, dtype=torch.float64, device=_dev())   # per step (sum, count)
        part = torch.zeros(512, dtype=torch.float64, device=_dev())
        bad = torch.zeros(1, dtype=torch.int32, device=_dev())
        rng = np.random.default_rng(seed)
        history = []
        for ep in range(epochs):
            order = torch.tensor(rng.permutation(rows), dtype=torch.int64, device=_dev())
            for k in range(nb):
                idx = order[k * batch_rows:(k + 1) * batch_rows]
                stotree.warm_gather(X, idx, Xb, bad)
                stotree.warm_gather(T, idx, Tb, bad)
                stotree.warm_gather(M, idx, Mb, bad)
                stotree.warm_mlp_forward(batch_rows, self.din, self.dh, self.dout, self.params, Xb, H, Y)
                # inverse count 0: the library forms 1 / (masked entries of the minibatch)
                stotree.warm_mse_grad(Y.numel(), Y, Tb, Mb, 0.0, dY, losses[k], part)
                stotree.warm_mlp_backward(batch_rows, self.din, self.dh, self.dout, self.params, Xb, H, dY,
                                          self.grad, work)
                self.step += 1
                stotree.warm_adam(self.params.numel(), self.params, self.grad, self.m, self.v, lr, 0.9, 0.999,
                                  1e-8, self.step)
            l2 = losses.cpu().numpy()        # one transfer per epoch
            if int(bad.cpu()[0]):
                raise RuntimeError("warm_gather: minibatch index out of range")
            history.append(l2[:, 0].sum() / max(l2[:, 1].sum(), 1.0))
            if log:
                log(f"epoch {ep}: masked MSE {history[-1]:.4e}")
        return history


def _x0_of(probs_or_x0):
    if isinstance(probs_or_x0, torch.Tensor):
        return probs_or_x0
    return torch.tensor(np.concatenate([p.x0 for p in probs_or_x0]), dtype=torch.float64, device=_dev())


def warm_start_duals(model, tf, probs_or_x0, lam, refine_steps=1):
    """Predicted duals refined by refine_steps solver iterations (the first
    forward-backward step sends the predicted duals of inactive constraints
    to zero), set against the same number of iterations from zero (the cold
    start): each instance keeps whichever reached the lower residual.  Both
    candidates have taken refine_steps iterations, so a solve from the kept
    one costs the same as the cold solve when the cold candidate wins.
    probs_or_x0: the instances' problems, or their concatenated x0 on the
    device.  Returns (y, keep); keep[b] says whether instance b starts from its
    prediction."""
    x0 = _x0_of(probs_or_x0)
    yc = torch.zeros(tf.m, dtype=torch.float64, device=_dev())
    yw = torch.zeros(tf.m, dtype=torch.float64, device=_dev())
    x, u = _primal_buffers(tf)
    opts = stotree.make_opts(lam=lam, eps=0.0, max_iter=refine_steps, mem=1, div_window=-1)
    stotree.nama_solve(tf, x0, yc, x, u, opts)
    rc = [i["res_scaled_inf"] for i in stotree.solve_info_batch(tf)]
    model.predict(tf, x0, yw)
    stotree.nama_solve(tf, x0, yw, x, u, opts)
    rw = [i["res_scaled_inf"] for i in stotree.solve_info_batch(tf)]
    keep = [a <= b for a, b in zip(rw, rc)]
    stotree.dual_merge(tf, yw, yc, keep)
    return yw, keep


def gpad_start(tf, probs_or_x0, lam, steps=5):
    """The warm start of the paper: steps accelerated-gradient updates from
    zero (GPAD); returns the last point."""
    x0 = _x0_of(probs_or_x0)
    y = torch.zeros(tf.m, dtype=torch.float64, device=_dev())
    x, u = _primal_buffers(tf)
    stotree.gpad_solve(tf, x0, y, x, u, stotree.make_opts(lam=lam, eps=0.0, max_iter=steps, div_window=-1))
    return y
