"""FP64 NumPy reference of the node-wise warm-start MLP.

TEST INFRASTRUCTURE ONLY: used by the tests to check the GPU forward,
backward, loss and Adam kernels; nothing in the product imports it.

Network din -> dh -> dh -> dout, ReLU, parameters in one flat vector
[W1 (din x dh), b1, W2 (dh x dh), b2, W3 (dh x dout), b3] (row-major).
Features of node i of an instance with initial state x0 (stage t_i):
[x0, c_i / c_scale, mean(c_j, j on the path 1..i) / c_scale, one-hot(t_i)].
Adam: Kingma and Ba (2015), with bias correction.
"""
from __future__ import annotations

import numpy as np


def layout(din, dh, dout):
    o = {}
    k = 0
    for name, size in (("W1", din * dh), ("b1", dh), ("W2", dh * dh), ("b2", dh),
                       ("W3", dh * dout), ("b3", dout)):
        o[name] = (k, k + size)
        k += size
    o["n"] = k
    return o


def unpack(p, din, dh, dout):
    L = layout(din, dh, dout)
    g = lambda n: p[L[n][0]:L[n][1]]
    return (g("W1").reshape(din, dh), g("b1"), g("W2").reshape(dh, dh), g("b2"),
            g("W3").reshape(dh, dout), g("b3"))


def forward(p, X, din, dh, dout):
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, dtype=np.float64), din, dh, dout)
    X = np.asarray(X, dtype=np.float64)
    H1 = np.maximum(X @ W1 + b1, 0.0)
    H2 = np.maximum(H1 @ W2 + b2, 0.0)
    Y = H2 @ W3 + b3
    return H1, H2, Y


def backward(p, X, H1, H2, dY, din, dh, dout):
    """Gradient of a scalar loss w.r.t. the flat parameters, given dY."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, dtype=np.float64), din, dh, dout)
    X = np.asarray(X, dtype=np.float64)
    dY = np.asarray(dY, dtype=np.float64)
    gW3 = H2.T @ dY
    gb3 = dY.sum(0)
    dH2 = (dY @ W3.T) * (H2 > 0)
    gW2 = H1.T @ dH2
    gb2 = dH2.sum(0)
    dH1 = (dH2 @ W2.T) * (H1 > 0)
    gW1 = X.T @ dH1
    gb1 = dH1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def mse(Y, T, mask):
    """(loss, dY) of sum(mask (Y - T)^2) / sum(mask)."""
    Y, T, mask = (np.asarray(a, dtype=np.float64) for a in (Y, T, mask))
    cnt = mask.sum()
    d = Y - T
    return float((mask * d * d).sum() / cnt), 2.0 * mask * d / cnt


def adam(p, g, m, v, lr, b1, b2, eps, step):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features(prob, x0, c_scale):
    """Feature rows of every node, by walking each node's ancestors."""
    t = prob.tree
    nx, N = prob.nx, t.N
    din = 3 * nx + N + 1
    X = np.zeros((t.V, din))
    stage = np.repeat(np.arange(N + 1), np.diff(t.stage_ptr))
    for i in range(t.V):
        X[i, :nx] = x0
        X[i, nx:2 * nx] = prob.c[i] / c_scale if i > 0 else 0.0
        if i > 0:
            s, j = np.zeros(nx), i
            while j > 0:
                s += prob.c[j]
                j = t.anc[j]
            X[i, 2 * nx:3 * nx] = s / stage[i] / c_scale
        X[i, 3 * nx + stage[i]] = 1.0
    return X


def dual_to_rows(prob, y):
    """Dual vector -> (rows [V][nx+nu], mask) with the root state rows masked."""
    t = prob.tree
    nx, nu = prob.nx, prob.nu
    T = np.zeros((t.V, nx + nu))
    M = np.zeros((t.V, nx + nu))
    o = 0
    for i in range(t.V):
        w = nx + nu if i < t.Vnl else nx
        T[i, :w] = y[o:o + w]
        M[i, :w] = 1.0
        o += w
    T[0, :nx] = 0.0
    M[0, :nx] = 0.0
    return T, M
