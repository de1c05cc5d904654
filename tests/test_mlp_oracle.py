"""Pins of the FP64 MLP oracle (no GPU): backward vs central finite
differences of the loss, Adam's first step vs its closed form, the feature
rows vs hand-computed values on a tiny tree, and the dual <-> rows map."""
import numpy as np

import oracle.mlp as om
import treegen


def _net(seed=0, din=7, dh=9, dout=4):
    rng = np.random.default_rng(seed)
    n = om.layout(din, dh, dout)["n"]
    return rng.standard_normal(n) * 0.5, din, dh, dout, rng


def test_backward_matches_finite_differences():
    p, din, dh, dout, rng = _net()
    X = rng.standard_normal((13, din))
    T = rng.standard_normal((13, dout))
    M = (rng.random((13, dout)) > 0.3).astype(float)

    def loss(pp):
        return om.mse(om.forward(pp, X, din, dh, dout)[2], T, M)[0]

    H1, H2, Y = om.forward(p, X, din, dh, dout)
    _, dY = om.mse(Y, T, M)
    g = om.backward(p, X, H1, H2, dY, din, dh, dout)
    h = 1e-6
    for k in rng.choice(p.size, 40, replace=False):
        e = np.zeros_like(p)
        e[k] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_mse_gradient_is_exact_derivative():
    rng = np.random.default_rng(1)
    Y, T = rng.standard_normal((5, 3)), rng.standard_normal((5, 3))
    M = np.ones((5, 3))
    M[0, 0] = 0
    l, dY = om.mse(Y, T, M)
    assert abs(l - ((Y - T) ** 2 * M).sum() / M.sum()) < 1e-15
    assert dY[0, 0] == 0.0


def test_adam_first_step_closed_form():
    """At step 1 the bias-corrected moments are g and g^2: the update is
    lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = om.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 0.01, 0.9, 0.999, 1e-8, 1)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_on_tiny_tree():
    rng = np.random.default_rng(2)
    prob = treegen.draw_problem(treegen.uniform_tree([2, 1]), 2, 1, rng)
    x0 = np.array([0.5, -1.0])
    X = om.features(prob, x0, 0.1)
    # node 3 is the child of node 1 (stage 2): path 1 -> 3
    assert np.allclose(X[3, :2], x0)
    assert np.allclose(X[3, 2:4], prob.c[3] / 0.1)
    assert np.allclose(X[3, 4:6], (prob.c[1] + prob.c[3]) / 2 / 0.1)
    assert np.array_equal(X[3, 6:], [0, 0, 1])
    assert np.array_equal(X[0, 2:6], np.zeros(4)) and X[0, 6] == 1


def test_dual_rows_map():
    rng = np.random.default_rng(3)
    prob = treegen.draw_problem(treegen.uniform_tree([2, 1]), 2, 1, rng)
    y = np.arange(prob.m, dtype=float) + 1
    T, M = om.dual_to_rows(prob, y)
    assert M[0, :2].sum() == 0 and M[0, 2] == 1 and T[0, 2] == 3
    assert M[3].tolist() == [1, 1, 0] and T[3, :2].tolist() == [3 * 3 + 1 + 0, 3 * 3 + 2]
