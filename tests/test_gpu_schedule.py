"""Sweep schedules, the autotuner and the HIP-graph sweep through the C ABI.

The chain order only re-maps work, so it must give bit-identical sweeps; the
lane-group width (a group may split the rows of a narrow product over its two
halves), the trunk cap and the trunk mode reorder sums (equal to rounding).  The tuned schedule and every graph replay are checked against the
CPU oracle and against eager sweeps."""
import numpy as np
import pytest

import oracle
import treegen
from gpu_cases import TOL_GRAD, case, row_scale

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


def mixed_forest():
    """Widths nx+nu from 6 to 142: every lane-group width and both column
    chunkings, ragged chain counts."""
    probs = [case(n) for n in ("tiny", "odd_ragged", "mid_width", "warm_blocks", "capped", "wide",
                               "single_path", "no_chain")]
    probs += treegen.draw_batch_instances(5, seed=91, scale=0.04, N_range=(5, 9))
    return probs


def _sweep(st, tf, x0, y, homogeneous, nrhs=1):
    import torch
    x = torch.full((nrhs * tf.x_len,), np.nan, dtype=torch.float64, device="cuda:0")
    u = torch.full((nrhs * tf.u_len,), np.nan, dtype=torch.float64, device="cuda:0")
    st.dual_grad(tf, x0, y, homogeneous, x, u, nrhs=nrhs)
    torch.cuda.synchronize()
    return x.cpu().numpy(), u.cpu().numpy()


def _check_oracle(tf, probs, y, xh, uh, homogeneous, x0):
    for b, p in enumerate(probs):
        d = tf.instances[b]
        yb = y[d["y_off"]:d["y_off"] + d["m"]]
        x0b = x0[d["x0_off"]:d["x0_off"] + d["nx"]]
        xb = xh[d["x_off"]:d["x_off"] + d["V"] * d["nx"]].reshape(d["V"], d["nx"])
        ub = uh[d["u_off"]:d["u_off"] + d["Vnl"] * d["nu"]].reshape(d["Vnl"], d["nu"])
        pb, fac = oracle.factor(p)
        xo, uo = oracle.sweep(pb, fac, row_scale(p) * yb, homogeneous=homogeneous, x0=x0b)
        s = max(1.0, np.abs(xo).max())
        assert np.abs(xb - xo).max() / s < TOL_GRAD, b
        assert np.abs(ub - uo).max() / s < TOL_GRAD, b


def test_schedules_are_bit_identical(st):
    probs = mixed_forest()
    tf = st.tree_factor_batch(probs, precondition=True)
    rng = np.random.default_rng(5)
    y = _t(rng.standard_normal(2 * tf.m))
    x0 = _t(rng.standard_normal(2 * tf.x0_len))
    assert st.sweep_schedule_get(tf) == (8, 1, 16, 0, 16)
    ref = {nrhs: _sweep(st, tf, x0, y, False, nrhs) for nrhs in (1, 2)}
    _check_oracle(tf, probs, y.cpu().numpy()[:tf.m], ref[1][0], ref[1][1], False, x0.cpu().numpy()[:tf.x0_len])
    for g in (8, 16, 32, 64):
        for order in (0, 1):
            st.sweep_schedule(tf, (g, order, 16, 0, 16))
            for nrhs in (1, 2):
                xh, uh = _sweep(st, tf, x0, y, False, nrhs)
                if g == 8:      # the default width: the chain order alone changes no bit
                    assert np.array_equal(xh, ref[nrhs][0]) and np.array_equal(uh, ref[nrhs][1]), (order, nrhs)
                else:           # wider groups may split rows over two half-groups: equal to rounding
                    s = np.abs(ref[nrhs][0]).max()
                    assert np.abs(xh - ref[nrhs][0]).max() <= 1e-12 * s, (g, order, nrhs)
                    assert np.abs(uh - ref[nrhs][1]).max() <= 1e-12 * s, (g, order, nrhs)
    for cap in (1, 2, 4, 8, 16):
        for fused in (0, 1, 2, 3, 4):
            st.sweep_schedule(tf, (8, 1, cap, fused, 16))
            for nrhs in (1, 2):
                xh, uh = _sweep(st, tf, x0, y, False, nrhs)
                s = np.abs(ref[nrhs][0]).max()
                assert np.abs(xh - ref[nrhs][0]).max() <= 1e-12 * s, (cap, fused, nrhs)
                assert np.abs(uh - ref[nrhs][1]).max() <= 1e-12 * s, (cap, fused, nrhs)
    # the one-launch and fused trunks leave their counters at zero: repeated
    # sweeps agree bitwise (a counter left behind would start the next sweep's
    # waits early or never)
    for fused in (1, 3, 4):
        st.sweep_schedule(tf, (8, 1, 16, fused, 16))
        a1 = _sweep(st, tf, x0, y, False, 1)
        for _ in range(3):
            a2 = _sweep(st, tf, x0, y, False, 1)
            assert np.array_equal(a1[0], a2[0]) and np.array_equal(a1[1], a2[1]), fused
        assert np.isfinite(a1[0]).all() and np.isfinite(a1[1]).all()
    with pytest.raises(st.StotreeError):
        st.sweep_schedule(tf, (12, 1, 16, 1, 16))
    with pytest.raises(st.StotreeError):
        st.sweep_schedule(tf, (8, 1, 16, 5, 16))
    with pytest.raises(st.StotreeError):
        st.sweep_schedule(tf, (8, 1, 16, 0, -1))
    with pytest.raises(ValueError):
        st.sweep_schedule(tf, (8, 1, 16, 0))
    tf.free()


def test_autotune_keeps_results_and_caches(st, tmp_path):
    probs = mixed_forest()
    tf = st.tree_factor_batch(probs, precondition=True)
    rng = np.random.default_rng(6)
    y_np = rng.standard_normal(tf.m)
    y, x0 = _t(y_np), _t(np.concatenate([p.x0 for p in probs]))
    cache = str(tmp_path / "tune.json")
    rec = st.sweep_autotune(tf, nrhs=1, reps=3, cache=cache)
    assert not rec["cached"] and rec["ms"] > 0
    g, order, cap, fused, pmin = rec["knobs"]
    assert g in (8, 16, 32, 64) and order in (0, 1) and cap in (1, 2, 4, 8, 16) and fused in (0, 1, 2, 3, 4)
    assert pmin == 16        # not a shared handle: the panel knob is left as it is
    assert st.sweep_schedule_get(tf) == tuple(rec["knobs"])
    for homogeneous in (False, True):
        xh, uh = _sweep(st, tf, x0, y, homogeneous)
        _check_oracle(tf, probs, y_np, xh, uh, homogeneous, x0.cpu().numpy())
    st.sweep_schedule(tf, (64, 0, 1, 0, 16))
    rec2 = st.sweep_autotune(tf, nrhs=1, cache=cache)
    assert rec2["cached"] and st.sweep_schedule_get(tf) == tuple(rec["knobs"])
    tf.free()


@pytest.mark.parametrize("nrhs,trunk", [(1, 0), (2, 0), (1, 3), (2, 4)])
def test_graph_replays_match_eager(st, nrhs, trunk):
    """Replays of one recorded sweep, with eager work and synchronisation
    between them, each against an eager sweep of the same inputs (trunk
    modes 3 and 4: the fused launches' counters reset within each replay)."""
    import torch
    probs = mixed_forest()
    tf = st.tree_factor_batch(probs, precondition=True)
    st.sweep_schedule(tf, (8, 1, 16, trunk, 16))
    rng = np.random.default_rng(7)
    y = _t(rng.standard_normal(nrhs * tf.m))
    x0 = _t(rng.standard_normal(nrhs * tf.x0_len))
    x = torch.zeros(nrhs * tf.x_len, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(nrhs * tf.u_len, dtype=torch.float64, device="cuda:0")
    g = st.SweepGraph(tf, x0, y, False, x, u, nrhs=nrhs)
    for rep in range(4):
        y.copy_(_t(rng.standard_normal(nrhs * tf.m)))      # new inputs at the bound address
        x.fill_(np.nan)
        u.fill_(np.nan)
        g.launch()
        torch.cuda.synchronize()
        xe, ue = _sweep(st, tf, x0, y, False, nrhs)
        assert np.array_equal(x.cpu().numpy(), xe) and np.array_equal(u.cpu().numpy(), ue), rep
        if rep == 0:
            _check_oracle(tf, probs, y.cpu().numpy()[:tf.m], xe[:tf.x_len], ue[:tf.u_len], False,
                          x0.cpu().numpy()[:tf.x0_len])
    st.sweep_schedule(tf, (16, 1, 16, 1, 16))
    with pytest.raises(st.StotreeError):
        g.launch()                         # schedule changed: must be recorded again
    g.free()
    tf.free()
