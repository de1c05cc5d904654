"""The allocation-free dual gradient (dual_grad_noalloc) through the C ABI:
its results equal dual_grad's on the same handle and inputs (the same
kernels, only the sweep workspace differs), on two calls in a row whose
second is smaller, also after the static scratch was filled by a larger
call; a call whose workspace exceeds the static scratch is refused."""
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


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _both(st, tf, x0, y, homogeneous, nrhs):
    """(dual_grad, dual_grad_noalloc) results for the same inputs."""
    import torch
    out = []
    for fn in (st.dual_grad, st.dual_grad_noalloc):
        x = torch.full((nrhs, tf.V, tf.nx), np.nan, dtype=torch.float64, device="cuda:0")
        u = torch.full((nrhs, tf.Vnl, tf.nu), np.nan, dtype=torch.float64, device="cuda:0")
        fn(tf, None if homogeneous else x0, y, homogeneous, x, u, nrhs=nrhs)
        torch.cuda.synchronize()
        out.append((x.cpu().numpy(), u.cpu().numpy()))
    return out


@pytest.mark.parametrize("trunk", [0, 4])
def test_noalloc_equals_dual_grad_on_two_calls(st, trunk):
    """trunk 4: the first stages above s* in one launch per direction, whose
    child-side products pass through the caller's x and u outputs."""
    rng = np.random.default_rng(23)
    big = treegen.draw_problem(treegen.uniform_tree([4, 4, 4, 1, 1, 1]), 20, 10, rng)
    small = case("tiny")
    print(f"noalloc (trunk mode {trunk}): big tree nrhs 2, then tiny tree nrhs 1", flush=True)
    for prob, nrhs in ((big, 2), (small, 1)):
        tf = st.tree_factor(prob, precondition=True)
        st.sweep_schedule(tf, (8, 1, 16, trunk, 16))
        x0 = _dev(np.tile(prob.x0, nrhs))
        pb, fac = oracle.factor(prob)
        sc = row_scale(prob, True)
        for homogeneous in (False, True):
            ybar = rng.standard_normal((nrhs, tf.m))
            (xa, ua), (xb, ub) = _both(st, tf, x0, _dev(ybar), homogeneous, nrhs)
            assert np.isfinite(xb).all() and np.isfinite(ub).all()
            scale = max(1.0, np.abs(xa).max(), np.abs(ua).max())
            assert np.abs(xb - xa).max() <= 1e-12 * scale
            assert np.abs(ub - ua).max() <= 1e-12 * scale
            for k in range(nrhs):      # and the oracle, at the dual-gradient tolerance
                xo, uo = oracle.sweep(pb, fac, sc * ybar[k], homogeneous=homogeneous)
                assert np.abs(xb[k] - xo).max() <= TOL_GRAD * max(1.0, np.abs(xo).max())
                assert np.abs(ub[k] - uo).max() <= TOL_GRAD * max(1.0, np.abs(uo).max())
        tf.free()


def test_noalloc_refuses_workspace_beyond_scratch(st):
    import torch
    # 64 right-hand sides on matrix-core panels need 64 x (sum V nx + sum V_nl nu)
    # doubles: 64 x 324,240 x 8 bytes = 166 MB > 128 MiB
    prob = treegen.draw_problem(treegen.uniform_tree([4, 4, 4, 4, 4, 1, 1, 1]), 50, 30,
                                np.random.default_rng(5))
    tf = st.tree_factor(prob, precondition=True)
    need = 64 * (tf.x_len + tf.u_len) * 8
    assert need > 128 * 2**20, need
    y = torch.zeros(64, tf.m, dtype=torch.float64, device="cuda:0")
    x = torch.zeros(64, tf.V, tf.nx, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(64, tf.Vnl, tf.nu, dtype=torch.float64, device="cuda:0")
    with pytest.raises(st.StotreeError) as ei:
        st.dual_grad_noalloc(tf, None, y, True, x, u, nrhs=64)
    assert ei.value.code == -1 and "static scratch" in str(ei.value)
    tf.free()
