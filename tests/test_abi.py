"""C-ABI checks that need no GPU: the library loads, exports every entry point
the header declares, and rejects malformed input on the host before any
device work (error codes of include/stotree.h)."""
import dataclasses
import os
import re
import subprocess

import numpy as np
import pytest

import treegen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def st():
    from paper_2107_01745_amd import stotree
    if not os.path.exists(stotree.LIB_PATH):
        from paper_2107_01745_amd import build
        build.build()
    stotree.lib()
    return stotree


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "stotree.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)))


def test_header_entry_points_are_exported(st):
    names = declared_functions()
    assert {"tree_factor", "dual_grad", "minfbe_solve", "nama_solve"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", st.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(st.EXPORTS) == set(names)


def test_library_has_gfx950_code(st):
    out = subprocess.run(["strings", st.LIB_PATH], capture_output=True, text=True, check=True).stdout
    assert "gfx950" in out


def _expect(st, prob, code, precondition=True):
    with pytest.raises(st.StotreeError) as ei:
        st.tree_factor(prob, precondition=precondition)
    assert ei.value.code == code, (ei.value.code, str(ei.value))
    assert st.stotree_last_error()


def base():
    return treegen.draw_problem(treegen.uniform_tree([2, 1, 1]), 3, 2, np.random.default_rng(0))


def test_rejects_bad_stage_ptr(st):
    p = base()
    sp = p.tree.stage_ptr.copy()
    sp[1] = 2
    _expect(st, dataclasses.replace(p, tree=dataclasses.replace(p.tree, stage_ptr=sp)), -2)


def test_rejects_bad_probabilities(st):
    p = base()
    pr = p.tree.prob.copy()
    pr[1] *= 1.5
    _expect(st, dataclasses.replace(p, tree=dataclasses.replace(p.tree, prob=pr)), -2)


def test_rejects_inconsistent_ancestor(st):
    p = base()
    anc = p.tree.anc.copy()
    anc[3] = 2 if anc[3] == 1 else 1
    _expect(st, dataclasses.replace(p, tree=dataclasses.replace(p.tree, anc=anc)), -2)


def test_rejects_box_lo_above_hi(st):
    p = base()
    umin = p.umin.copy()
    umin[0, 0] = 2.0
    _expect(st, dataclasses.replace(p, umin=umin), -4)


def test_rejects_nonfinite_data(st):
    p = base()
    A = p.A.copy()
    A[1, 0, 0] = np.nan
    _expect(st, dataclasses.replace(p, A=A), -5)


def test_rejects_sizes(st):
    p = treegen.draw_problem(treegen.uniform_tree([1, 1]), 200, 100, np.random.default_rng(0))
    _expect(st, p, -1)


def test_rejects_degenerate_sizes(st):
    """No inputs (nu = 0), a tree that is only its root (N = 0) and an empty
    batch are rejected with ERR_ARG before any device work."""
    _expect(st, treegen.draw_problem(treegen.uniform_tree([2, 1, 1]), 3, 0, np.random.default_rng(0)), -1)
    _expect(st, treegen.draw_problem(treegen.uniform_tree([]), 3, 2, np.random.default_rng(0)), -1)
    with pytest.raises(st.StotreeError) as ei:
        st.tree_factor_batch([])
    assert ei.value.code == -1


def test_schedule_graph_calls_reject_null_on_host(st):
    import ctypes as C
    L = st.lib()
    k = (C.c_int32 * 5)(8, 1, 16, 1, 16)
    assert L.sweep_schedule(None, k) == -1
    assert L.sweep_schedule_get(None, k) == -1
    assert L.sweep_autotune(None, 1, 3, k, None, None) == -1
    assert L.sweep_graph_launch(None, None) == -1
    out = C.c_void_p(1)
    assert L.sweep_graph_create(None, None, None, 1, 1, None, None, C.byref(out)) == -1
    assert out.value is None            # *out cleared on failure
    L.sweep_graph_free(None)            # no-op
    assert "NULL" in st.stotree_last_error()


def test_shared_handle_rejects_bad_count_on_host(st):
    with pytest.raises(st.StotreeError) as ei:
        st.tree_factor_shared(base(), 0)
    assert ei.value.code == -1 and "count" in str(ei.value)
