"""The instrumented solve (needs a GPU).  cdcs_admm_solve_timed runs the
iterations of cdcs_admm_solve with eager launches and HIP events around each
kernel kind: its iterates must equal those of the graph-captured solve from
the same state bit for bit (bench.py relies on this to attribute the timed
iterations' time to kernels), and every kind is bracketed once per
iteration."""
import ctypes

import numpy as np
import pytest

from paper_1609_06068_amd import cdcs, synth

pytestmark = pytest.mark.gpu

K = 24


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    cdcs.load_library()
    return _t


def _copy(st):
    return {k: (v.clone() if v is not None else None) for k, v in st.items()}


@pytest.mark.parametrize("name,form", [("c1", "primal"), ("c1", "dual"), ("c3_small", "primal")])
def test_timed_solve_matches_graph_solve(torch, name, form):
    prob = getattr(synth, name)()
    sol = cdcs.Solver(prob)
    st0 = sol.new_state(form)
    sol.solve(st0, form=form, tol=0.0, max_iter=7, check_every=7)  # a state away from zero
    start = _copy(st0)
    ref = sol.solve(st0, form=form, tol=0.0, max_iter=K, check_every=8)
    st1 = _copy(start)
    info, times = sol.solve_timed(st1, form=form, tol=0.0, max_iter=K)
    assert info.iters == ref.iters == K
    for key in ("x", "y", "blk", "lam") + (("v",) if form == "dual" else ()):
        assert torch.equal(st1[key], st0[key]), key
    assert info.obj_primal == ref.obj_primal and info.obj_dual == ref.obj_dual
    for kind in ("project", "gemv_Au", "trmv", "gemv_ATy", "scatter"):
        ms, n = times[kind]
        assert n == K, (kind, n)
        assert ms > 0.0, kind
    # the bracketed kernels run inside the solve's wall time
    assert sum(ms for ms, _ in times.values()) <= info.loop_s * 1e3
    sol.close()


def test_timed_solve_batch(torch):
    probs = synth.c4(count=3)
    sol = cdcs.BatchSolver(probs)
    st0 = sol.new_state("primal")
    start = _copy(st0)
    sol.solve(st0, form="primal", tol=0.0, max_iter=K, check_every=12)
    st1 = _copy(start)
    info, times = sol.solve_timed(st1, form="primal", tol=0.0, max_iter=K)
    assert info.iters == K
    for key in ("x", "y", "blk", "lam"):
        assert torch.equal(st1[key], st0[key]), key
    assert times["project"][1] == times["scatter"][1] == times["gemv_Au"][1] == K
    assert times["trmv"] == (0.0, 0) and times["gemv_ATy"] == (0.0, 0)
    sol.close()


def test_timed_solve_rejects_null_outputs(torch):
    L = cdcs.load_library()
    sol = cdcs.Solver(synth.c1())
    st = sol.new_state("primal")
    cs = sol._cstate(st)
    opts = cdcs._Options(1.0, 0.0, 2, cdcs.PRIMAL, 0)
    info = cdcs._Info()
    ms = np.zeros(5)
    r = L.cdcs_admm_solve_timed(sol._h, ctypes.byref(cs), ctypes.byref(opts), ctypes.byref(info), ms.ctypes.data,
                                None, None)
    assert r == cdcs.E_ARG
    sol.close()
