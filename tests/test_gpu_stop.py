"""Stopping inside an iteration (needs a GPU).  An Alg. 1 iteration runs
scatter -> residual check -> affine step -> projection; a stop decided by the
check (convergence, or the iteration cap inside a captured graph that holds
more iterations than are left) skips the rest of the iteration, so the state
must hold the last completed iterate: a solve that ends after n iterations
equals an eager solve of exactly n iterations, bit for bit.  Dense A (C1)
and sparse A (a small uneven-clique SDP): the sparse x-update copies u into x
inside the affine step, never in the scatter."""
import numpy as np
import pytest

from paper_1609_06068_amd import cdcs, synth

pytestmark = pytest.mark.gpu

KEYS = ("x", "y", "blk", "lam", "vw")


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    cdcs.load_library()
    return _t


@pytest.mark.parametrize("name", ["c1", "c3_small"])
def test_cap_inside_a_graph(torch, name):
    sol = cdcs.Solver(getattr(synth, name)())
    assert sol.sparse_a == (name == "c3_small")
    a = sol.new_state("primal")
    sol.solve(a, form="primal", tol=0.0, max_iter=23, check_every=10)  # 3 graphs of 10: 7 iterations stopped
    b = sol.new_state("primal")
    sol.solve(b, form="primal", tol=0.0, max_iter=23, check_every=0)
    for k in KEYS:
        assert torch.equal(a[k], b[k]), k
    sol.close()


@pytest.mark.parametrize("name", ["c1", "c3_small"])
def test_converged_solve_keeps_the_last_iterate(torch, name):
    prob = getattr(synth, name)()
    sol = cdcs.Solver(prob)
    a = sol.new_state("primal")
    info = sol.solve(a, form="primal", tol=1e-3, max_iter=5000, check_every=25)
    assert info.converged and 0 < info.iters < 5000
    b = sol.new_state("primal")
    ref = sol.solve(b, form="primal", tol=0.0, max_iter=info.iters, check_every=0)
    for k in KEYS:
        assert torch.equal(a[k], b[k]), k
    assert info.obj_primal == ref.obj_primal and info.obj_dual == ref.obj_dual
    # the reported objective is that of the returned x: <C, X> = sum_e w_e c_e x_e
    x = a["x"].cpu().numpy()
    w = np.where(prob.ei == prob.ej, 1.0, 2.0)
    assert abs(float(np.sum(w * prob.c * x)) - info.obj_primal) <= 1e-9 * max(1.0, abs(info.obj_primal))
    sol.close()
