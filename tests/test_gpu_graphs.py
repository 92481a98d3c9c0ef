"""Graph capture of the iteration (needs a GPU): a solve launches exactly
max_iter iterations (full graphs of check_every iterations and one graph of
the remainder), cdcs_admm_prepare captures those graphs without touching the
state, and graph, prepared-graph and eager solves give the same bits."""
import numpy as np
import pytest

from paper_1609_06068_amd import cdcs, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    cdcs.load_library()
    return _t


@pytest.mark.parametrize("form", ["primal", "dual"])
@pytest.mark.parametrize("prob_fn", [synth.c1, synth.c3_small], ids=["dense_A", "sparse_A"])
def test_tail_graph_and_prepare(torch, form, prob_fn):
    prob = prob_fn()
    sol = cdcs.Solver(prob)
    ref = sol.new_state(form)
    ie = sol.solve(ref, form=form, tol=0.0, max_iter=23, check_every=0)
    assert ie.iters == 23
    for ce in (10, 50, 23, 1):
        st = sol.new_state(form)
        before = {k: v.clone() for k, v in st.items() if v is not None}
        sol.prepare(st, form=form, tol=0.0, max_iter=23, check_every=ce)
        torch.cuda.synchronize()
        for k, v in before.items():
            assert torch.equal(st[k], v), k  # prepare runs nothing
        info = sol.solve(st, form=form, tol=0.0, max_iter=23, check_every=ce)
        assert info.iters == 23
        for k in ("x", "y", "blk", "lam") + (("v",) if form == "dual" else ()):
            assert torch.equal(st[k], ref[k]), (ce, k)
        assert np.array_equal(sol.history(23), sol.history(23))
    sol.close()


def test_prepare_argument_errors(torch):
    sol = cdcs.Solver(synth.c1())
    st = sol.new_state("primal")
    with pytest.raises(cdcs.CdcsError) as e:
        sol.prepare(st, max_iter=0)
    assert e.value.status == cdcs.E_ARG
    with pytest.raises(cdcs.CdcsError):
        sol.prepare(st, form="dual")  # no v buffer
    sol.prepare(st, check_every=0)  # eager: nothing to capture
    sol.close()
