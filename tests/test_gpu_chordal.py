"""SDPs whose pattern is not chordal and comes without cliques (needs a GPU).

cdcs_setup with cliques = NULL extends the pattern to a chordal one and takes
its maximal cliques (paper Sec. II-A); by Grone's and Agler's theorems
(Sec. II-C) the decomposed problem has the optimum of the undecomposed SDP.
The oracle solves the undecomposed problem (one clique holding every vertex,
zero data off the pattern) and the library's converged objectives must match
it within 1e-4 relative; the library's x on the fill entries completes X to a
matrix whose clique blocks are positive semidefinite."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1609_06068_amd import cdcs, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    cdcs.load_library()
    return _t


@pytest.mark.parametrize("form", ["primal", "dual"])
@pytest.mark.parametrize("seed", [1, 2])
def test_nonchordal_pattern_reaches_the_undecomposed_optimum(torch, seed, form):
    prob = synth.random_sparse(n=24, extra=18, m=12, seed=seed)
    full = synth.with_cliques(prob, [np.arange(prob.n, dtype=np.int32)])
    ref = O.Oracle(full).solve(form, max_iter=20000, tol=1e-6)
    assert ref.converged
    fi, fj, cptr, cvert = cdcs.chordal_extension(prob.n, prob.ei, prob.ej)
    assert fi.shape[0] > 0
    sol = cdcs.Solver(prob)
    assert sol.nnz == prob.nU + fi.shape[0] and sol.p == cptr.shape[0] - 1
    st = sol.new_state(form)
    # FP32 clique blocks floor the relative residuals near 1e-6: solve to 1e-5
    info = sol.solve(st, form=form, tol=1e-5, max_iter=20000, check_every=50)
    assert info.converged
    for got, want in ((info.obj_primal, ref.obj_primal), (info.obj_dual, ref.obj_dual)):
        assert abs(got - want) <= 1e-4 * max(1.0, abs(want)), (got, want)
    # X on pattern + fill: every clique block positive semidefinite
    x = st["x"].cpu().numpy()
    X = np.asarray(-1.0 * x if form == "dual" else x)  # Alg. 2 keeps X = -rho x
    ei = np.concatenate([prob.ei, fi])
    ej = np.concatenate([prob.ej, fj])
    full_X = np.zeros((prob.n, prob.n))
    full_X[ei, ej] = X
    full_X[ej, ei] = X
    for k in range(cptr.shape[0] - 1):
        cl = cvert[cptr[k]:cptr[k + 1]]
        B = full_X[np.ix_(cl, cl)]
        assert np.linalg.eigvalsh(B).min() >= -1e-4 * max(1.0, np.linalg.norm(B))
    sol.close()


def test_chordal_pattern_without_cliques(torch):
    prob = synth.c1()
    bare = dataclasses.replace(prob, clique_ptr=None, clique_vert=None)
    a, b = cdcs.Solver(prob), cdcs.Solver(bare)
    assert b.nnz == prob.nU and b.p == prob.p
    ia = a.solve(a.new_state("primal"), tol=1e-5, max_iter=5000)
    ib = b.solve(b.new_state("primal"), tol=1e-5, max_iter=5000)
    assert ia.converged and ib.converged
    assert abs(ia.obj_primal - ib.obj_primal) <= 1e-6 * max(1.0, abs(ia.obj_primal))
    a.close()
    b.close()
