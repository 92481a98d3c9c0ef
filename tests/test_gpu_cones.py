"""Vector cones (free, orthant, second-order) beside the PSD cliques on the
gfx950 library (needs a GPU).

Algorithms 1 and 2 on a mixed-cone instance against the oracle's iterates
after 50 iterations (1e-4 relative, FP32 cone blocks) and at convergence;
linear programs against HiGHS; the closed-form SOCP; a large orthant split
into several work blocks and a long second-order cone; the chordal-extension
path with cones; and the validation errors."""
import dataclasses

import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import oracle as O
from paper_1609_06068_amd import cdcs, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    cdcs.load_library()
    return _t


def _wrel(a, b, w):
    return np.sqrt(np.sum(w * (a - b) ** 2)) / max(np.sqrt(np.sum(w * b * b)), 1e-300)


def _packed(dec, blocks):
    """Oracle blocks (clique matrices, then cone vectors) as packed slots."""
    out = []
    for k, B in enumerate(blocks):
        if k < dec.p:
            ia, ib = np.tril_indices(B.shape[0])
            out.append(B[ia, ib])
        else:
            out.append(np.asarray(B))
    return np.concatenate(out)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_mixed_cones_iterates_at_50(torch, form):
    prob = synth.mixed_small()
    o = O.Oracle(prob)
    ref = o.solve(form, rho=1.0, max_iter=50)
    sol = cdcs.Solver(prob)
    assert sol.nvcones == 4 and sol.nslots == sol.nslots_psd + 32
    st = sol.new_state(form)
    info = sol.solve(st, form=form, tol=0.0, max_iter=50, check_every=10)
    assert info.iters == 50
    w = o.dec.w
    assert _wrel(st["x"].cpu().numpy(), ref.x, w) <= 1e-4
    assert _rel(st["blk"].cpu().numpy().astype(np.float64), _packed(o.dec, ref.blocks)) <= 1e-4
    assert _rel(st["lam"].cpu().numpy().astype(np.float64), _packed(o.dec, ref.lam)) <= 1e-4
    if form == "dual":
        assert _rel(st["v"].cpu().numpy().astype(np.float64), _packed(o.dec, ref.v)) <= 1e-4
    # residual histories
    hist = sol.history(50)
    assert np.allclose(hist[:, 0], ref.eps_p, rtol=1e-3, atol=1e-7)
    assert np.allclose(hist[:, 1], ref.eps_d, rtol=1e-3, atol=1e-7)
    sol.close()


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_mixed_cones_converged_objective(torch, form):
    prob = synth.mixed_small()
    ref = O.Oracle(prob).solve("primal", max_iter=8000, tol=1e-8)
    sol = cdcs.Solver(prob)
    st = sol.new_state(form)
    info = sol.solve(st, form=form, tol=1e-5, max_iter=8000, check_every=50)
    assert info.converged
    assert abs(info.obj_primal - ref.obj_primal) <= 1e-4 * max(1.0, abs(ref.obj_primal))
    assert abs(info.obj_dual - ref.obj_primal) <= 1e-4 * max(1.0, abs(ref.obj_primal))
    sol.close()


def test_lp_matches_highs(torch):
    prob = synth.lp(300, 60, 21)
    ref = linprog(prob.c, A_eq=prob.A, b_eq=prob.b, bounds=[(0, None)] * prob.nU, method="highs")
    assert ref.status == 0
    sol = cdcs.Solver(prob)
    assert sol.p == 0 and sol.nvcones == 1
    st = sol.new_state("primal")
    info = sol.solve(st, form="primal", tol=1e-6, max_iter=40000, check_every=100)
    assert info.converged
    assert abs(info.obj_primal - ref.fun) <= 1e-4 * abs(ref.fun)
    sol.close()


def test_socp_closed_form(torch):
    a = np.array([3.0, -4.0, 12.0, 0.5])
    sol = cdcs.Solver(synth.socp_norm(a))
    for form in ("primal", "dual"):
        st = sol.new_state(form)
        info = sol.solve(st, form=form, tol=1e-6, max_iter=20000, check_every=100)
        assert info.converged
        assert abs(info.obj_primal - np.linalg.norm(a)) <= 1e-5 * np.linalg.norm(a), form
    sol.close()


def test_long_cones_several_blocks(torch):
    """An orthant of 10,000 and a second-order cone of 3,000 (several work
    blocks of at most 1024 slots each; the cone's norm from per-block partial
    sums), a free cone of 20, no cliques."""
    prob = synth.mixed_cones(0, 0, 0, 30, [(synth.CONE_ORTHANT, 10000), (synth.CONE_SOC, 3000),
                                            (synth.CONE_FREE, 20)], seed=7005)
    o = O.Oracle(prob)
    ref = o.solve("primal", max_iter=40)
    sol = cdcs.Solver(prob)
    st = sol.new_state("primal")
    sol.solve(st, form="primal", tol=0.0, max_iter=40, check_every=10)
    assert _wrel(st["x"].cpu().numpy(), ref.x, o.dec.w) <= 1e-4
    assert _rel(st["lam"].cpu().numpy().astype(np.float64), _packed(o.dec, ref.lam)) <= 1e-4
    sol.close()


def test_chordal_path_with_cones(torch):
    """Without cliques the PSD part is decomposed by the chordal extension
    (the cone vertices stay out of it); the solve matches the one with the
    generator's cliques."""
    prob = synth.mixed_small()
    nocl = dataclasses.replace(prob, clique_ptr=None, clique_vert=None)
    a = cdcs.Solver(prob)
    b = cdcs.Solver(nocl)
    assert b.p == a.p and b.nslots == a.nslots and b.nvcones == 4
    ia = a.solve(a.new_state("primal"), form="primal", tol=1e-5, max_iter=8000, check_every=50)
    ib = b.solve(b.new_state("primal"), form="primal", tol=1e-5, max_iter=8000, check_every=50)
    assert ia.converged and ib.converged
    assert abs(ia.obj_primal - ib.obj_primal) <= 1e-4 * max(1.0, abs(ia.obj_primal))
    a.close()
    b.close()


def test_cone_validation_errors(torch):
    prob = synth.mixed_small()
    bad = dataclasses.replace(prob, cone_vert=prob.cone_vert.copy())
    bad.cone_vert[0] = prob.clique(0)[0]
    with pytest.raises(cdcs.CdcsError) as e:
        cdcs.Solver(bad)
    assert e.value.status == cdcs.E_PATTERN
    bad = dataclasses.replace(prob, cone_kind=np.array([2, 1, 2, 2], np.int32),
                              cone_ptr=np.array([0, 1, 17, 23, 32], np.int64))
    with pytest.raises(cdcs.CdcsError) as e:
        cdcs.Solver(bad)
    assert e.value.status == cdcs.E_PATTERN
    bad = dataclasses.replace(prob, cone_kind=np.array([0, 1, 2, 7], np.int32))
    with pytest.raises(cdcs.CdcsError) as e:
        cdcs.Solver(bad)
    assert e.value.status == cdcs.E_ARG
    sol = cdcs.Solver(prob)
    st = sol.new_state("primal")
    ev = torch.empty(max(sol.nevals, 1), dtype=torch.float32, device="cuda")
    V = torch.empty(max(sol.nwarm, 1), dtype=torch.float32, device="cuda")
    with pytest.raises(cdcs.CdcsError) as e:
        sol.unrolled_step(st, torch.as_tensor(prob.c, device="cuda"), torch.as_tensor(prob.b, device="cuda"),
                          1.0, ev, V)
    assert e.value.status == cdcs.E_ARG
    sol.close()


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_sparse_a_with_cones_iterates_at_50(torch, form):
    """Vector cones only, CSR constraints (the sparse-A kernels and the sparse
    factor) and a second-order cone spread over several work blocks."""
    prob = synth.lp_sparse(3000, 120, 10, seed=7007, soc=1500, free=40)
    o = O.Oracle(prob)
    ref = o.solve(form, rho=1.0, max_iter=50)
    sol = cdcs.Solver(prob)
    assert sol.sparse_a
    st = sol.new_state(form)
    sol.solve(st, form=form, tol=0.0, max_iter=50, check_every=10)
    assert _wrel(st["x"].cpu().numpy(), ref.x, o.dec.w) <= 1e-4
    assert _rel(st["blk"].cpu().numpy().astype(np.float64), _packed(o.dec, ref.blocks)) <= 1e-4
    assert _rel(st["lam"].cpu().numpy().astype(np.float64), _packed(o.dec, ref.lam)) <= 1e-4
    sol.close()
