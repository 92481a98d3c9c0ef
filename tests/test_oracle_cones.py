"""Pins of the oracle's vector cones (free, nonnegative orthant, second-order
cone beside the PSD cliques) against what the mathematics fixes: the Moreau
decomposition and a generic constrained minimiser for the projections, a
linear-programming solver (scipy's HiGHS) for LPs, a closed-form SOCP, and the
optimality conditions of mixed-cone instances for Algorithms 1 and 2."""
import numpy as np
import pytest
from scipy.optimize import linprog, minimize

from oracle import oracle as O
from paper_1609_06068_amd import synth


def _in_soc(v, tol=1e-12):
    return v[0] >= np.linalg.norm(v[1:]) - tol


@pytest.mark.parametrize("q", [2, 3, 7, 40])
def test_soc_projection_moreau(q):
    """v = P(v) - P(-v), P(v) and P(-v) in the (self-dual) cone and
    orthogonal: the Moreau decomposition characterises the projection."""
    rng = np.random.default_rng(q)
    for _ in range(200):
        v = rng.standard_normal(q) * rng.uniform(0.1, 10)
        v[0] *= rng.uniform(0, 3)
        a, b = O.soc_project(v), O.soc_project(-v)
        assert np.allclose(a - b, v, rtol=1e-13, atol=1e-13)
        assert _in_soc(a) and _in_soc(b)
        assert abs(a @ b) <= 1e-12 * (v @ v)


def test_soc_projection_special_cases_and_minimiser():
    v = np.array([5.0, 3.0, 4.0])            # on the boundary: itself
    assert np.array_equal(O.soc_project(v), v)
    v = np.array([-5.0, 3.0, 4.0])           # in the polar cone: 0
    assert np.array_equal(O.soc_project(v), np.zeros(3))
    v = np.array([0.0, 3.0, 4.0])            # ((0 + 5) / 2) (1, (3, 4) / 5)
    assert np.allclose(O.soc_project(v), [2.5, 1.5, 2.0], rtol=0, atol=1e-15)
    rng = np.random.default_rng(11)
    for _ in range(20):
        v = rng.standard_normal(5)
        res = minimize(lambda q: np.sum((q - v) ** 2), x0=np.concatenate([[3.0], np.zeros(4)]),
                       constraints=[{"type": "ineq", "fun": lambda q: q[0] - np.sqrt(np.sum(q[1:] ** 2) + 1e-300)}],
                       method="SLSQP", options={"ftol": 1e-14, "maxiter": 500})
        assert np.linalg.norm(res.x - O.soc_project(v)) <= 1e-5


def test_orthant_and_free_projections():
    v = np.array([-1.0, 0.0, 2.5, -0.0])
    assert np.array_equal(O.vector_cone_project(1, v), [0.0, 0.0, 2.5, 0.0])
    assert np.array_equal(O.vector_cone_project(0, v), v)


def test_gather_scatter_adjoint_with_vector_cones():
    """<sum_k H_k^T B_k, x>_w = sum_k <B_k, H_k x> over cliques (Frobenius)
    and vector cones (Euclidean)."""
    prob = synth.mixed_small()
    dec = O.Decomposition(prob)
    assert dec.ncones == prob.p + prob.ncones
    rng = np.random.default_rng(2)
    x = rng.standard_normal(prob.nU)
    blocks = []
    for B in dec.zero_blocks():
        R = rng.standard_normal(B.shape)
        blocks.append((R + R.T) / 2 if R.ndim == 2 else R)
    lhs = dec.wdot(dec.scatter(blocks), x)
    rhs = sum(float(np.sum(blocks[k] * dec.gather(x, k))) for k in range(dec.ncones))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    # every entry is covered once by a vector cone or by its cliques
    ones = dec.scatter([np.ones_like(B) for B in dec.zero_blocks()])
    assert np.array_equal(ones, dec.D)


def test_cone_validation():
    prob = synth.mixed_small()
    bad = synth.Problem(**{**prob.__dict__})
    bad.cone_vert = prob.cone_vert.copy()
    bad.cone_vert[0] = prob.clique(0)[0]     # a vertex of a clique
    with pytest.raises(O.OracleError):
        O.Decomposition(bad)
    bad2 = synth.Problem(**{**prob.__dict__})
    bad2.cone_kind = np.array([2, 1, 2, 2], np.int32)
    bad2.cone_ptr = np.array([0, 1, 17, 23, 32], np.int64)   # a one-vertex second-order cone
    with pytest.raises(O.OracleError):
        O.Decomposition(bad2)


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_lp_matches_highs(form):
    prob = synth.lp(40, 15, 3)
    o = O.Oracle(prob)
    r = o.solve(form, max_iter=40000, tol=1e-9)
    ref = linprog(prob.c, A_eq=prob.A, b_eq=prob.b, bounds=[(0, None)] * prob.nU, method="highs")
    assert ref.status == 0 and r.converged
    assert abs(r.obj_primal - ref.fun) <= 1e-6 * abs(ref.fun)
    assert np.linalg.norm(r.X_sdp - ref.x) <= 1e-4 * np.linalg.norm(ref.x)


def test_free_and_orthant_lp_matches_highs():
    """Free variables (the cone R^n, dual cone {0}) next to an orthant."""
    prob = synth.mixed_cones(0, 0, 0, 12, [(synth.CONE_FREE, 5), (synth.CONE_ORTHANT, 30)], seed=7003)
    o = O.Oracle(prob)
    ref = linprog(prob.c, A_eq=prob.A, b_eq=prob.b, bounds=[(None, None)] * 5 + [(0, None)] * 30, method="highs")
    for form in ("primal", "dual"):
        r = o.solve(form, max_iter=40000, tol=1e-9)
        assert r.converged
        assert abs(r.obj_primal - ref.fun) <= 1e-6 * max(1.0, abs(ref.fun)), form


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_socp_closed_form(form):
    a = np.array([3.0, -4.0, 12.0, 0.5])
    prob = synth.socp_norm(a)
    r = O.Oracle(prob).solve(form, max_iter=20000, tol=1e-10)
    assert r.converged
    assert abs(r.obj_primal - np.linalg.norm(a)) <= 1e-7 * np.linalg.norm(a)
    assert abs(r.obj_dual - np.linalg.norm(a)) <= 1e-7 * np.linalg.norm(a)
    # dual multiplier y = a / ||a||
    assert np.allclose(r.y_sdp, a / np.linalg.norm(a), atol=1e-6)


def test_mixed_cones_both_forms_optimal():
    prob = synth.mixed_small()
    o = O.Oracle(prob)
    rp = o.solve("primal", max_iter=8000, tol=1e-8)
    rd = o.solve("dual", max_iter=8000, tol=1e-8)
    assert rp.converged and rd.converged
    for r in (rp, rd):
        k = o.sdp_kkt_residuals(r)
        assert k["pinf"] <= 1e-7 and k["dinf"] <= 1e-6 and k["gap"] <= 1e-6, k
        assert k["xmin"] >= -1e-6 and k["zmin"] >= -1e-6, k
    assert abs(rp.obj_primal - rd.obj_primal) <= 1e-6 * max(1.0, abs(rp.obj_primal))
