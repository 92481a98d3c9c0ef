"""Pins of the oracle's homogeneous self-dual embedding (HSDE) solver.

* the linear step ut = (I + Q)^-1 w against the explicit skew matrix Q, built
  densely in orthonormal (svec) coordinates on a tiny mixed-cone instance;
* the invariants of the iteration (u in C, v in C*, u orthogonal to v);
* solved instances against Algorithm 1, HiGHS (LPs) and a closed-form SOCP;
* infeasible and unbounded instances: the status (matching HiGHS on LPs) and
  the certificates, checked against their definitions;
* the residual identities the GPU iteration evaluates instead of extra
  passes over A (derived from the linear step), against the direct formulas.
"""
import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import oracle as O
from paper_1609_06068_amd import synth


def _tiny():
    return synth.mixed_cones(2, 2, 1, 4, [(synth.CONE_FREE, 2), (synth.CONE_ORTHANT, 3), (synth.CONE_SOC, 3)], 7010)


def _svec_maps(h):
    """Orthonormal coordinates: entries scaled by sqrt(w); a clique block by
    its lower triangle with off-diagonals scaled by sqrt(2)."""
    dec = h.dec
    sw = np.sqrt(dec.w)
    blocks = dec.zero_blocks()

    def bvec(B):
        if B.ndim == 1:
            return B.copy()
        ia, ib = np.tril_indices(B.shape[0])
        return np.where(ia == ib, 1.0, np.sqrt(2.0)) * B[ia, ib]

    def bmat(v, like):
        if like.ndim == 1:
            return v.copy()
        k = like.shape[0]
        ia, ib = np.tril_indices(k)
        val = np.where(ia == ib, 1.0, 1.0 / np.sqrt(2.0)) * v
        B = np.zeros((k, k))
        B[ia, ib] = val
        B[ib, ia] = val
        return B

    sizes = [bvec(B).shape[0] for B in blocks]
    return sw, bvec, bmat, sizes, blocks


def test_linear_step_against_dense_skew_matrix():
    h = O.Hsde(_tiny())
    dec, prob = h.dec, h.prob
    sw, bvec, bmat, sizes, blocks = _svec_maps(h)
    nU, m = dec.nU, prob.m
    ncs = sum(sizes)
    # Ahat in orthonormal coordinates: A rows and -H rows
    At = prob.A * sw[None, :]
    Hrows = []
    for k in range(dec.ncones):
        cols = []
        for e in range(nU):
            x = np.zeros(nU)
            x[e] = 1.0 / sw[e]
            cols.append(bvec(dec.gather(x, k)))
        Hrows.append(np.array(cols).T)
    Ahat = np.vstack([At, -np.vstack(Hrows)])
    chat = prob.c * sw
    bhat = np.concatenate([prob.b, np.zeros(ncs)])
    N = nU + m + ncs + 1
    Q = np.zeros((N, N))
    Q[:nU, nU:nU + m + ncs] = Ahat.T
    Q[:nU, -1] = chat
    Q[nU:nU + m + ncs, :nU] = -Ahat
    Q[nU:nU + m + ncs, -1] = bhat
    Q[-1, :nU] = -chat
    Q[-1, nU:nU + m + ncs] = -bhat
    assert np.array_equal(Q, -Q.T)
    rng = np.random.default_rng(0)
    for _ in range(5):
        w = rng.standard_normal(N)
        wx = w[:nU] / sw
        wy = w[nU:nU + m]
        wz, o = [], nU + m
        for k, B in enumerate(blocks):
            wz.append(bmat(w[o:o + sizes[k]], B))
            o += sizes[k]
        ux, uy, uz, ut = h.solve_iq(wx, wy, wz, w[-1])
        u = np.concatenate([ux * sw, uy] + [bvec(B) for B in uz] + [[ut]])
        assert np.linalg.norm((np.eye(N) + Q) @ u - w) <= 1e-11 * np.linalg.norm(w)


def test_invariants_every_iteration():
    """After each iteration u = (x, y, z, tau) lies in C, v = (s, kappa) in
    C*, and <z_k, s_k> = 0, tau kappa = 0 (Moreau decomposition)."""
    h = O.Hsde(synth.mixed_small())
    dec = h.dec
    state = h.initial()
    for _ in range(60):
        x, y, z, s, tau, kappa, _ = h.step(*state)
        assert tau >= 0 and kappa >= 0 and tau * kappa == 0.0
        for k in range(dec.ncones):
            assert O.cone_margin(dec, k, s[k]) >= -1e-12 * (1 + np.abs(s[k]).max())
            assert O.cone_margin(dec, k, z[k], dual=True) >= -1e-12 * (1 + np.abs(z[k]).max())
            assert abs(float(np.sum(z[k] * s[k]))) <= 1e-12 * (1 + np.sum(z[k] ** 2) + np.sum(s[k] ** 2))
        state = (x, y, z, s, tau, kappa)


def test_residual_identities():
    """The GPU iteration evaluates the residuals from differences of
    successive iterates: with (x, y, z, s, tau) -> (x+, y+, z+, s+, tau+) and
    the linear step's ut_tau,
      A(x+) - tau+ b                         = (y+ - y) + (ut_tau - tau+) b,
      s+_k - H_k x+                          = z+_k - z_k,
      A^T y+ - sum H^T z+ + tau+ c           = (x - x+) - sum_k H_k^T (s+_k - s_k) + (tau+ - ut_tau) c."""
    h = O.Hsde(synth.mixed_small())
    dec, prob = h.dec, h.prob
    state = h.initial()
    for it in range(30):
        x, y, z, s, tau, kappa = state
        x1, y1, z1, s1, tau1, kappa1, ut = h.step(*state)
        lhs = h.A_op(x1) - tau1 * prob.b
        rhs = (y1 - y) + (ut - tau1) * prob.b
        assert np.linalg.norm(lhs - rhs) <= 1e-10 * (1 + np.linalg.norm(lhs))
        for k in range(dec.ncones):
            assert np.allclose(s1[k] - dec.gather(x1, k), z1[k] - z[k], rtol=0, atol=1e-12)
        lhs = h.AT_op(y1) - dec.scatter(z1) + tau1 * prob.c
        rhs = (x - x1) - dec.scatter([s1[k] - s[k] for k in range(dec.ncones)]) + (tau1 - ut) * prob.c
        assert np.linalg.norm(lhs - rhs) <= 1e-10 * (1 + np.linalg.norm(lhs))
        state = (x1, y1, z1, s1, tau1, kappa1)


def test_solved_matches_algorithm_1():
    for prob in (synth.c1(), synth.mixed_small()):
        r = O.Hsde(prob).solve(max_iter=20000, tol=1e-9)
        ref = O.Oracle(prob).admm_primal(max_iter=20000, tol=1e-9)
        assert r.status == O.HSDE_SOLVED and ref.converged
        assert abs(r.obj_primal - ref.obj_primal) <= 1e-6 * max(1.0, abs(ref.obj_primal))
        assert abs(r.obj_dual - ref.obj_dual) <= 1e-6 * max(1.0, abs(ref.obj_dual))
        assert np.linalg.norm(r.X_sdp - ref.X_sdp) <= 1e-4 * np.linalg.norm(ref.X_sdp)


def test_lp_statuses_match_highs():
    cases = [("feasible", 3, O.HSDE_SOLVED, 0), ("infeasible", 4, O.HSDE_INFEASIBLE, 2),
             ("unbounded", 5, O.HSDE_UNBOUNDED, 3)]
    for status, seed, want, highs_status in cases:
        prob = synth.lp(40, 15, seed, status)
        r = O.Hsde(prob).solve(max_iter=40000, tol=1e-8)
        ref = linprog(prob.c, A_eq=prob.A, b_eq=prob.b, bounds=[(0, None)] * prob.nU, method="highs")
        assert ref.status == highs_status
        assert r.status == want, status
        if want == O.HSDE_SOLVED:
            assert abs(r.obj_primal - ref.fun) <= 1e-6 * abs(ref.fun)
        elif want == O.HSDE_INFEASIBLE:
            # Farkas: b^T y = 1 and A^T y <= 0 (no x >= 0 has A x = b)
            assert abs(prob.b @ r.cert_y - 1.0) <= 1e-12
            assert np.max(prob.A.T @ r.cert_y) <= 1e-6
        else:
            # a ray: A x = 0, x >= 0, c^T x = -1
            assert abs(prob.c @ r.cert_x + 1.0) <= 1e-12
            assert np.linalg.norm(prob.A @ r.cert_x) <= 1e-6 and r.cert_x.min() >= -1e-6


def test_socp_closed_form():
    a = np.array([3.0, -4.0, 12.0, 0.5])
    r = O.Hsde(synth.socp_norm(a)).solve(max_iter=20000, tol=1e-10)
    assert r.status == O.HSDE_SOLVED
    assert abs(r.obj_primal - np.linalg.norm(a)) <= 1e-7 * np.linalg.norm(a)


def test_sdp_certificates():
    prob = synth.sdp_infeasible()
    h = O.Hsde(prob)
    r = h.solve(max_iter=20000, tol=1e-7)
    assert r.status == O.HSDE_INFEASIBLE
    # b^T y = 1 and A^T y in -K*: -A^T y is a PSD-completable... its negative
    # is sum_k H_k^T z_k with z_k PSD, so every clique block of A^T y is NSD
    aty = h.AT_op(r.cert_y)
    assert abs(prob.b @ r.cert_y - 1.0) <= 1e-12
    scale = np.abs(aty).max()
    zsum = h.dec.scatter(r.z) / (-(prob.b @ r.y))
    assert np.linalg.norm(aty + zsum) <= 1e-6 * (1 + scale)
    prob = synth.sdp_unbounded()
    h = O.Hsde(prob)
    r = h.solve(max_iter=20000, tol=1e-7)
    assert r.status == O.HSDE_UNBOUNDED
    X = r.cert_x
    assert abs(h.dec.wdot(prob.c, X) + 1.0) <= 1e-12
    assert np.linalg.norm(h.A_op(X)) <= 1e-6 * (1 + np.abs(X).max())
    for k in range(h.dec.p):
        assert np.linalg.eigvalsh(h.dec.gather(X, k)).min() >= -1e-6
