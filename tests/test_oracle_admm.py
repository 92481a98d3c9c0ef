"""Pins for the oracle's decomposition, KKT solve and Algorithms 1 and 2.

Nothing here compares the oracle with itself: the decomposition and KKT solve
are checked against the literal vec / Kronecker form of Sec. III-A solved by a
dense library solve; the algorithms against closed-form optima (Rayleigh
quotient, lambda_max, block-diagonal sums), Grone/Agler equivalence, primal/
dual agreement, the original SDP's optimality conditions and invariants that
follow from the projection (Moreau decomposition)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1609_06068_amd import synth


def _E(n, cl):
    E = np.zeros((len(cl), n))
    E[np.arange(len(cl)), cl] = 1.0
    return E


def _vec_setup(prob):
    """Literal vec-form objects: vec(X) column stacking, H_k = E_k (x) E_k."""
    n = prob.n
    Hs = [np.kron(_E(n, prob.clique(k)), _E(n, prob.clique(k))) for k in range(prob.p)]
    Dvec = sum(H.T @ H for H in Hs)
    Avec = np.zeros((prob.m, n * n))
    cvec = np.zeros(n * n)
    A = prob.A_dense()
    for e, (i, j) in enumerate(zip(prob.ei, prob.ej)):
        for (r, s) in {(i, j), (j, i)}:
            Avec[:, s * n + r] = A[:, e]   # vec stacks columns: (r, s) -> s*n + r
            cvec[s * n + r] = prob.c[e]
    return Hs, Dvec, Avec, cvec


def _pos(n, i, j):
    return j * n + i


def test_decomposition_matches_kronecker_form():
    prob = synth.small_chordal(n=14, p=5, smax=5, m=3, seed=11)
    dec = O.Decomposition(prob)
    Hs, Dvec, _, _ = _vec_setup(prob)
    n = prob.n
    d = np.diag(Dvec)
    for e, (i, j) in enumerate(zip(prob.ei, prob.ej)):
        assert d[_pos(n, i, j)] == dec.D[e] == d[_pos(n, j, i)]
    # D is diagonal (rows of H_k orthonormal), zero off the pattern
    assert np.count_nonzero(Dvec - np.diag(d)) == 0
    rng = np.random.default_rng(0)
    x = rng.standard_normal(prob.nU)
    X = np.zeros((n, n))
    X[prob.ei, prob.ej] = x
    X[prob.ej, prob.ei] = x
    xv = X.reshape(-1, order="F")
    blocks = []
    for k in range(prob.p):
        s = len(prob.clique(k))
        assert np.array_equal(dec.gather(x, k), (Hs[k] @ xv).reshape(s, s, order="F"))
        R = rng.standard_normal((s, s))
        blocks.append(R + R.T)
    sv = sum(Hs[k].T @ blocks[k].reshape(-1, order="F") for k in range(prob.p))
    got = dec.scatter(blocks)
    for e, (i, j) in enumerate(zip(prob.ei, prob.ej)):
        assert np.isclose(got[e], sv[_pos(n, i, j)], rtol=1e-14, atol=1e-14)
    # D^{-1} sum_k H_k^T H_k x = x
    back = dec.scatter([dec.gather(x, k) for k in range(prob.p)]) / dec.D
    assert np.allclose(back, x, rtol=1e-14)
    # weighted inner product equals the vec inner product
    y = rng.standard_normal(prob.nU)
    Y = np.zeros((n, n))
    Y[prob.ei, prob.ej] = y
    Y[prob.ej, prob.ei] = y
    assert np.isclose(dec.wdot(x, y), np.sum(X * Y), rtol=1e-13)


@pytest.mark.parametrize("seed", [1, 2])
def test_kkt_solve_matches_dense_vec_kkt(seed):
    prob = synth.small_chordal(n=12, p=4, smax=5, m=4, seed=seed)
    dec = O.Decomposition(prob)
    kkt = O.KKT(prob, dec)
    Hs, Dvec, Avec, _ = _vec_setup(prob)
    n = prob.n
    on = np.flatnonzero(np.diag(Dvec) > 0)   # vec positions on the pattern
    N = on.shape[0]
    K = np.zeros((N + prob.m, N + prob.m))
    K[:N, :N] = Dvec[np.ix_(on, on)]
    K[:N, N:] = Avec[:, on].T
    K[N:, :N] = Avec[:, on]
    rng = np.random.default_rng(seed)
    r1 = rng.standard_normal(prob.nU)
    r2 = rng.standard_normal(prob.m)
    R1 = np.zeros((n, n))
    R1[prob.ei, prob.ej] = r1
    R1[prob.ej, prob.ei] = r1
    rhs = np.concatenate([R1.reshape(-1, order="F")[on], r2])
    sol = np.linalg.solve(K, rhs)
    xv = np.zeros(n * n)
    xv[on] = sol[:N]
    x, y = kkt.solve(r1, r2)
    for e, (i, j) in enumerate(zip(prob.ei, prob.ej)):
        assert np.isclose(x[e], xv[_pos(n, i, j)], rtol=1e-10, atol=1e-10)
        assert np.isclose(x[e], xv[_pos(n, j, i)], rtol=1e-10, atol=1e-10)
    assert np.allclose(y, sol[N:], rtol=1e-10, atol=1e-10)


def test_one_primal_iteration_matches_vec_form():
    """One step of Alg. 1 written with explicit H_k and a dense KKT solve."""
    prob = synth.small_chordal(n=12, p=4, smax=5, m=3, seed=21)
    o = O.Oracle(prob)
    Hs, Dvec, Avec, cvec = _vec_setup(prob)
    n = prob.n
    rho = 0.7
    rng = np.random.default_rng(3)
    xk, lam = [], []
    for k in range(prob.p):
        s = len(prob.clique(k))
        R = rng.standard_normal((s, s))
        xk.append(R @ R.T)
        G = rng.standard_normal((s, s))
        lam.append(G + G.T)
    # literal vec form
    on = np.flatnonzero(np.diag(Dvec) > 0)
    N = on.shape[0]
    rhs1 = sum(Hs[k].T @ (xk[k] + lam[k] / rho).reshape(-1, order="F") for k in range(prob.p)) - cvec / rho
    K = np.zeros((N + prob.m, N + prob.m))
    K[:N, :N] = Dvec[np.ix_(on, on)]
    K[:N, N:] = Avec[:, on].T
    K[N:, :N] = Avec[:, on]
    sol = np.linalg.solve(K, np.concatenate([rhs1[on], prob.b]))
    xv = np.zeros(n * n)
    xv[on] = sol[:N]
    ref_xk, ref_lam = [], []
    for k in range(prob.p):
        s = len(prob.clique(k))
        Hx = (Hs[k] @ xv).reshape(s, s, order="F")
        lam_, Q = np.linalg.eigh(Hx - lam[k] / rho)
        Pk = (Q * np.maximum(lam_, 0)) @ Q.T
        ref_xk.append(Pk)
        ref_lam.append(lam[k] + rho * (Pk - Hx))
    res = o.admm_primal(rho=rho, max_iter=1, xk=xk, lam=lam)
    for k in range(prob.p):
        assert np.allclose(res.blocks[k], ref_xk[k], atol=1e-10)
        assert np.allclose(res.lam[k], ref_lam[k], atol=1e-10)


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_trace_constraint_gives_lambda_min(form):
    prob = synth.trace_problem(4, 3, 2, seed=7)
    o = O.Oracle(prob)
    res = o.solve(form, max_iter=20000, tol=1e-9)
    Cf = np.zeros((prob.n, prob.n))
    Cf[prob.ei, prob.ej] = prob.c
    Cf[prob.ej, prob.ei] = prob.c
    lmin = np.linalg.eigvalsh(Cf).min()
    assert res.converged
    assert abs(res.obj_primal - lmin) <= 1e-6 * max(1, abs(lmin))
    assert abs(res.obj_dual - lmin) <= 1e-6 * max(1, abs(lmin))


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_lambda_max_closed_form(form):
    """min t s.t. t I - M PSD has optimum lambda_max(M)."""
    prob = synth.lambda_max_problem(6, seed=3)
    o = O.Oracle(prob)
    res = o.solve(form, max_iter=20000, tol=1e-10)
    lmax = np.linalg.eigvalsh(prob.meta["M"]).max()
    assert res.converged
    assert abs(-res.obj_dual - lmax) <= 1e-7 * max(1, abs(lmax))


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_block_diagonal_sum_of_lambda_min(form):
    prob = synth.block_trace_problem(l=5, d=4, seed=2)
    o = O.Oracle(prob)
    res = o.solve(form, max_iter=20000, tol=1e-9)
    C = prob.meta["C"]
    d = prob.meta["d"]
    ref = sum(np.linalg.eigvalsh(C[i * d:(i + 1) * d, i * d:(i + 1) * d]).min() for i in range(prob.meta["l"]))
    assert res.converged
    assert abs(res.obj_primal - ref) <= 1e-6 * max(1, abs(ref))


def test_grone_agler_decomposed_equals_undecomposed():
    prob = synth.block_arrow(l=4, d=4, h=2, m=6, seed=3)
    full = synth.with_cliques(prob, [np.arange(prob.n, dtype=np.int32)])
    r1 = O.Oracle(prob).solve("primal", max_iter=20000, tol=1e-8)
    r2 = O.Oracle(full).solve("primal", max_iter=20000, tol=1e-8)
    assert r1.converged and r2.converged
    assert abs(r1.obj_primal - r2.obj_primal) <= 1e-6 * max(1, abs(r2.obj_primal))


def test_primal_and_dual_algorithms_agree_and_satisfy_sdp_kkt():
    prob = synth.c1()
    o = O.Oracle(prob)
    rp = o.solve("primal", max_iter=3000, tol=1e-7)
    rd = o.solve("dual", max_iter=3000, tol=1e-7)
    assert rp.converged and rd.converged
    scale = max(1.0, abs(rp.obj_primal))
    assert abs(rp.obj_primal - rd.obj_dual) <= 1e-5 * scale
    assert abs(rp.obj_dual - rd.obj_primal) <= 1e-5 * scale
    for r in (rp, rd):
        kk = o.sdp_kkt_residuals(r)
        assert kk["pinf"] < 1e-6 and kk["dinf"] < 1e-6 and kk["gap"] < 1e-5
        assert kk["xmin"] > -1e-5 and kk["zmin"] > -1e-5


def test_primal_invariants_every_iteration():
    """lam_k = rho P+(-W) and x_k = P+(W) (Moreau): both PSD and orthogonal."""
    prob = synth.small_chordal(n=20, p=6, smax=6, m=5, seed=5)
    o = O.Oracle(prob)

    def cb(it, x, y, xk, lam):
        for X, L in zip(xk, lam):
            assert np.linalg.eigvalsh(X).min() > -1e-10
            assert np.linalg.eigvalsh(L).min() > -1e-10
            assert abs(np.sum(X * L)) < 1e-9 * (1 + np.linalg.norm(X) * np.linalg.norm(L))

    o.admm_primal(rho=1.3, max_iter=30, callback=cb)


def test_dual_multiplier_shortcut_sign():
    """With the Y-block first, lam_k = -rho H_k x (the printed +rho is a sign slip)."""
    prob = synth.small_chordal(n=20, p=6, smax=6, m=5, seed=6)
    o = O.Oracle(prob)
    rho = 0.8
    seen = []

    def cb(it, x, y, z, lam):
        for k, L in enumerate(lam):
            Hx = o.dec.gather(x, k)
            assert np.allclose(L, -rho * Hx, atol=1e-10)
            seen.append(np.linalg.norm(L + rho * Hx) < np.linalg.norm(L - rho * Hx) + 1e-12)

    o.admm_dual(rho=rho, max_iter=20, callback=cb)
    assert all(seen)


def test_iteration_cap_reports_not_converged():
    res = O.Oracle(synth.c1()).solve("primal", max_iter=1, tol=1e-12)
    assert res.iters == 1 and not res.converged


def test_rank_deficient_A_is_rejected():
    prob = synth.block_arrow(l=3, d=3, h=2, m=4, seed=1)
    prob.A = prob.A.copy()
    prob.A[3] = prob.A[2]
    with pytest.raises(O.OracleError) as e:
        O.Oracle(prob)
    assert e.value.status == O.E_RANK


def test_bad_patterns_are_rejected():
    prob = synth.block_arrow(l=3, d=3, h=2, m=4, seed=1)
    bad = synth.Problem(**{**prob.__dict__})
    bad.clique_vert = prob.clique_vert.copy()
    bad.clique_vert[0], bad.clique_vert[1] = bad.clique_vert[1], bad.clique_vert[0]
    with pytest.raises(O.OracleError):
        O.Decomposition(bad)
    bad2 = synth.Problem(**{**prob.__dict__})
    bad2.clique_ptr = prob.clique_ptr[:-1].copy()   # drop the last clique: entries uncovered
    with pytest.raises(O.OracleError):
        O.Decomposition(bad2)
