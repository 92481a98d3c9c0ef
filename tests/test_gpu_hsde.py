"""The homogeneous self-dual embedding solver on the gfx950 library (needs a
GPU), against the oracle (oracle.Hsde).

* iterates after 50 iterations (x, y, s, z, tau, kappa; 1e-4 relative, FP32
  cone blocks) and the per-iteration residuals, which the library evaluates
  from differences of successive iterates and the oracle from their
  definitions;
* the same on the clique-tree workload's small instance (sparse A, the
  sparse factor of I + A diag(w / E) A^T);
* graphs and eager launches give identical iterates;
* outcomes: solved (stopping point and objectives against the oracle's
  HSDE, objective against Algorithm 1's optimum and HiGHS's), primal
  infeasible and dual infeasible (certificates checked against their
  definitions) on LPs and SDPs, and the closed-form SOCP."""
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


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def _packed(dec, blocks):
    out = []
    for k, B in enumerate(blocks):
        if k < dec.p:
            ia, ib = np.tril_indices(B.shape[0])
            out.append(B[ia, ib])
        else:
            out.append(np.asarray(B))
    return np.concatenate(out)


def _np(t):
    return t.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("which", ["mixed", "c3_small"])
def test_iterates_and_residuals_at_50(torch, which):
    prob = synth.mixed_small() if which == "mixed" else synth.c3_small()
    h = O.Hsde(prob)
    ref = h.solve(max_iter=50, tol=0.0)
    sol = cdcs.Solver(prob)
    if which == "c3_small":
        assert sol.sparse_a and sol.nnz_l > 0  # the sparse factor serves the HSDE matrix too
    st = sol.new_hsde_state()
    info = sol.hsde_solve(st, tol=0.0, max_iter=50, check_every=10)
    assert info.iters == 50 and info.status == cdcs.OK
    assert _rel(_np(st["x"]) * np.sqrt(h.dec.w), ref.x * np.sqrt(h.dec.w)) <= 1e-4
    assert _rel(_np(st["y"]), ref.y) <= 1e-4
    assert _rel(_np(st["s"]), _packed(h.dec, ref.s)) <= 1e-4
    assert _rel(_np(st["z"]), _packed(h.dec, ref.z)) <= 1e-4
    tk = _np(st["tk"])
    assert abs(tk[0] - ref.tau) <= 1e-4 * max(ref.tau, 1e-3)
    assert abs(tk[1] - ref.kappa) <= 1e-4 * max(ref.kappa, 1e-3) + 1e-9
    hist = sol.hsde_history(50)
    for col, r in ((0, ref.res_pri), (1, ref.res_dual), (2, ref.gap)):
        assert np.allclose(hist[:, col], r, rtol=1e-3, atol=1e-6), (col, hist[:5, col], r[:5])
    sol.close()


def test_graphs_equal_eager(torch):
    prob = synth.mixed_small()
    sol = cdcs.Solver(prob)
    a = sol.new_hsde_state()
    b = sol.new_hsde_state()
    sol.hsde_solve(a, tol=0.0, max_iter=37, check_every=10)
    sol.hsde_solve(b, tol=0.0, max_iter=37, check_every=0)
    for k in ("x", "y", "s", "z", "tk", "vw"):
        assert torch.equal(a[k], b[k]), k
    sol.close()


@pytest.mark.parametrize("make", ["c1", "mixed"])
def test_solved_matches_algorithm_1(torch, make):
    prob = synth.c1() if make == "c1" else synth.mixed_small()
    # the optimum (Algorithm 1 to 1e-9) and the oracle's HSDE at the same tolerance
    ref = O.Oracle(prob).admm_primal(max_iter=20000, tol=1e-9)
    oh = O.Hsde(prob).solve(max_iter=20000, tol=1e-5)
    sol = cdcs.Solver(prob)
    st = sol.new_hsde_state()
    info = sol.hsde_solve(st, tol=1e-5, max_iter=20000, check_every=50)
    assert info.status == cdcs.OK and oh.status == O.HSDE_SOLVED, info
    # the same stopping point (the scaled residuals decide it; FP32 cone
    # blocks may move it by a few iterations) and the same objectives
    assert abs(info.iters - oh.iters) <= 0.05 * oh.iters + 2, (info.iters, oh.iters)
    assert abs(info.obj_primal - oh.obj_primal) <= 1e-4 * max(1.0, abs(oh.obj_primal))
    assert abs(info.obj_dual - oh.obj_dual) <= 1e-4 * max(1.0, abs(oh.obj_dual))
    # within the tolerance's reach of the optimum
    assert abs(info.obj_primal - ref.obj_primal) <= 1e-3 * max(1.0, abs(ref.obj_primal))
    # the solution the iterate encodes: consistent with the reported
    # objectives, primal feasible and in the cones to the solve's tolerance
    X, ysdp = sol.hsde_solution(st, 0)
    X, ysdp = _np(X), _np(ysdp)
    dec = O.Decomposition(prob)
    assert abs(dec.wdot(prob.c, X) - info.obj_primal) <= 1e-10 * max(1.0, abs(info.obj_primal))
    assert abs(prob.b @ ysdp - info.obj_dual) <= 1e-10 * max(1.0, abs(info.obj_dual))
    # the solved test bounds both parts of the primal residual of (X, s / tau):
    # ||A(X) - b|| and ||s_k / tau - H_k X|| (s_k / tau is in the cone, so no
    # eigenvalue of H_k X lies below minus that distance)
    A = prob.A_dense()
    bound = 1.01 * info.res_pri * (1 + np.linalg.norm(prob.b)) + 1e-9
    assert info.res_pri <= 1e-5
    assert np.linalg.norm(A @ (dec.w * X) - prob.b) <= bound
    assert min(O.cone_margin(dec, k, dec.gather(X, k)) for k in range(dec.ncones)) >= -bound
    sol.close()


def test_lp_outcomes_match_highs(torch):
    for status, seed, want in (("feasible", 3, cdcs.OK), ("infeasible", 4, cdcs.PRIMAL_INFEASIBLE),
                               ("unbounded", 5, cdcs.DUAL_INFEASIBLE)):
        prob = synth.lp(40, 15, seed, status)
        ref = linprog(prob.c, A_eq=prob.A, b_eq=prob.b, bounds=[(0, None)] * prob.nU, method="highs")
        sol = cdcs.Solver(prob)
        st = sol.new_hsde_state()
        info = sol.hsde_solve(st, tol=1e-6, max_iter=40000, check_every=100)
        assert info.status == want, (status, info)
        if want == cdcs.OK:
            assert abs(info.obj_primal - ref.fun) <= 1e-4 * abs(ref.fun)
        elif want == cdcs.PRIMAL_INFEASIBLE:
            _, y = sol.hsde_solution(st, 1)
            y = _np(y)
            assert abs(prob.b @ y - 1.0) <= 1e-9
            assert np.max(prob.A.T @ y) <= 1e-4
        else:
            X, _ = sol.hsde_solution(st, 2)
            X = _np(X)
            assert abs(prob.c @ X + 1.0) <= 1e-9
            assert np.linalg.norm(prob.A @ X) <= 1e-4 and X.min() >= -1e-4
        sol.close()


def test_sdp_certificates(torch):
    prob = synth.sdp_infeasible()
    sol = cdcs.Solver(prob)
    st = sol.new_hsde_state()
    info = sol.hsde_solve(st, tol=1e-6, max_iter=20000, check_every=50)
    assert info.status == cdcs.PRIMAL_INFEASIBLE, info
    _, y = sol.hsde_solution(st, 1)
    y = _np(y)
    assert abs(prob.b @ y - 1.0) <= 1e-9
    # A^T y is minus a sum of clique-supported PSD blocks: each clique block NSD up to rounding
    dec = O.Decomposition(prob)
    aty = prob.A.T @ y
    scale = np.abs(aty).max()
    for k in range(dec.p):
        assert np.linalg.eigvalsh(dec.gather(aty, k)).max() <= 1e-4 * scale
    sol.close()
    # the ray test reads ||(A(x), s - Hx)|| ||c||_w <= tol (-<c, x>_w); the FP32
    # cone blocks and eigensolves leave s - Hx a floor near 1e-6 of the ray's
    # size, so the test tolerance stays above that
    prob = synth.sdp_unbounded()
    sol = cdcs.Solver(prob)
    st = sol.new_hsde_state()
    info = sol.hsde_solve(st, tol=1e-5, max_iter=20000, check_every=50)
    assert info.status == cdcs.DUAL_INFEASIBLE, info
    X, _ = sol.hsde_solution(st, 2)
    X = _np(X)
    w = np.where(prob.ei == prob.ej, 1.0, 2.0)
    assert abs(np.sum(w * prob.c * X) + 1.0) <= 1e-9
    assert np.linalg.norm(prob.A @ (w * X)) <= 1e-4 * (1 + np.abs(X).max())
    for k in range(dec.p):
        assert np.linalg.eigvalsh(dec.gather(X, k)).min() >= -1e-4 * np.abs(X).max()
    sol.close()


def test_socp_closed_form(torch):
    a = np.array([3.0, -4.0, 12.0, 0.5])
    sol = cdcs.Solver(synth.socp_norm(a))
    st = sol.new_hsde_state()
    info = sol.hsde_solve(st, tol=1e-7, max_iter=20000, check_every=50)
    assert info.status == cdcs.OK
    assert abs(info.obj_primal - np.linalg.norm(a)) <= 1e-5 * np.linalg.norm(a)
    sol.close()


def test_errors(torch):
    sol = cdcs.Solver(synth.mixed_small())
    st = sol.new_hsde_state()
    st_bad = dict(st)
    st_bad["tk"] = None
    with pytest.raises(cdcs.CdcsError) as e:
        sol.hsde_solve(st_bad, tol=0.0, max_iter=5)
    assert e.value.status == cdcs.E_ARG
    with pytest.raises(cdcs.CdcsError) as e:
        sol.hsde_solution(st, 3)
    assert e.value.status == cdcs.E_ARG
    sol.close()


def test_timed_solve_same_iterates(torch):
    """The instrumented HSDE solve launches the same kernels eagerly: it ends
    on the graph-captured solve's iterates bit for bit and brackets every
    kernel kind once per iteration."""
    prob = synth.c3_small()
    sol = cdcs.Solver(prob)
    a = sol.new_hsde_state()
    b = sol.new_hsde_state()
    sol.hsde_solve(a, tol=0.0, max_iter=23, check_every=10)
    info, times = sol.hsde_solve_timed(b, tol=0.0, max_iter=23)
    assert info.iters == 23
    for k in ("x", "y", "s", "z", "tk"):
        assert torch.equal(a[k], b[k]), k
    for name, (ms, n) in times.items():
        assert n == 23 and ms > 0.0, name
    sol.close()


@pytest.mark.parametrize("which", ["sparse_cones", "large_cliques"])
def test_iterates_at_20_other_paths(torch, which):
    """HSDE iterates after 20 iterations on vector cones with CSR constraints,
    and on a mix of cliques below and above the LDS limit (the latter through
    the sign-function projection)."""
    if which == "sparse_cones":
        prob = synth.lp_sparse(3000, 120, 10, seed=7007, soc=1500, free=40)
    else:
        prob = synth.peo_chordal(p=10, smin=4, smax=200, omax=8, m=60, nnz_row=20, seed=5252)
        assert prob.clique_sizes().max() > 126
    h = O.Hsde(prob)
    ref = h.solve(max_iter=20, tol=0.0)
    sol = cdcs.Solver(prob)
    st = sol.new_hsde_state()
    info = sol.hsde_solve(st, tol=0.0, max_iter=20, check_every=10)
    assert info.iters == 20 and info.status == cdcs.OK
    sw = np.sqrt(h.dec.w)
    assert _rel(_np(st["x"]) * sw, ref.x * sw) <= 1e-4
    assert _rel(_np(st["y"]), ref.y) <= 1e-4
    assert _rel(_np(st["s"]), _packed(h.dec, ref.s)) <= 1e-4
    assert _rel(_np(st["z"]), _packed(h.dec, ref.z)) <= 1e-4
    sol.close()
