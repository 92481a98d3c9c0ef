"""Numerical edge cases of the affine step and the stopping rule (needs a GPU).

* Nearly dependent constraints.  The affine projection multiplies by the
  inverse Cholesky factors formed at setup instead of substituting.  For
  M = A diag(w/D) A^T with condition number kappa, both that and the oracle's
  substitution give y with relative error O(kappa u) (u = 2^-53; the explicit
  inverse of a triangular L is accurate to O(cond(L) u) relative to
  |L^-1||L||L^-1|, and cond(L)^2 = kappa).  The test makes kappa >= 1e8 and
  checks both against an extended-precision solve at 64 kappa u.
* A that FP32 does not represent.  The library stores w A in FP32, so it
  solves with A32 = fl32(A): a KKT solution satisfies
  |A(w x) - r2|_i <= 2^-24 sum_e |A_ie| |w_e x_e| (plus the solve's own
  error), which the test checks with 2^-23, and the converged objective stays
  within the 1e-4 bar of the oracle's on the unrounded A.
* NaN / Inf in the state: the residual check flags them and the solve
  returns CDCS_E_NUMERIC within one iteration (per instance on a batch
  handle); every kernel's loops are bounded, so nothing waits on them.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1609_06068_amd import cdcs, synth

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    cdcs.load_library()
    return _t


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def _with_A(prob, A):
    """The same SDP with constraint matrix A (b = A(X0) keeps it feasible)."""
    w = np.where(prob.ei == prob.ej, 1.0, 2.0)
    b = A @ (w * prob.meta["x0"])
    return dataclasses.replace(prob, A=A, b=b, meta=dict(prob.meta))


def _overlap_counts(prob):
    return O.Decomposition(prob).D


def _kkt_extended(prob, r1, r2):
    """Block elimination of [D A^T; A 0][x; y] = [r1; r2] in extended
    precision (numpy longdouble Cholesky), the reference for the FP64 solves."""
    ld = np.longdouble
    w = np.where(prob.ei == prob.ej, 1.0, 2.0).astype(ld)
    D = _overlap_counts(prob).astype(ld)
    A = prob.A.astype(ld)
    M = (A * (w / D)[None, :]) @ A.T
    m = M.shape[0]
    L = np.zeros_like(M)
    for j in range(m):
        s = M[j, j] - np.dot(L[j, :j], L[j, :j])
        L[j, j] = np.sqrt(s)
        L[j + 1:, j] = (M[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    t = A @ (w * r1.astype(ld) / D) - r2.astype(ld)
    z = np.zeros(m, dtype=ld)
    for i in range(m):
        z[i] = (t[i] - np.dot(L[i, :i], z[:i])) / L[i, i]
    y = np.zeros(m, dtype=ld)
    for i in range(m - 1, -1, -1):
        y[i] = (z[i] - np.dot(L[i + 1:, i], y[i + 1:])) / L[i, i]
    x = (r1.astype(ld) - A.T @ y) / D
    return x.astype(np.float64), y.astype(np.float64), M.astype(np.float64)


def test_affine_projection_with_nearly_dependent_constraints(torch):
    base = synth.c1()
    rng = np.random.default_rng(8)
    A = base.A.copy()
    R = rng.standard_normal(base.nU)
    A[-1] = np.asarray(A[-2] + 1e-4 * R, dtype=np.float32).astype(np.float64)  # FP32-exact, nearly A[-2]
    prob = _with_A(base, A)
    r1 = rng.standard_normal(prob.nU)
    r2 = rng.standard_normal(prob.m)
    x_ref, y_ref, M = _kkt_extended(prob, r1, r2)
    kappa = np.linalg.cond(M)
    assert kappa >= 1e8, kappa
    bound = 64 * kappa * U64
    sol = cdcs.Solver(prob)
    x, y = sol.affine_project(torch.as_tensor(r1, device="cuda"), torch.as_tensor(r2, device="cuda"))
    x, y = x.cpu().numpy(), y.cpu().numpy()
    xo, yo = O.KKT(prob, O.Decomposition(prob)).solve(r1, r2)
    assert _rel(yo, y_ref) <= bound  # the oracle's substitution
    assert _rel(y, y_ref) <= bound, (_rel(y, y_ref), bound)
    assert _rel(x, x_ref) <= bound, (_rel(x, x_ref), bound)
    sol.close()


def test_constraints_not_representable_in_fp32(torch):
    base = synth.c1()
    rng = np.random.default_rng(9)
    A = base.A * (1.0 + 2.0 ** -30 * rng.standard_normal(base.A.shape))
    assert np.any(np.asarray(A, dtype=np.float32).astype(np.float64) != A)
    prob = _with_A(base, A)
    w = np.where(prob.ei == prob.ej, 1.0, 2.0)
    sol = cdcs.Solver(prob)
    r1 = rng.standard_normal(prob.nU)
    x, _ = sol.affine_project(torch.as_tensor(r1, device="cuda"), torch.as_tensor(prob.b, device="cuda"))
    x = x.cpu().numpy()
    res = np.abs(A @ (w * x) - prob.b)
    bound = 2.0 ** -23 * (np.abs(A) @ np.abs(w * x)) + 1e-12 * np.linalg.norm(prob.b)
    assert np.all(res <= bound), float(np.max(res / bound))
    ref = O.Oracle(prob).admm_primal(rho=1.0, max_iter=3000, tol=1e-4)
    st = sol.new_state("primal")
    info = sol.solve(st, form="primal", rho=1.0, tol=1e-4, max_iter=3000, check_every=50)
    assert ref.converged and info.converged
    assert abs(info.obj_primal - ref.obj_primal) <= 1e-4 * max(1.0, abs(ref.obj_primal))
    assert abs(info.obj_dual - ref.obj_dual) <= 1e-4 * max(1.0, abs(ref.obj_dual))
    sol.close()


@pytest.mark.parametrize("form,buf,val", [("primal", "lam", float("nan")), ("primal", "blk", float("inf")),
                                          ("dual", "v", float("nan"))])
def test_nonfinite_state_is_reported_as_numeric(torch, form, buf, val):
    prob = synth.c1()
    sol = cdcs.Solver(prob)
    st = sol.new_state(form)
    st[buf][7] = val
    for ce in (10, 0):  # graph and eager launches
        s2 = {k: (v.clone() if v is not None else None) for k, v in st.items()}
        info = sol.solve(s2, form=form, rho=1.0, tol=1e-4, max_iter=100, check_every=ce, raise_on_numeric=False)
        assert info.status == cdcs.E_NUMERIC, info
        assert info.iters <= 2, info
        assert "NaN" in cdcs.load_library().cdcs_last_error().decode() or info.jacobi_cap_hits > 0
        with pytest.raises(cdcs.CdcsError) as ei:
            sol.solve({k: (v.clone() if v is not None else None) for k, v in st.items()}, form=form,
                      tol=1e-4, max_iter=100, check_every=ce)
        assert ei.value.status == cdcs.E_NUMERIC
    sol.close()


def test_nonfinite_instance_stops_alone_in_a_batch(torch):
    probs = [synth.block_arrow(l, d, h, m, seed=900 + i)
             for i, (l, d, h, m) in enumerate([(5, 8, 2, 25), (6, 6, 3, 30), (4, 10, 4, 20)])]
    sol = cdcs.BatchSolver(probs)
    st = sol.new_state("primal")
    off = sol.offsets[sol.clique_off[1]]
    st["lam"][int(off) + 3] = float("nan")
    info = sol.solve(st, form="primal", tol=1e-4, max_iter=3000, check_every=25, raise_on_numeric=False)
    assert info.status == cdcs.E_NUMERIC
    inst = sol.instance_info()
    assert inst[1].status == cdcs.E_NUMERIC and inst[1].iters <= 2
    assert inst[0].status == cdcs.OK and inst[2].status == cdcs.OK
    for q in (0, 2):
        ref = O.Oracle(probs[q]).admm_primal(max_iter=3000, tol=1e-4)
        assert abs(inst[q].obj_primal - ref.obj_primal) <= 1e-4 * max(1.0, abs(ref.obj_primal))
    sol.close()
