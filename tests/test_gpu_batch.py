"""Many independent SDPs in one handle (needs a GPU): per-instance parity with
the oracle, per-instance stopping, and agreement with single-SDP handles."""
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


def _small_batch():
    shapes = [(10, 10, 5, 50), (5, 8, 2, 25), (7, 12, 6, 35), (3, 4, 3, 9), (12, 6, 4, 60), (6, 20, 9, 30)]
    return [synth.block_arrow(l, d, h, m, seed=700 + i) for i, (l, d, h, m) in enumerate(shapes)]


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def _split(sol, st, q, probs):
    e0, e1 = sol.entry_off[q], sol.entry_off[q + 1]
    k0, k1 = sol.clique_off[q], sol.clique_off[q + 1]
    x = st["x"].cpu().numpy()[e0:e1]
    off = sol.offsets
    blk = st["blk"].cpu().numpy()[off[k0]:off[k1]].astype(np.float64)
    lam = st["lam"].cpu().numpy()[off[k0]:off[k1]].astype(np.float64)
    return x, blk, lam


def test_batch_iterates_after_50_iterations(torch):
    probs = _small_batch()
    sol = cdcs.BatchSolver(probs)
    st = sol.new_state("primal")
    info = sol.solve(st, form="primal", tol=0.0, max_iter=50, check_every=10)
    assert info.iters == 50 and info.jacobi_cap_hits == 0
    for q, prob in enumerate(probs):
        ref = O.Oracle(prob).admm_primal(max_iter=50)
        x, blk, lam = _split(sol, st, q, probs)
        assert _rel(x, ref.x) <= 1e-4, q
        assert _rel(blk, cdcs.pack_blocks(ref.blocks)) <= 1e-4, q
        assert _rel(lam, cdcs.pack_blocks(ref.lam)) <= 1e-4, q
    sol.close()


def test_batch_per_instance_stopping(torch):
    probs = _small_batch()
    sol = cdcs.BatchSolver(probs)
    st = sol.new_state("primal")
    info = sol.solve(st, form="primal", tol=1e-4, max_iter=3000, check_every=25)
    assert info.converged
    inst = sol.instance_info()
    for q, prob in enumerate(probs):
        ref = O.Oracle(prob).admm_primal(max_iter=3000, tol=1e-4)
        assert ref.converged and inst[q].status == cdcs.OK
        assert abs(inst[q].iters - ref.iters) <= max(3, ref.iters // 50), (q, inst[q].iters, ref.iters)
        assert abs(inst[q].obj_primal - ref.obj_primal) <= 1e-4 * max(1.0, abs(ref.obj_primal))
        assert abs(inst[q].obj_dual - ref.obj_dual) <= 1e-4 * max(1.0, abs(ref.obj_dual))
        assert max(inst[q].eps_p, inst[q].eps_d) <= 1e-4
        assert inst[q].time_to_tol_s > 0
        # the state of an instance that stopped early is frozen at its own stop
        x, _, _ = _split(sol, st, q, probs)
        assert abs(float(np.sum(np.where(prob.ei == prob.ej, 1.0, 2.0) * prob.c * x)) - inst[q].obj_primal) <= 1e-9 * max(
            1.0, abs(inst[q].obj_primal))
    order = np.argsort([i.iters for i in inst])
    times = np.array([inst[q].time_to_tol_s for q in order])
    assert np.all(np.diff(times) >= -1e-6)  # later stops, later stamps
    sol.close()


def test_batch_matches_single_handles(torch):
    probs = _small_batch()[:3]
    sol = cdcs.BatchSolver(probs)
    st = sol.new_state("primal")
    sol.solve(st, form="primal", tol=0.0, max_iter=30, check_every=0)
    for q, prob in enumerate(probs):
        one = cdcs.Solver(prob)
        s1 = one.new_state("primal")
        one.solve(s1, form="primal", tol=0.0, max_iter=30, check_every=0)
        x, blk, lam = _split(sol, st, q, probs)
        assert _rel(x, s1["x"].cpu().numpy()) <= 1e-5
        assert _rel(lam, s1["lam"].cpu().numpy().astype(np.float64)) <= 1e-5
        one.close()
    sol.close()


def test_batch_affine_projection(torch):
    probs = _small_batch()
    sol = cdcs.BatchSolver(probs)
    rng = np.random.default_rng(3)
    r1 = rng.standard_normal(sol.nnz)
    r2 = rng.standard_normal(sol.m)
    x, y = sol.affine_project(torch.as_tensor(r1, device="cuda"), torch.as_tensor(r2, device="cuda"))
    x, y = x.cpu().numpy(), y.cpu().numpy()
    for q, prob in enumerate(probs):
        e0, e1 = sol.entry_off[q], sol.entry_off[q + 1]
        r0, r1_ = sol.row_off[q], sol.row_off[q + 1]
        xr, yr = O.Oracle(prob).kkt.solve(r1[e0:e1], r2[r0:r1_])
        assert _rel(x[e0:e1], xr) <= 1e-10 and _rel(y[r0:r1_], yr) <= 1e-10
    sol.close()


def test_batch_errors(torch):
    probs = _small_batch()[:2]
    sol = cdcs.BatchSolver(probs)
    st = sol.new_state("primal")  # no v buffer
    with pytest.raises(cdcs.CdcsError) as e:
        sol.solve(st, form="dual", tol=0.0, max_iter=2)
    assert e.value.status == cdcs.E_ARG
    sol.close()
    bad = synth.Problem(**{**probs[1].__dict__})
    bad.A = probs[1].A.copy()
    bad.A[1] = bad.A[0]
    with pytest.raises(cdcs.CdcsError) as e:
        cdcs.BatchSolver([probs[0], bad])
    assert e.value.status == cdcs.E_RANK and "problem 1" in str(e.value)


def test_many_sdp_workload_subset(torch):
    """64 instances of the many-SDP workload in one handle; every instance
    converges, and sampled instances match the oracle's objective."""
    probs = synth.c4(count=64)
    sol = cdcs.BatchSolver(probs)
    st = sol.new_state("primal")
    info = sol.solve(st, form="primal", tol=1e-4, max_iter=2000, check_every=50)
    inst = sol.instance_info()
    assert info.jacobi_cap_hits == 0
    assert all(i.status == cdcs.OK for i in inst)
    for q in (0, 17, 63):
        ref = O.Oracle(probs[q]).admm_primal(max_iter=2000, tol=1e-4)
        assert abs(inst[q].obj_primal - ref.obj_primal) <= 1e-4 * max(1.0, abs(ref.obj_primal))
    sol.close()


def _split_v(sol, st, q):
    k0, k1 = sol.clique_off[q], sol.clique_off[q + 1]
    off = sol.offsets
    return st["v"].cpu().numpy()[off[k0]:off[k1]].astype(np.float64)


def test_batch_dual_iterates_after_50_iterations(torch):
    """Algorithm 2 on a batch handle: per-instance parity with the oracle."""
    probs = _small_batch()
    sol = cdcs.BatchSolver(probs)
    st = sol.new_state("dual")
    info = sol.solve(st, form="dual", tol=0.0, max_iter=50, check_every=10)
    assert info.iters == 50 and info.jacobi_cap_hits == 0
    for q, prob in enumerate(probs):
        ref = O.Oracle(prob).admm_dual(max_iter=50)
        x, blk, lam = _split(sol, st, q, probs)
        assert _rel(x, ref.x) <= 1e-4, q
        assert _rel(blk, cdcs.pack_blocks(ref.blocks)) <= 1e-4, q
        assert _rel(lam, cdcs.pack_blocks(ref.lam)) <= 1e-4, q
        assert _rel(_split_v(sol, st, q), cdcs.pack_blocks(ref.v)) <= 1e-4, q
    sol.close()


def test_batch_dual_per_instance_stopping(torch):
    probs = _small_batch()
    sol = cdcs.BatchSolver(probs)
    st = sol.new_state("dual")
    info = sol.solve(st, form="dual", tol=1e-4, max_iter=3000, check_every=25)
    assert info.converged
    inst = sol.instance_info()
    for q, prob in enumerate(probs):
        ref = O.Oracle(prob).admm_dual(max_iter=3000, tol=1e-4)
        assert ref.converged and inst[q].status == cdcs.OK
        assert abs(inst[q].iters - ref.iters) <= max(3, ref.iters // 50), (q, inst[q].iters, ref.iters)
        assert abs(inst[q].obj_primal - ref.obj_primal) <= 1e-4 * max(1.0, abs(ref.obj_primal))
        assert abs(inst[q].obj_dual - ref.obj_dual) <= 1e-4 * max(1.0, abs(ref.obj_dual))
        assert max(inst[q].eps_p, inst[q].eps_d) <= 1e-4
    sol.close()


def test_batch_dual_matches_single_handles(torch):
    probs = _small_batch()[:3]
    sol = cdcs.BatchSolver(probs)
    st = sol.new_state("dual")
    sol.solve(st, form="dual", tol=0.0, max_iter=30, check_every=0)
    for q, prob in enumerate(probs):
        one = cdcs.Solver(prob)
        s1 = one.new_state("dual")
        one.solve(s1, form="dual", tol=0.0, max_iter=30, check_every=0)
        x, blk, lam = _split(sol, st, q, probs)
        assert _rel(x, s1["x"].cpu().numpy()) <= 1e-5
        assert _rel(lam, s1["lam"].cpu().numpy().astype(np.float64)) <= 1e-5
        one.close()
    sol.close()
