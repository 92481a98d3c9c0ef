"""Launch plans of the batched projection (needs a GPU): the persistent queue
launch over all cliques and the per-bucket launches, at every workgroup size,
against the oracle on the uneven-clique instance, and the queue's ticket
counter across eager, graph and instrumentation launches."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1609_06068_amd import cdcs, synth

pytestmark = pytest.mark.gpu

PLANS = [(True, 256), (True, 512), (False, 64), (False, 256), (False, 512)]


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    cdcs.load_library()
    return _t


@pytest.fixture(scope="module")
def small():
    prob = synth.c3_small()
    return prob, O.Oracle(prob).solve("primal", rho=1.0, max_iter=30)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def _lam(sol, st):
    return np.concatenate([B.ravel() for B in cdcs.unpack_blocks(st["lam"].cpu().numpy().astype(np.float64),
                                                                 sol.sizes, sol.offsets)])


@pytest.mark.parametrize("plan", PLANS, ids=[f"{'queue' if q else 'buckets'}{t}" for q, t in PLANS])
def test_every_plan_matches_the_oracle(torch, small, plan):
    prob, ref = small
    sol = cdcs.Solver(prob)
    sol.set_projection_plan(*plan)
    tun = sol.tuning()
    assert tun["persistent"] == plan[0]
    st = sol.new_state("primal")
    info = sol.solve(st, form="primal", tol=0.0, max_iter=30, check_every=10)
    assert info.iters == 30 and info.jacobi_cap_hits == 0
    assert _rel(st["x"].cpu().numpy(), ref.x) <= 1e-4
    assert _rel(_lam(sol, st), np.concatenate([B.ravel() for B in ref.lam])) <= 1e-4
    sol.close()


def test_queue_tickets_stay_aligned_across_launch_kinds(torch, small):
    """The queue launch relies on every launch drawing exactly p + grid
    tickets.  Interleave eager iterations, graph replays and instrumentation
    launches; a fresh solve afterwards must equal a fresh solve before."""
    prob, _ = small
    sol = cdcs.Solver(prob)
    sol.set_projection_plan(True, 256)
    a = sol.new_state("primal")
    sol.solve(a, form="primal", tol=0.0, max_iter=12, check_every=4)
    junk = sol.new_state("primal")
    sol.solve(junk, form="primal", tol=0.0, max_iter=5, check_every=0)
    sol.profile_kernel(junk, cdcs.K_PROJECT, reps=7)
    sol.solve(junk, form="primal", tol=0.0, max_iter=9, check_every=3)
    b = sol.new_state("primal")
    sol.solve(b, form="primal", tol=0.0, max_iter=12, check_every=4)
    for k in ("x", "blk", "lam"):
        assert torch.equal(a[k], b[k]), k
    sol.close()


def test_parallel_bucket_launches_give_the_same_bits(torch, small):
    """The per-bucket launches on parallel streams run the same kernels on
    the same cliques as in stream order: eager and graph-captured solves of
    both plans agree bit for bit, and the plan is reported."""
    prob, _ = small
    sol = cdcs.Solver(prob)
    out = {}
    for parallel in (False, True):
        sol.set_projection_plan(False, 256, parallel=parallel)
        assert sol.tuning()["parallel_buckets"] == parallel and not sol.tuning()["persistent"]
        for ce in (0, 10):
            st = sol.new_state("primal")
            sol.solve(st, form="primal", tol=0.0, max_iter=20, check_every=ce)
            out[(parallel, ce)] = {k: st[k].clone() for k in ("x", "blk", "lam", "vw")}
    for key in out:
        for k in ("x", "blk", "lam", "vw"):
            assert torch.equal(out[key][k], out[(False, 0)][k]), (key, k)
    sol.close()


def test_queue_and_bucket_launches_agree(torch, small):
    prob, _ = small
    out = []
    for plan in [(True, 256), (False, 256)]:
        sol = cdcs.Solver(prob)
        sol.set_projection_plan(*plan)
        st = sol.new_state("primal")
        sol.solve(st, form="primal", tol=0.0, max_iter=20, check_every=10)
        out.append(st["x"].cpu().numpy())
        sol.close()
    assert _rel(out[0], out[1]) <= 1e-6


def test_tuning_report_and_plan_errors(torch, small):
    prob, _ = small
    sol = cdcs.Solver(prob)
    t = sol.tuning()
    assert t["queue_us"] > 0 and t["buckets_us"] > 0 and t["parallel_us"] > 0
    # the fastest of the three forms
    assert t["persistent"] == (t["queue_us"] < min(t["buckets_us"], t["parallel_us"]))
    assert t["parallel_buckets"] == (not t["persistent"] and t["parallel_us"] < t["buckets_us"])
    assert sum(b["count"] for b in t["buckets"]) == prob.p
    assert [b["size"] for b in t["buckets"]] == sorted(b["size"] for b in t["buckets"])
    assert all(b["size"] in (16, 32, 48, 64, 80, 96, 112, 128) for b in t["buckets"])
    if t["persistent"]:
        assert t["threads"] in (256, 512) and 0 < t["grid"] <= prob.p
    with pytest.raises(cdcs.CdcsError) as e:
        sol.set_projection_plan(True, 64)
    assert e.value.status == cdcs.E_ARG
    with pytest.raises(cdcs.CdcsError):
        sol.set_projection_plan(False, 100)
    sol.close()


def test_batch_handle_queue_plan(torch):
    """The queue launch over the cliques of many instances, with per-instance
    stopping flags."""
    shapes = [(10, 10, 5, 50), (5, 8, 2, 25), (7, 12, 6, 35), (3, 4, 3, 9)]
    probs = [synth.block_arrow(l, d, h, m, seed=900 + i) for i, (l, d, h, m) in enumerate(shapes)]
    res = {}
    for plan in [(True, 256), (False, 256)]:
        sol = cdcs.BatchSolver(probs)
        sol.set_projection_plan(*plan)
        st = sol.new_state("primal")
        info = sol.solve(st, form="primal", tol=1e-4, max_iter=2000, check_every=25)
        assert info.converged
        res[plan] = [i.iters for i in sol.instance_info()], st["x"].cpu().numpy()
        sol.close()
    (it_q, x_q), (it_b, x_b) = res[(True, 256)], res[(False, 256)]
    assert it_q == it_b
    assert _rel(x_q, x_b) <= 1e-6


def test_queue_with_many_cliques_per_workgroup(torch):
    """More cliques than queue workgroups, so every workgroup projects several
    cliques of different buckets in turn inside one launch (LDS and the
    warm-start state pass from clique to clique).  The queue launch must
    agree with the per-bucket launches through warm-started ADMM iterations,
    and the eigensolver must stay at its warm-start sweep count."""
    prob = synth.peo_chordal(p=1500, smin=4, smax=96, omax=8, m=2000, nnz_row=20, seed=4242)
    out = {}
    for plan in [(True, 512), (False, 512)]:
        sol = cdcs.Solver(prob)
        sol.set_projection_plan(*plan)
        t = sol.tuning()
        if plan[0]:
            assert t["grid"] < prob.p  # several cliques per workgroup
        st = sol.new_state("primal")
        info = sol.solve(st, form="primal", tol=0.0, max_iter=60, check_every=20)
        assert info.jacobi_cap_hits == 0
        out[plan] = (st["x"].cpu().numpy(), _lam(sol, st), info.jacobi_sweeps / (info.iters * prob.p))
        sol.close()
    (xq, lq, swq), (xb, lb, swb) = out[(True, 512)], out[(False, 512)]
    assert _rel(xq, xb) <= 1e-5
    assert _rel(lq, lb) <= 1e-5
    assert swq <= 1.25 * swb + 0.05


@pytest.mark.parametrize("threads,grid", [(256, 4), (512, 3), (256, 1)])
def test_queue_with_several_cliques_per_workgroup_vs_oracle(torch, small, threads, grid):
    """A queue launch with a grid far below the clique count: each workgroup
    draws cliques of several size buckets in turn (largest first), carrying
    LDS and the warm-start state from clique to clique, through 30 ADMM
    iterations; the iterates must match the oracle."""
    prob, ref = small
    sol = cdcs.Solver(prob)
    sol.set_projection_plan(True, threads, grid)
    t = sol.tuning()
    assert t["persistent"] and t["grid"] == grid and t["threads"] == threads
    st = sol.new_state("primal")
    info = sol.solve(st, form="primal", tol=0.0, max_iter=30, check_every=10)
    assert info.iters == 30 and info.jacobi_cap_hits == 0
    assert _rel(st["x"].cpu().numpy(), ref.x) <= 1e-4
    assert _rel(st["blk"].cpu().numpy().astype(np.float64), cdcs.pack_blocks(ref.blocks)) <= 1e-4
    assert _rel(_lam(sol, st), np.concatenate([B.ravel() for B in ref.lam])) <= 1e-4
    sol.close()


def test_queue_grid_limits(torch, small):
    prob, _ = small
    sol = cdcs.Solver(prob)
    sol.set_projection_plan(True, 256)
    gmax = sol.tuning()["grid"]
    with pytest.raises(cdcs.CdcsError) as e:
        sol.set_projection_plan(True, 256, gmax + 1)
    assert e.value.status == cdcs.E_ARG
    with pytest.raises(cdcs.CdcsError):
        sol.set_projection_plan(True, 256, -1)
    sol.close()


@pytest.mark.parametrize("plan", [(True, 256, 5), (True, 512, 0), (False, 256, 0), (False, 64, 0)])
def test_project_cliques_with_the_plan_vs_oracle(torch, small, plan):
    """cdcs_psd_project_cliques: the handle's launch plan on given blocks
    (cold start), per clique within 1e-5 ||W||_F of the oracle's projection."""
    prob, _ = small
    sol = cdcs.Solver(prob)
    sol.set_projection_plan(*plan)
    sizes = np.asarray(sol.sizes)
    blocks = [synth.random_symmetric(int(s), seed=300 + k) for k, s in enumerate(sizes)]
    W32 = [np.asarray(B, dtype=np.float32) for B in blocks]
    Wp = torch.as_tensor(cdcs.pack_blocks(W32), device="cuda")
    P = cdcs.unpack_blocks(sol.project_cliques(Wp).cpu().numpy(), sizes, sol.offsets)
    for B, G in zip(W32, P):
        ref = O.psd_project(B.astype(np.float64))
        assert np.linalg.norm(G - ref) <= 1e-5 * np.linalg.norm(B.astype(np.float64))
    # the plan's repeated launches give the same bits (the queue's tickets stay aligned)
    P2 = sol.project_cliques(Wp).cpu().numpy()
    P3 = sol.project_cliques(Wp).cpu().numpy()
    assert np.array_equal(P2, P3)
    sol.close()


@pytest.mark.parametrize("plan", [(True, 512), (False, 256), (False, 512), (False, 0)],
                         ids=["queue512", "buckets256", "buckets512", "tuned"])
def test_cliques_up_to_126_vs_oracle(torch, plan):
    """A clique tree with cliques of 60..126 vertices (buckets 64 to 128):
    every launch plan through 20 ADMM iterations against the oracle (the
    queue launch over buckets above 96 takes 512 threads only)."""
    prob = synth.peo_chordal(p=8, smin=60, smax=126, omax=8, m=60, nnz_row=20, seed=4343)
    assert prob.clique_sizes().max() > 112
    ref = O.Oracle(prob).solve("primal", rho=1.0, max_iter=20)
    sol = cdcs.Solver(prob)
    with pytest.raises(cdcs.CdcsError) as e:
        sol.set_projection_plan(True, 256)
    assert e.value.status == cdcs.E_ARG
    if plan != (False, 0):
        sol.set_projection_plan(*plan)
    st = sol.new_state("primal")
    info = sol.solve(st, form="primal", tol=0.0, max_iter=20, check_every=10)
    assert info.iters == 20 and info.jacobi_cap_hits == 0
    assert _rel(st["x"].cpu().numpy(), ref.x) <= 1e-4
    assert _rel(_lam(sol, st), np.concatenate([B.ravel() for B in ref.lam])) <= 1e-4
    sol.close()
