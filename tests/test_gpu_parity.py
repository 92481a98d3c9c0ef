"""Parity of the gfx950 library against the CPU FP64 oracle (needs a GPU).

Tolerances (per result, relative):
  * per-clique projection: ||P_gpu - P_ref||_F / ||W||_F <= 1e-5 (FP32 eigensolve);
  * affine projection (FP64 solve, FP32-exact A): <= 1e-10;
  * ADMM iterates after 50 iterations: ||x_gpu - x_ref|| / ||x_ref|| <= 1e-4, same for x_k, lambda_k;
  * converged objective: |obj_gpu - obj_ref| / max(1, |obj_ref|) <= 1e-4.
"""
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


def _f32(B):
    return np.asarray(B, dtype=np.float32).astype(np.float64)


def _proj_err(torch, blocks):
    """Max per-block relative error of the batched projection vs the oracle."""
    sizes = np.array([B.shape[0] for B in blocks])
    W32 = [np.asarray(B, dtype=np.float32) for B in blocks]
    Wp = torch.as_tensor(cdcs.pack_blocks(W32), device="cuda")
    P = cdcs.psd_project_batched(Wp, sizes).cpu().numpy()
    Pb = cdcs.unpack_blocks(P, sizes)
    errs = []
    for B, G in zip(W32, Pb):
        ref = O.psd_project(B.astype(np.float64))
        nw = np.linalg.norm(B.astype(np.float64))
        errs.append(np.linalg.norm(G - ref) / nw if nw > 0 else np.linalg.norm(G))
    return np.array(errs), Pb


SWEEP = [1, 2, 3, 4, 5, 7, 8, 15, 16, 17, 24, 30, 31, 32, 33, 40, 44, 63, 64, 65, 80, 95, 96, 97, 111, 112, 113,
         120, 125, 126]


@pytest.mark.parametrize("bucket", [(1, 32), (33, 64), (65, 96), (97, 126)])
def test_projection_parity_size_sweep(torch, bucket):
    lo, hi = bucket
    sizes = [s for s in SWEEP if lo <= s <= hi] * 2
    blocks = [synth.random_symmetric(s, seed=1000 + 7 * t + s) for t, s in enumerate(sizes)]
    errs, _ = _proj_err(torch, blocks)
    assert errs.max() <= 1e-5, (errs.max(), sizes[int(errs.argmax())])


def test_projection_mixed_buckets_in_one_call(torch):
    sizes = [96, 3, 50, 31, 64, 1, 17]
    blocks = [synth.random_symmetric(s, seed=77 + s) for s in sizes]
    errs, _ = _proj_err(torch, blocks)
    assert errs.max() <= 1e-5


def test_projection_special_cases(torch):
    rng = np.random.default_rng(3)
    G = rng.standard_normal((20, 20))
    S = G @ G.T
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    rep = (Q * np.array([2.0] * 5 + [-1.0] * 4 + [0.0] * 3)) @ Q.T
    cases = [np.zeros((6, 6)), S, -S, np.diag([3.0, -1.0, 0.5, -2.0]), rep,
             1e-20 * synth.random_symmetric(10, 5), 1e20 * synth.random_symmetric(10, 6),
             np.array([[-4.0]]), np.array([[4.0]])]
    errs, Pb = _proj_err(torch, cases)
    assert errs.max() <= 1e-5, errs
    assert np.array_equal(Pb[0], np.zeros((6, 6)))
    assert np.abs(Pb[2]).max() <= 1e-5 * np.linalg.norm(S)


def test_projection_rank_extremes(torch):
    """Every eigenvalue positive at full bucket sizes (the rebuild sums over
    all columns), none positive, and a few positive eigenvalues (a sum
    shorter than the block, padded with zero columns), across the buckets
    that multiply on the matrix cores."""
    rng = np.random.default_rng(11)
    cases = []
    for s, npos in ((32, 1), (48, 5), (64, 7), (80, 9), (95, 13), (96, 17)):
        G = rng.standard_normal((s, s))
        S = G @ G.T / s + 0.1 * np.eye(s)
        cases += [S, -S]
        Q, _ = np.linalg.qr(rng.standard_normal((s, s)))
        ev = -rng.uniform(0.5, 2.0, s)
        ev[:npos] *= -1.0
        cases.append((Q * ev) @ Q.T)
    errs, Pb = _proj_err(torch, cases)
    assert errs.max() <= 1e-5, (errs.max(), int(errs.argmax()))
    for t in range(1, len(cases), 3):  # negative definite: exactly zero
        assert np.abs(Pb[t]).max() <= 1e-6 * np.linalg.norm(cases[t]), t


def test_projection_eigen_outputs(torch):
    sizes = np.array([5, 30, 64])
    blocks = [np.asarray(synth.random_symmetric(s, seed=s), dtype=np.float32) for s in sizes]
    Wp = torch.as_tensor(cdcs.pack_blocks(blocks), device="cuda")
    P, ev, V, eoff, voff = cdcs.psd_project_batched(Wp, sizes, eig=True)
    ev, V, eoff, voff = ev.cpu().numpy(), V.cpu().numpy(), eoff.cpu().numpy(), voff.cpu().numpy()
    for t, s in enumerate(sizes):
        lam = ev[eoff[t]:eoff[t + 1]].astype(np.float64)
        Vt = V[voff[t]:voff[t + 1]].reshape(s, s).astype(np.float64)
        B = blocks[t].astype(np.float64)
        assert np.allclose(np.sort(lam), np.linalg.eigvalsh(B), atol=1e-5 * np.linalg.norm(B))
        assert np.linalg.norm(Vt.T @ Vt - np.eye(s)) <= 1e-5
        assert np.linalg.norm((Vt * lam) @ Vt.T - B) <= 1e-5 * np.linalg.norm(B)


@pytest.mark.parametrize("maker", ["c1", "mid"])
def test_affine_projection_parity(torch, maker):
    prob = synth.c1() if maker == "c1" else synth.block_arrow(l=20, d=12, h=6, m=300, seed=42)
    orc = O.Oracle(prob)
    sol = cdcs.Solver(prob)
    rng = np.random.default_rng(1)
    r1 = rng.standard_normal(prob.nU)
    r2 = rng.standard_normal(prob.m)
    x, y = sol.affine_project(torch.as_tensor(r1, device="cuda"), torch.as_tensor(r2, device="cuda"))
    xr, yr = orc.kkt.solve(r1, r2)
    x, y = x.cpu().numpy(), y.cpu().numpy()
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) <= 1e-10
    assert np.linalg.norm(y - yr) / np.linalg.norm(yr) <= 1e-10
    # KKT rows: D x + A^T y = r1 and sum_e w A x = r2
    A = prob.A_dense()
    assert np.allclose(orc.dec.D * x + A.T @ y, r1, atol=1e-9)
    assert np.allclose(A @ (orc.dec.w * x), r2, atol=1e-9)
    sol.close()


def _blocks_of(sol, packed_t):
    return cdcs.unpack_blocks(packed_t.cpu().numpy().astype(np.float64), sol.sizes, sol.offsets)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("form", ["primal", "dual"])
@pytest.mark.parametrize("graph", [0, 10])
def test_admm_iterates_after_50_iterations_c1(torch, form, graph):
    prob = synth.c1()
    ref = O.Oracle(prob).solve(form, rho=1.0, max_iter=50)
    sol = cdcs.Solver(prob)
    st = sol.new_state(form)
    info = sol.solve(st, form=form, rho=1.0, tol=0.0, max_iter=50, check_every=graph)
    assert info.iters == 50 and info.jacobi_cap_hits == 0
    assert _rel(st["x"].cpu().numpy(), ref.x) <= 1e-4
    blk = _blocks_of(sol, st["blk"])
    lam = _blocks_of(sol, st["lam"])
    assert _rel(np.concatenate([B.ravel() for B in blk]), np.concatenate([B.ravel() for B in ref.blocks])) <= 1e-4
    assert _rel(np.concatenate([B.ravel() for B in lam]), np.concatenate([B.ravel() for B in ref.lam])) <= 1e-4
    if form == "dual":
        v = _blocks_of(sol, st["v"])
        assert _rel(np.concatenate([B.ravel() for B in v]), np.concatenate([B.ravel() for B in ref.v])) <= 1e-4
    hist = sol.history(50)
    assert np.allclose(hist[:, 0], ref.eps_p, rtol=1e-3, atol=1e-7)
    assert np.allclose(hist[:, 1], ref.eps_d, rtol=1e-3, atol=1e-7)
    sol.close()


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_converged_objective_c1(torch, form):
    prob = synth.c1()
    ref = O.Oracle(prob).solve(form, rho=1.0, max_iter=2000, tol=1e-4)
    sol = cdcs.Solver(prob)
    st = sol.new_state(form)
    info = sol.solve(st, form=form, rho=1.0, tol=1e-4, max_iter=2000, check_every=50)
    assert info.converged and ref.converged
    for got, want in [(info.obj_primal, ref.obj_primal), (info.obj_dual, ref.obj_dual)]:
        assert abs(got - want) / max(1.0, abs(want)) <= 1e-4
    assert abs(info.iters - ref.iters) <= max(3, ref.iters // 50)
    sol.close()


def test_graph_and_eager_give_identical_bits(torch):
    prob = synth.block_arrow(l=12, d=8, h=4, m=40, seed=9)
    sol = cdcs.Solver(prob)
    outs = []
    for graph in [0, 7, 7]:
        st = sol.new_state("primal")
        sol.solve(st, form="primal", tol=0.0, max_iter=21, check_every=graph)
        outs.append([st[k].cpu().numpy().copy() for k in ("x", "y", "blk", "lam")])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
    sol.close()


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_split_solve_equals_one_solve(torch, form):
    """18 + 12 iterations from the saved state equal 30 in one solve, bit for
    bit: the state carries the eigensolver's eigenvector warm start (vw) from
    one call to the next."""
    prob = synth.c1()
    sol = cdcs.Solver(prob)
    assert sol.nwarm == int(np.sum(np.asarray(sol.sizes, dtype=np.int64) ** 2))
    a = sol.new_state(form)
    sol.solve(a, form=form, tol=0.0, max_iter=30, check_every=0)
    b = sol.new_state(form)
    sol.solve(b, form=form, tol=0.0, max_iter=18, check_every=6)
    sol.solve(b, form=form, tol=0.0, max_iter=12, check_every=0)
    keys = ("x", "y", "blk", "lam", "vw") + (("v",) if form == "dual" else ())
    for k in keys:
        assert torch.equal(a[k], b[k]), k
    sol.close()


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_split_solve_without_warm_buffer(torch, form):
    """Without vw in the state the handle restarts the eigenvector warm start
    from the identity in every solve, so iteration 19 takes a cold Jacobi run:
    the same projection to FP32 accuracy, not the same bits."""
    prob = synth.c1()
    sol = cdcs.Solver(prob)
    a = sol.new_state(form)
    sol.solve(a, form=form, tol=0.0, max_iter=30, check_every=0)
    b = sol.new_state(form)
    b["vw"] = None
    sol.solve(b, form=form, tol=0.0, max_iter=18, check_every=0)
    sol.solve(b, form=form, tol=0.0, max_iter=12, check_every=0)
    keys = ("x", "blk", "lam", "v") if form == "dual" else ("x", "blk", "lam")
    for k in keys:
        assert _rel(b[k].cpu().numpy().astype(np.float64), a[k].cpu().numpy().astype(np.float64)) <= 1e-5
    # a solve without vw is a function of the rest of the state
    c = sol.new_state(form)
    c["vw"] = None
    sol.solve(c, form=form, tol=0.0, max_iter=18, check_every=0)
    d = {k: (v.clone() if v is not None else None) for k, v in c.items()}
    sol.solve(c, form=form, tol=0.0, max_iter=12, check_every=0)
    sol.solve(d, form=form, tol=0.0, max_iter=12, check_every=4)
    for k in keys:
        assert torch.equal(c[k], d[k]), k
    with pytest.raises(cdcs.CdcsError) as e:
        cdcs._check(cdcs.load_library().cdcs_warm_reset(sol._h, None, None), "cdcs_warm_reset")
    assert e.value.status == cdcs.E_ARG
    sol.close()


def test_setup_errors(torch):
    prob = synth.block_arrow(l=3, d=3, h=2, m=4, seed=1)
    bad = synth.Problem(**{**prob.__dict__})
    bad.A = prob.A.copy()
    bad.A[3] = bad.A[2]
    with pytest.raises(cdcs.CdcsError) as e:
        cdcs.Solver(bad)
    assert e.value.status == cdcs.E_RANK
    bad2 = synth.Problem(**{**prob.__dict__})
    bad2.clique_vert = prob.clique_vert.copy()
    bad2.clique_vert[[0, 1]] = bad2.clique_vert[[1, 0]]
    with pytest.raises(cdcs.CdcsError) as e:
        cdcs.Solver(bad2)
    assert e.value.status == cdcs.E_PATTERN


# ---- the benchmark workload: block-arrow l=200, d=20, h=10, m=2000 ------------

@pytest.fixture(scope="module")
def c2(torch):
    prob = synth.c2()
    return prob


def test_c2_affine_projection_parity(torch, c2):
    orc = O.Oracle(c2)
    sol = cdcs.Solver(c2)
    assert not sol.sparse_a and not sol.sparse_factor  # dense constraints: dense factor
    rng = np.random.default_rng(2)
    r1 = rng.standard_normal(c2.nU)
    r2 = rng.standard_normal(c2.m)
    x, y = sol.affine_project(torch.as_tensor(r1, device="cuda"), torch.as_tensor(r2, device="cuda"))
    xr, yr = orc.kkt.solve(r1, r2)
    assert _rel(x.cpu().numpy(), xr) <= 1e-10
    assert _rel(y.cpu().numpy(), yr) <= 1e-10
    sol.close()


def test_c2_solve_as_benchmarked(torch, c2):
    """Graph-captured solve, 500-iteration cap, tol 1e-4: converges, and the
    result satisfies the SDP optimality conditions (any-size property)."""
    sol = cdcs.Solver(c2)
    st = sol.new_state("primal")
    info = sol.solve(st, form="primal", rho=1.0, tol=1e-4, max_iter=500, check_every=50)
    assert info.jacobi_cap_hits == 0
    assert info.converged, info
    x = st["x"].cpu().numpy()
    y_sdp = -st["y"].cpu().numpy()
    A = c2.A
    w = np.where(c2.ei == c2.ej, 1.0, 2.0)
    pinf = np.linalg.norm(A @ (w * x) - c2.b) / (1 + np.linalg.norm(c2.b))
    assert pinf <= 1e-6
    gap = abs(info.obj_primal - info.obj_dual) / (1 + abs(info.obj_primal) + abs(info.obj_dual))
    assert gap <= 1e-3
    assert np.isclose(info.obj_dual, float(np.dot(c2.b, y_sdp)), rtol=1e-12)
    sol.close()
