"""Uneven cliques with a sparse A (needs a GPU).

The clique-tree generator runs at two sizes: 40 cliques of 4..96 vertices with
m = 150 constraints, where the oracle runs Algorithms 1 and 2 in seconds
(element-by-element parity); and the full workload of 3000 cliques with
m = 8000 constraints of 20 coefficients each, checked through properties
that hold at any size: the KKT rows of the affine projection, the projection
characterisation P(W) >= 0, P(W) - W >= 0, <P(W), P(W) - W> = 0 on sampled
cliques, and oracle projections of sampled generator blocks.

Tolerances as for the block-arrow workloads: affine projection 1e-10
(FP64 solve), projection 1e-5 relative to ||W||_F (FP32 eigensolve), ADMM
iterates after 50 iterations 1e-4."""
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


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def _csr(prob):
    import scipy.sparse as sp
    return sp.csr_matrix((prob.A_val, prob.A_idx.astype(np.int64), prob.A_ptr), shape=(prob.m, prob.nU))


def _kkt_rows(prob, D, x, y, r1, r2):
    """Relative residuals of D x + A^T y = r1 and sum_e w_e A_ie x_e = r2."""
    A = _csr(prob)
    w = np.where(prob.ei == prob.ej, 1.0, 2.0)
    return (np.linalg.norm(D * x + A.T @ y - r1) / np.linalg.norm(r1),
            np.linalg.norm(A @ (w * x) - r2) / np.linalg.norm(r2))


# ---- small instance: element-by-element parity with the oracle -------------

@pytest.fixture(scope="module")
def small(torch):
    prob = synth.c3_small()
    return prob, O.Oracle(prob)


def test_small_instance_takes_the_sparse_path(torch, small):
    prob, _ = small
    sol = cdcs.Solver(prob)
    assert sol.sparse_a and sol.nnz_a == prob.A_idx.shape[0]
    sizes = prob.clique_sizes()
    assert sizes.min() <= 16 and sizes.max() > 64   # every size bucket is used
    sol.close()


def test_small_affine_projection_parity(torch, small):
    prob, orc = small
    sol = cdcs.Solver(prob)
    rng = np.random.default_rng(31)
    r1 = rng.standard_normal(prob.nU)
    r2 = rng.standard_normal(prob.m)
    x, y = sol.affine_project(torch.as_tensor(r1, device="cuda"), torch.as_tensor(r2, device="cuda"))
    x, y = x.cpu().numpy(), y.cpu().numpy()
    xr, yr = orc.kkt.solve(r1, r2)
    assert _rel(x, xr) <= 1e-10 and _rel(y, yr) <= 1e-10
    e1, e2 = _kkt_rows(prob, orc.dec.D, x, y, r1, r2)
    assert e1 <= 1e-12 and e2 <= 1e-12
    sol.close()


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_small_iterates_after_50_iterations(torch, small, form):
    prob, orc = small
    ref = orc.solve(form, rho=1.0, max_iter=50)
    sol = cdcs.Solver(prob)
    st = sol.new_state(form)
    info = sol.solve(st, form=form, rho=1.0, tol=0.0, max_iter=50, check_every=25)
    assert info.iters == 50 and info.jacobi_cap_hits == 0
    assert _rel(st["x"].cpu().numpy(), ref.x) <= 1e-4
    off, sizes = sol.offsets, sol.sizes
    blk = cdcs.unpack_blocks(st["blk"].cpu().numpy().astype(np.float64), sizes, off)
    lam = cdcs.unpack_blocks(st["lam"].cpu().numpy().astype(np.float64), sizes, off)
    assert _rel(np.concatenate([B.ravel() for B in blk]), np.concatenate([B.ravel() for B in ref.blocks])) <= 1e-4
    assert _rel(np.concatenate([B.ravel() for B in lam]), np.concatenate([B.ravel() for B in ref.lam])) <= 1e-4
    hist = sol.history(50)
    assert np.allclose(hist[:, 0], ref.eps_p, rtol=1e-3, atol=1e-7)
    assert np.allclose(hist[:, 1], ref.eps_d, rtol=1e-3, atol=1e-7)
    sol.close()


# ---- the full uneven workload: any-size properties and sampled outputs ------

@pytest.fixture(scope="module")
def full(torch):
    prob = synth.c3()
    sol = cdcs.Solver(prob)
    yield prob, sol, O.Decomposition(prob)
    sol.close()


def test_full_affine_projection_kkt_rows(torch, full):
    prob, sol, dec = full
    assert sol.sparse_a and sol.m == 8000 and sol.p == 3000
    # constraints with 20 random entries rarely share one: M is nearly
    # diagonal and its inverse factor is kept sparse
    assert sol.sparse_factor and sol.nnz_factor < 8000 * 8001 // 16
    rng = np.random.default_rng(32)
    r1 = rng.standard_normal(prob.nU)
    r2 = rng.standard_normal(prob.m)
    x, y = sol.affine_project(torch.as_tensor(r1, device="cuda"), torch.as_tensor(r2, device="cuda"))
    e1, e2 = _kkt_rows(prob, dec.D, x.cpu().numpy(), y.cpu().numpy(), r1, r2)
    assert e1 <= 1e-10 and e2 <= 1e-10, (e1, e2)


def test_full_first_iteration_projection_properties(torch, full):
    """One iteration of Alg. 1 from zero: x solves the KKT system with
    r1 = -c, r2 = b; each sampled clique block is the PSD projection of
    W_k = H_k x, and lambda_k = rho (X_k - W_k)."""
    prob, sol, dec = full
    st = sol.new_state("primal")
    info = sol.solve(st, form="primal", rho=1.0, tol=0.0, max_iter=1, check_every=0)
    assert info.iters == 1 and info.jacobi_cap_hits == 0
    x = st["x"].cpu().numpy()
    e1, e2 = _kkt_rows(prob, dec.D, x, st["y"].cpu().numpy(), -prob.c, prob.b)
    assert e1 <= 1e-10 and e2 <= 1e-10, (e1, e2)
    off, sizes = sol.offsets, sol.sizes
    blk_all = st["blk"].cpu().numpy().astype(np.float64)
    lam_all = st["lam"].cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(33)
    order = np.argsort(sizes)
    sample = np.concatenate([order[:5], order[-5:], rng.choice(prob.p, 30, replace=False)])
    for k in sample:
        k = int(k)
        s = int(sizes[k])
        W = dec.gather(x, k)
        nw = np.linalg.norm(W)
        X = cdcs.unpack_blocks(blk_all[off[k]:off[k + 1]], [s])[0]
        L = cdcs.unpack_blocks(lam_all[off[k]:off[k + 1]], [s])[0]
        assert np.linalg.eigvalsh(X).min() >= -1e-5 * nw, k
        assert np.linalg.eigvalsh(X - W).min() >= -1e-5 * nw, k
        assert abs(np.sum(X * (X - W))) <= 1e-5 * nw * nw, k
        assert np.linalg.norm(L - (X - W)) <= 1e-5 * nw, k


def test_full_projection_sampled_against_oracle(torch, full):
    """The batched projection over all 3000 clique sizes of the workload in
    one call (generator blocks); 40 sampled blocks against the oracle."""
    prob = full[0]
    sizes = prob.clique_sizes()
    rng = np.random.default_rng(34)
    blocks32 = []
    for t, s in enumerate(sizes):
        R = rng.standard_normal((int(s), int(s))).astype(np.float32)
        blocks32.append((R + R.T) * np.float32(0.5))
    Wp = torch.as_tensor(cdcs.pack_blocks(blocks32), device="cuda")
    P = cdcs.psd_project_batched(Wp, sizes).cpu().numpy()
    off = cdcs.packed_offsets(sizes)
    for k in rng.choice(prob.p, 40, replace=False):
        k = int(k)
        s = int(sizes[k])
        got = cdcs.unpack_blocks(P[off[k]:off[k + 1]].astype(np.float64), [s])[0]
        W = blocks32[k].astype(np.float64)
        ref = O.psd_project(W)
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(W), (k, s)


def test_full_fifty_iterations_in_graphs(torch, full):
    prob, sol, _ = full
    st = sol.new_state("primal")
    info = sol.solve(st, form="primal", rho=1.0, tol=0.0, max_iter=50, check_every=25)
    assert info.iters == 50 and info.jacobi_cap_hits == 0
    hist = sol.history(50)
    assert np.all(np.isfinite(hist))
    assert hist[-1, 0] < hist[0, 0] and hist[-1, 1] < hist[1, 1]
    x = st["x"].cpu().numpy()
    assert np.all(np.isfinite(x))
