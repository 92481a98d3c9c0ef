"""Differentiation through the gfx950 library (needs a GPU).

The FP32 projection adjoint (Daleckii-Krein) and the unrolled-ADMM gradients
are compared with the oracle's FP64 reverse-mode derivative (tolerance 1e-3
relative, FP32 eigensolves) and, at the differentiation workload, with FP64
central finite differences of the oracle (tests/golden/c5_fd.json, written by
tests/golden/make_c5_fd.py from oracle/ only)."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1609_06068_amd import cdcs, synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_fd.json")


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    cdcs.load_library()
    return _t


def _pack_grad_to_full(gp, k):
    """Packed cotangent -> symmetric G (off-diagonals halved)."""
    G = np.zeros((k, k))
    ia, ib = np.tril_indices(k)
    G[ia, ib] = gp
    G[ib, ia] = gp
    G[~np.eye(k, dtype=bool)] *= 0.5
    return G


def _full_to_packed_grad(Wbar, k):
    ia, ib = np.tril_indices(k)
    return np.where(ia == ib, Wbar[ia, ib], Wbar[ia, ib] + Wbar[ib, ia])


def test_projection_vjp_matches_oracle(torch):
    sizes = np.array([1, 3, 8, 17, 24, 30, 33, 48, 64, 80, 96, 100, 126])
    rng = np.random.default_rng(4)
    W32 = [np.asarray(synth.random_symmetric(int(s), seed=300 + int(s)), dtype=np.float32) for s in sizes]
    gps = [rng.standard_normal(int(s) * (int(s) + 1) // 2).astype(np.float32) for s in sizes]
    Wp = torch.as_tensor(cdcs.pack_blocks(W32), device="cuda")
    P, ev, V, eoff, voff = cdcs.psd_project_batched(Wp, sizes, eig=True)
    sizes_d = torch.as_tensor(sizes.astype(np.int32), device="cuda")
    off_d = torch.as_tensor(cdcs.packed_offsets(sizes), device="cuda")
    gP = torch.as_tensor(np.concatenate(gps), device="cuda")
    gW = cdcs.psd_project_vjp(gP, ev, V, eoff, voff, sizes_d, off_d, int(sizes.max())).cpu().numpy()
    off = cdcs.packed_offsets(sizes)
    for t, k in enumerate(sizes):
        k = int(k)
        lam, Q, _ = O.jacobi_eigh(W32[t].astype(np.float64))
        ref = _full_to_packed_grad(O.psd_project_vjp(lam, Q, _pack_grad_to_full(gps[t].astype(np.float64), k)), k)
        got = gW[off[t]:off[t + 1]]
        assert np.linalg.norm(got - ref) <= 1e-4 * max(1.0, np.linalg.norm(gps[t])), (k, np.linalg.norm(got - ref))


def test_gather_scatter_match_oracle(torch):
    prob = synth.c1()
    dec = O.Decomposition(prob)
    sol = cdcs.Solver(prob)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(prob.nU)
    packed = sol.gather(torch.as_tensor(x, device="cuda")).cpu().numpy()
    ref = cdcs.pack_blocks([dec.gather(x, k) for k in range(prob.p)])
    assert np.array_equal(packed, ref)
    blocks = []
    for s in prob.clique_sizes():
        R = rng.standard_normal((s, s))
        blocks.append(R + R.T)
    out = sol.scatter(torch.as_tensor(cdcs.pack_blocks(blocks), device="cuda")).cpu().numpy()
    assert np.allclose(out, dec.scatter(blocks), rtol=1e-14, atol=1e-14)
    sol.close()


def test_affine_adjoint_matches_oracle(torch):
    from paper_1609_06068_amd import autograd as ag
    prob = synth.c1()
    o = O.Oracle(prob)
    U = O.Unrolled(o, K=1)
    sol = cdcs.Solver(prob)
    rng = np.random.default_rng(5)
    r1 = torch.as_tensor(rng.standard_normal(prob.nU), device="cuda").requires_grad_(True)
    b = torch.as_tensor(prob.b, device="cuda").requires_grad_(True)
    gx = rng.standard_normal(prob.nU)
    x = ag.Affine.apply(r1, b, sol)
    x.backward(torch.as_tensor(gx, device="cuda"))
    r1bar, bbar = U._affine_adjoint(gx)
    assert np.allclose(r1.grad.cpu().numpy(), r1bar, rtol=1e-10, atol=1e-12)
    assert np.allclose(b.grad.cpu().numpy(), bbar, rtol=1e-10, atol=1e-12)
    sol.close()


def _gpu_grads(torch, prob, sol, K, which):
    from paper_1609_06068_amd import autograd as ag
    c = torch.as_tensor(prob.c, device="cuda").requires_grad_(True)
    b = torch.as_tensor(prob.b, device="cuda").requires_grad_(True)
    x = ag.unrolled_x(sol, c, b, K=K, rho=1.0)
    w = ag.entry_weights(prob)
    if which == "linear":
        L = (w * c * x).sum()
    else:
        d = x - torch.as_tensor(prob.meta["x0"], device="cuda")
        L = (w * d * d).sum()
    L.backward()
    return float(L.detach()), c.grad.cpu().numpy(), b.grad.cpu().numpy(), x.detach().cpu().numpy()


@pytest.mark.parametrize("which", ["linear", "target"])
def test_unrolled_gradient_c1(torch, which):
    prob = synth.c1()
    o = O.Oracle(prob)
    K = 20
    U = O.Unrolled(o, K=K)
    x = U.forward(prob.c, prob.b)
    if which == "linear":
        L, g = O.loss_linear(prob, o.dec, x)
        direct = o.dec.w * x
    else:
        L, g = O.loss_target(o.dec, x, prob.meta["x0"])
        direct = 0.0
    cbar, bbar = U.backward(g)
    cbar = cbar + direct
    sol = cdcs.Solver(prob)
    Lg, gc, gb, xg = _gpu_grads(torch, prob, sol, K, which)
    assert np.linalg.norm(xg - x) <= 1e-5 * np.linalg.norm(x)
    assert abs(Lg - L) <= 1e-5 * max(1.0, abs(L))
    dc = synth.unit_directions(prob.nU, 20, 77)
    db = synth.unit_directions(prob.m, 20, 78)
    for D, got, ref in [(dc, gc, cbar), (db, gb, bbar)]:
        a, r = D @ got, D @ ref
        assert np.all(np.abs(a - r) <= 1e-3 * np.maximum(np.abs(r), 1e-3 * np.abs(r).max())), (a, r)
    # the gradient is a deterministic function of (c, b)
    _, gc2, gb2, _ = _gpu_grads(torch, prob, sol, K, which)
    assert np.array_equal(gc2, gc) and np.array_equal(gb2, gb)
    sol.close()


def test_unrolled_forward_is_the_product_iteration(torch):
    """cdcs_unrolled_step with the handle's own c and b is cdcs_admm_step bit
    for bit (the gradient is taken through the iteration the solver runs),
    and it saves the eigenpairs of that iteration's projections."""
    prob = synth.c3_small()
    sol = cdcs.Solver(prob)
    a = sol.new_state("primal")
    bst = sol.new_state("primal")
    c = torch.as_tensor(prob.c, device="cuda")
    b = torch.as_tensor(prob.b, device="cuda")
    ev = torch.empty(sol.nevals, dtype=torch.float32, device="cuda")
    V = torch.empty(sol.nwarm, dtype=torch.float32, device="cuda")
    for _ in range(7):
        sol.step(a, form="primal")
        sol.unrolled_step(bst, c, b, 1.0, ev, V)
    for k in ("x", "y", "blk", "lam", "vw"):
        assert torch.equal(a[k], bst[k]), k
    assert torch.equal(V, bst["vw"])
    # the saved eigenpairs reproduce the last projection: x_k = V max(L, 0) V^T
    sizes = np.asarray(sol.sizes)
    eo = np.concatenate([[0], np.cumsum(sizes)])
    vo = np.concatenate([[0], np.cumsum(sizes * sizes)])
    evh, Vh = ev.cpu().numpy().astype(np.float64), V.cpu().numpy().astype(np.float64)
    blk = cdcs.unpack_blocks(bst["blk"].cpu().numpy().astype(np.float64), sizes, sol.offsets)
    for k, s in enumerate(sizes):
        Q = Vh[vo[k]:vo[k + 1]].reshape(s, s)
        P = (Q * np.maximum(evh[eo[k]:eo[k + 1]], 0.0)) @ Q.T
        assert np.linalg.norm(P - blk[k]) <= 1e-5 * max(1.0, np.linalg.norm(blk[k]))
    sol.close()


@pytest.mark.parametrize("which", ["linear", "target"])
def test_c5_gradients_vs_oracle_and_finite_differences(torch, which):
    """Differentiation workload: l=100, d=16, h=8, m=800, K=100 unrolled
    iterations with per-iteration checkpointing, 20 directions in c and b."""
    gold = json.load(open(GOLDEN))
    prob = synth.c5()
    sol = cdcs.Solver(prob)
    _, gc, gb, _ = _gpu_grads(torch, prob, sol, 100, which)
    dc = synth.unit_directions(prob.nU, gold["directions"], gold["seed_c"])
    db = synth.unit_directions(prob.m, gold["directions"], gold["seed_b"])
    for key, D, g in [("dc", dc, gc), ("db", db, gb)]:
        got = D @ g
        adj = np.asarray(gold["oracle_adjoint"][which][key])
        f6 = np.asarray(gold["fd"]["1e-06"][which][key])
        f5 = np.asarray(gold["fd"]["1e-05"][which][key])
        scale = np.abs(adj).max()
        # the FP32 adjoint against the FP64 reverse-mode derivative
        assert np.all(np.abs(got - adj) <= 1e-3 * np.maximum(np.abs(adj), 1e-2 * scale)), (key, got, adj)
        # against FP64 central differences (step 1e-6), within the FD error
        # band measured by the step-1e-5 differences
        band = 2 * np.abs(f6 - f5) + 1e-3 * np.abs(adj)
        assert np.all(np.abs(got - f6) <= band + 1e-3 * np.abs(f6)), (key, got, f6)
    sol.close()
