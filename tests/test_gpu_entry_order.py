"""Entry order at the interface (needs a GPU).  A problem and the same problem
with its pattern entries listed in a shuffled order must give the same results
up to that permutation, bit for bit: the handle numbers entries internally by
their first appearance in the packed clique blocks, which does not depend on
the listing order, and permutes global vectors at every entry point."""
import dataclasses

import numpy as np
import pytest

from paper_1609_06068_amd import cdcs, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    cdcs.load_library()
    return _t


def _shuffled(prob, seed):
    """The same SDP with entry q of the new list = entry perm[q] of the old."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(prob.nU)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(prob.nU)
    kw = dict(ei=prob.ei[perm].copy(), ej=prob.ej[perm].copy(), c=prob.c[perm].copy())
    if prob.A is not None:
        kw["A"] = np.ascontiguousarray(prob.A[:, perm])
    else:
        kw["A_idx"] = inv[prob.A_idx].astype(prob.A_idx.dtype)
    return dataclasses.replace(prob, **kw), perm


@pytest.mark.parametrize("name", ["c1", "c3_small"])  # dense A / sparse (CSR) A
def test_shuffled_entry_order_gives_permuted_results(torch, name):
    prob = getattr(synth, name)()
    sprob, perm = _shuffled(prob, 5)
    perm_t = torch.as_tensor(perm, device="cuda")
    out = []
    for p in (prob, sprob):
        sol = cdcs.Solver(p)
        sol.set_projection_plan(False, 256)  # same launches on both handles
        st = sol.new_state("primal")
        info = sol.solve(st, form="primal", tol=0.0, max_iter=30, check_every=10)
        assert info.iters == 30
        out.append((sol, st))
    (sol0, st0), (sol1, st1) = out
    # ADMM iterates: global x permuted, clique blocks and multipliers identical
    assert torch.equal(st1["x"], st0["x"][perm_t])
    assert torch.equal(st1["y"], st0["y"])
    assert torch.equal(st1["blk"], st0["blk"])
    assert torch.equal(st1["lam"], st0["lam"])
    # entry selectors and the affine projection on an arbitrary vector
    g = torch.Generator(device="cpu").manual_seed(11)
    v = torch.randn(prob.nU, dtype=torch.float64, generator=g).cuda()
    assert torch.equal(sol1.gather(v[perm_t]), sol0.gather(v))
    packed = torch.randn(sol0.nslots, dtype=torch.float64, generator=g).cuda()
    assert torch.equal(sol1.scatter(packed), sol0.scatter(packed)[perm_t])
    r2 = torch.randn(prob.m, dtype=torch.float64, generator=g).cuda()
    x0, y0 = sol0.affine_project(v, r2)
    x1, y1 = sol1.affine_project(v[perm_t], r2)
    assert torch.equal(x1, x0[perm_t])
    assert torch.equal(y1, y0)
    sol0.close()
    sol1.close()
