"""The sparse factor of M = A D^-1 A^T for sparse constraints (needs a GPU).

When A is kept sparse, the setup orders M's rows on the host (constraints
that share a pattern entry are adjacent; a perfect elimination order when that
graph is chordal, else minimum degree), computes L column by column on the
device, level by level of the elimination tree, and L^-1 along the tree paths;
no m x m matrix is formed.  Checked: the affine projection (the KKT solve it
serves) against the oracle's dense Cholesky and substitutions (1e-10
relative) for constraint graphs that are empty (independent rows), a chain
(deep elimination tree), a cycle (not chordal: minimum-degree fill) and the
clique-tree workload's random rows; duplicate rows are reported as
CDCS_E_RANK; the 3000-clique workload takes the sparse factor."""
import dataclasses

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


def _with_rows(prob, rows, seed):
    """prob with CSR constraints on the given entry lists (N(0,1) values,
    FP32-representable), b = A(X0)."""
    rng = np.random.default_rng(seed)
    ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.concatenate([np.asarray(r, dtype=np.int32) for r in rows])
    val = np.asarray(rng.standard_normal(idx.shape[0]), dtype=np.float32).astype(np.float64)
    w = np.where(prob.ei == prob.ej, 1.0, 2.0)
    b = np.array([np.dot(val[ptr[i]:ptr[i + 1]], (w * prob.meta["x0"])[idx[ptr[i]:ptr[i + 1]]])
                  for i in range(len(rows))])
    return dataclasses.replace(prob, A=None, A_ptr=ptr, A_idx=idx, A_val=val, b=b, meta=dict(prob.meta))


def _graphs(nU, m, kind, rng):
    """Entry lists of m constraints: 3 entries of their own each, plus shared
    entries that make M's graph: none; groups of 4 rows sharing one entry
    (4 x 4 blocks); 5-cycles (rows i, i+1 mod 5 of a group share an entry: not
    chordal); one chain through all rows (a path: its elimination tree is
    deep and L^-1 a dense triangle)."""
    pool = rng.choice(nU, size=3 * m + 2 * m + 1, replace=False)
    own = pool[:3 * m].reshape(m, 3)
    shared = pool[3 * m:]
    rows = []
    for i in range(m):
        r = set(int(v) for v in own[i])
        g, t = divmod(i, 5)
        if kind == "groups":
            r.add(int(shared[i // 4]))
        elif kind == "cycles":
            r |= {int(shared[5 * g + t]), int(shared[5 * g + (t + 4) % 5])}
        elif kind == "chain":
            r |= {int(shared[i]), int(shared[i + 1])}
        rows.append(sorted(r))
    return rows


@pytest.mark.parametrize("kind", ["independent", "groups", "cycles", "random", "chain"])
def test_sparse_factor_affine_projection_vs_oracle(torch, kind):
    base = synth.c3_small()
    rng = np.random.default_rng(11)
    if kind == "random":
        prob = base  # 20 random entries per row (the workload's own rows)
    else:
        prob = _with_rows(base, _graphs(base.nU, 120, kind, rng), seed=12)
    sol = cdcs.Solver(prob)
    assert sol.sparse_a
    if kind == "chain":
        assert sol.nnz_l == 0  # L^-1 would be a dense triangle: the dense factor is used
    else:
        assert sol.nnz_l > 0, "sparse factor expected"
    r1 = rng.standard_normal(prob.nU)
    r2 = rng.standard_normal(prob.m)
    x, y = sol.affine_project(torch.as_tensor(r1, device="cuda"), torch.as_tensor(r2, device="cuda"))
    xo, yo = O.KKT(prob, O.Decomposition(prob)).solve(r1, r2)
    assert _rel(y.cpu().numpy(), yo) <= 1e-10
    assert _rel(x.cpu().numpy(), xo) <= 1e-10
    # and the solve from it: 30 ADMM iterations against the oracle
    ref = O.Oracle(prob).solve("primal", rho=1.0, max_iter=30)
    st = sol.new_state("primal")
    sol.solve(st, form="primal", tol=0.0, max_iter=30, check_every=10)
    assert _rel(st["x"].cpu().numpy(), ref.x) <= 1e-4
    sol.close()


def test_sparse_factor_detects_dependent_rows(torch):
    base = synth.c3_small()
    rows = _graphs(base.nU, 40, "independent", np.random.default_rng(3))
    rows[7] = list(rows[3])
    prob = _with_rows(base, rows, seed=4)
    prob.A_val[prob.A_ptr[7]:prob.A_ptr[8]] = 2.0 * prob.A_val[prob.A_ptr[3]:prob.A_ptr[4]]
    with pytest.raises(cdcs.CdcsError) as e:
        cdcs.Solver(prob)
    assert e.value.status == cdcs.E_RANK


def test_uneven_workload_takes_the_sparse_factor(torch):
    prob = synth.c3()
    sol = cdcs.Solver(prob)
    assert sol.sparse_a and sol.nnz_l > 0 and sol.sparse_factor
    assert sol.nnz_l < 4 * sol.m  # M is nearly diagonal
    sol.close()
