"""The uneven-clique generator (clique tree in perfect-elimination order, sparse
A) and the oracle's sparse-A KKT solve.

The generator is checked against what defines a chordal pattern with the given
maximal cliques (a perfect elimination ordering exists, the cliques are
maximal, the clique tree has the running-intersection property); the oracle's
CSR branch of the KKT solve against the literal vec-form KKT system of
Sec. III-A solved by a dense library solve."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1609_06068_amd import synth


def _adjacency(prob):
    adj = [set() for _ in range(prob.n)]
    for i, j in zip(prob.ei.tolist(), prob.ej.tolist()):
        if i != j:
            adj[i].add(j)
            adj[j].add(i)
    return adj


def _mcs_order(adj):
    """Maximum cardinality search visit order (Tarjan and Yannakakis)."""
    n = len(adj)
    weight = [0] * n
    order, seen = [], [False] * n
    for _ in range(n):
        v = max((u for u in range(n) if not seen[u]), key=lambda u: weight[u])
        seen[v] = True
        order.append(v)
        for u in adj[v]:
            if not seen[u]:
                weight[u] += 1
    return order


def _is_chordal(adj, order):
    """The reverse MCS order is a perfect elimination ordering iff chordal."""
    pos = {v: t for t, v in enumerate(order)}
    for v in order:
        earlier = [u for u in adj[v] if pos[u] < pos[v]]
        if earlier:
            parent = max(earlier, key=lambda u: pos[u])
            if not set(earlier) - {parent} <= adj[parent]:
                return False
    return True


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_peo_pattern_is_chordal_with_maximal_cliques(seed):
    prob = synth.peo_chordal(p=12, smin=3, smax=9, omax=3, m=5, nnz_row=4, seed=seed)
    O.Decomposition(prob)  # every clique pair is a pattern entry, every entry covered
    adj = _adjacency(prob)
    order = _mcs_order(adj)
    assert _is_chordal(adj, order)
    cl = [set(prob.clique(k).tolist()) for k in range(prob.p)]
    for a in range(prob.p):
        for b in range(prob.p):
            assert a == b or not cl[a] <= cl[b]
    # every maximal clique of a chordal graph is {v} with its neighbours that
    # come later in the elimination ordering; each such set lies in a clique
    pos = {v: t for t, v in enumerate(order)}
    for v in range(prob.n):
        S = {v} | {u for u in adj[v] if pos[u] < pos[v]}
        assert any(S <= c for c in cl)
    # the pattern is exactly the union of C_k x C_k
    pairs = {(max(a, b), min(a, b)) for c in cl for a in c for b in c}
    assert pairs == set(zip(prob.ei.tolist(), prob.ej.tolist()))


def test_peo_clique_tree_running_intersection():
    prob = synth.peo_chordal(p=40, smin=4, smax=20, omax=8, m=5, nnz_row=4, seed=9)
    cl = [set(prob.clique(k).tolist()) for k in range(prob.p)]
    sizes = prob.clique_sizes()
    assert sizes.min() >= 4 and sizes.max() <= 20
    union = set(cl[0])
    for k in range(1, prob.p):
        sep = cl[k] & union
        assert 1 <= len(sep) <= 8
        assert any(sep <= cl[j] for j in range(k))   # separator inside one earlier clique
        assert len(cl[k] - union) >= 1                # a fresh vertex
        union |= cl[k]
    assert len(union) == prob.n


def test_peo_constraints_and_right_hand_side():
    prob = synth.peo_chordal(p=10, smin=4, smax=12, omax=4, m=30, nnz_row=7, seed=5)
    assert prob.A is None
    assert np.array_equal(np.diff(prob.A_ptr), np.full(prob.m, 7))
    for i in range(prob.m):
        row = prob.A_idx[prob.A_ptr[i]:prob.A_ptr[i + 1]]
        assert np.unique(row).shape[0] == 7 and row.min() >= 0 and row.max() < prob.nU
    assert np.array_equal(prob.A_val, prob.A_val.astype(np.float32).astype(np.float64))
    # b = A(X0) with <A_i, X0> = trace(A_i X0) on the full symmetric matrices
    n = prob.n
    A = prob.A_dense()
    X0 = np.zeros((n, n))
    X0[prob.ei, prob.ej] = prob.meta["x0"]
    X0[prob.ej, prob.ei] = prob.meta["x0"]
    for i in range(prob.m):
        Ai = np.zeros((n, n))
        Ai[prob.ei, prob.ej] = A[i]
        Ai[prob.ej, prob.ei] = A[i]
        assert np.isclose(prob.b[i], np.trace(Ai @ X0), rtol=1e-12, atol=1e-12)


def test_uneven_workload_shape():
    prob = synth.c3()
    sizes = prob.clique_sizes()
    assert prob.p == 3000 and prob.m == 8000
    assert sizes.min() >= 4 and sizes.max() <= 96 and abs(sizes.mean() - 50) < 2
    assert 1.2e5 < prob.n < 1.5e5
    assert prob.A_idx.shape[0] == 20 * 8000


def _vec_kkt(prob, r1, r2):
    """The KKT system [D A^T; A 0] of Sec. III-B.1 in literal vec form."""
    n = prob.n
    Dvec = np.zeros(n * n)
    for k in range(prob.p):
        c = prob.clique(k)
        for a in c:
            for b in c:
                Dvec[b * n + a] += 1.0
    on = np.flatnonzero(Dvec > 0)
    N = on.shape[0]
    A = prob.A_dense()
    Avec = np.zeros((prob.m, n * n))
    for e, (i, j) in enumerate(zip(prob.ei, prob.ej)):
        for (r, s) in {(i, j), (j, i)}:
            Avec[:, s * n + r] = A[:, e]
    K = np.zeros((N + prob.m, N + prob.m))
    K[:N, :N] = np.diag(Dvec[on])
    K[:N, N:] = Avec[:, on].T
    K[N:, :N] = Avec[:, on]
    R1 = np.zeros((n, n))
    R1[prob.ei, prob.ej] = r1
    R1[prob.ej, prob.ei] = r1
    sol = np.linalg.solve(K, np.concatenate([R1.reshape(-1, order="F")[on], r2]))
    xv = np.zeros(n * n)
    xv[on] = sol[:N]
    return xv, sol[N:]


def test_oracle_sparse_kkt_matches_vec_form():
    prob = synth.peo_chordal(p=5, smin=3, smax=6, omax=2, m=6, nnz_row=3, seed=13)
    kkt = O.KKT(prob, O.Decomposition(prob))
    assert not isinstance(kkt.A, np.ndarray)  # the CSR branch
    rng = np.random.default_rng(13)
    r1 = rng.standard_normal(prob.nU)
    r2 = rng.standard_normal(prob.m)
    xv, yv = _vec_kkt(prob, r1, r2)
    x, y = kkt.solve(r1, r2)
    n = prob.n
    for e, (i, j) in enumerate(zip(prob.ei, prob.ej)):
        assert np.isclose(x[e], xv[j * n + i], rtol=1e-10, atol=1e-10)
    assert np.allclose(y, yv, rtol=1e-10, atol=1e-10)
