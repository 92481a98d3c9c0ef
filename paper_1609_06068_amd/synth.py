"""Seeded synthetic SDP instances with chordal aggregate sparsity.

This module only *draws inputs*: a sparsity pattern with its maximal cliques,
constraint matrices A_1..A_m, a right-hand side b and a cost C, in the standard
primal/dual forms of Section I of the paper (operators A(X) = [<A_i, X>] and
A*(y) = sum_i A_i y_i).  It contains none of the ADMM arithmetic; both the CPU
oracle and the GPU library consume the same arrays.

Storage convention (shared input format, not an algorithm):
  * the pattern is a list of distinct lower-triangular entries (ei[e], ej[e])
    with ei >= ej, diagonal included; "entry e" means that list position;
  * every symmetric n x n matrix on the pattern is stored by its value on each
    entry (a matrix value, not a weighted one);
  * A is an m x nU array (dense on the pattern) or a CSR over entries;
  * cliques are a CSR (clique_ptr, clique_vert) with vertices sorted in the
    natural order (Section II-B: E_k lists the vertices of C_k in increasing
    order).

Instances are made strictly feasible by construction: b = A(X0) with X0 a
Gram matrix, and C = A*(y0) + Z0 with Z0 a sum of clique-supported PSD blocks
(Agler's form, Section II-C).  All draws use numpy PCG64 with the given seed.
A is rounded to FP32-representable values so that a FP32 copy of A is exact.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


CONE_FREE, CONE_ORTHANT, CONE_SOC = 0, 1, 2


@dataclass
class Problem:
    n: int
    ei: np.ndarray          # int32 [nU]   row index of entry e (ei >= ej)
    ej: np.ndarray          # int32 [nU]   column index of entry e
    clique_ptr: np.ndarray  # int64 [p+1]
    clique_vert: np.ndarray  # int32 [sum s_k], sorted within each clique
    b: np.ndarray           # float64 [m]
    c: np.ndarray           # float64 [nU]  values of C on the entries
    A: np.ndarray | None = None      # float64 [m, nU] dense-on-pattern A
    A_ptr: np.ndarray | None = None  # int64 [m+1]   CSR alternative
    A_idx: np.ndarray | None = None  # int32 [nnzA]  entry indices
    A_val: np.ndarray | None = None  # float64 [nnzA]
    meta: dict = field(default_factory=dict)
    # vector cones (CDCS's cone types besides PSD): cone q covers the diagonal
    # entries of vertices cone_vert[cone_ptr[q]:cone_ptr[q+1]]; cone_kind[q] is
    # CONE_FREE, CONE_ORTHANT or CONE_SOC (second-order cone, first vertex t)
    cone_kind: np.ndarray | None = None  # int32 [ncones]
    cone_ptr: np.ndarray | None = None   # int64 [ncones+1]
    cone_vert: np.ndarray | None = None  # int32 [sum of cone sizes]

    @property
    def ncones(self) -> int:
        return 0 if self.cone_kind is None else int(self.cone_kind.shape[0])

    def cone(self, q: int) -> np.ndarray:
        return self.cone_vert[self.cone_ptr[q]:self.cone_ptr[q + 1]]

    @property
    def nU(self) -> int:
        return int(self.ei.shape[0])

    @property
    def m(self) -> int:
        return int(self.b.shape[0])

    @property
    def p(self) -> int:
        return int(self.clique_ptr.shape[0] - 1)

    def clique(self, k: int) -> np.ndarray:
        return self.clique_vert[self.clique_ptr[k]:self.clique_ptr[k + 1]]

    def clique_sizes(self) -> np.ndarray:
        return np.diff(self.clique_ptr).astype(np.int64)

    def A_dense(self) -> np.ndarray:
        """A as an m x nU array (materialises a CSR A)."""
        if self.A is not None:
            return self.A
        out = np.zeros((self.m, self.nU))
        for i in range(self.m):
            lo, hi = self.A_ptr[i], self.A_ptr[i + 1]
            np.add.at(out[i], self.A_idx[lo:hi], self.A_val[lo:hi])
        return out


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _f32(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _entry_lookup(n: int, ei: np.ndarray, ej: np.ndarray):
    """Sorted keys for (i, j) -> entry position lookups (input bookkeeping)."""
    key = ei.astype(np.int64) * n + ej.astype(np.int64)
    order = np.argsort(key, kind="stable")
    return key[order], order


def _find_entries(n, lookup, ii, jj):
    skey, order = lookup
    hi = np.maximum(ii, jj).astype(np.int64)
    lo = np.minimum(ii, jj).astype(np.int64)
    q = hi * n + lo
    pos = np.searchsorted(skey, q)
    if np.any(pos >= skey.shape[0]) or np.any(skey[np.minimum(pos, skey.shape[0] - 1)] != q):
        raise ValueError("pair not in pattern")
    return order[pos]


def _pattern_from_cliques(n: int, cliques: list[np.ndarray]):
    """Lower-triangular entries of the union of C_k x C_k, clique-major.

    Entries first met in clique k are listed with clique k, in the clique's
    packed lower-triangular (row-major) order; this keeps each clique's private
    entries contiguous.
    """
    seen = {}
    ei, ej = [], []
    for cl in cliques:
        s = cl.shape[0]
        for a in range(s):
            va = int(cl[a])
            for bb in range(a + 1):
                vb = int(cl[bb])
                key = (va, vb)
                if key not in seen:
                    seen[key] = len(ei)
                    ei.append(va)
                    ej.append(vb)
    return np.asarray(ei, dtype=np.int32), np.asarray(ej, dtype=np.int32)


def _block_arrow_pattern(l: int, d: int, h: int):
    """Block-arrow pattern (Section V-A, Fig. 2): l diagonal blocks of size d
    plus an arrow head of size h.  Cliques C_i = B_i U H.  Entries are listed
    clique by clique (rows of the clique-local lower triangle that touch B_i),
    then the head x head entries once at the end."""
    n = l * d + h
    head = np.arange(l * d, n, dtype=np.int32)
    cliques = [np.concatenate([np.arange(i * d, (i + 1) * d, dtype=np.int32), head]) for i in range(l)]
    s = d + h
    # clique-local packed lower-tri rows a, columns b <= a with b < d
    loc_a, loc_b = [], []
    for a in range(s):
        for bb in range(min(a, d - 1) + 1):
            loc_a.append(a)
            loc_b.append(bb)
    loc_a = np.asarray(loc_a)
    loc_b = np.asarray(loc_b)
    ei = np.concatenate([cl[loc_a] for cl in cliques] + [head[np.tril_indices(h)[0]]]) if h > 0 else \
        np.concatenate([cl[loc_a] for cl in cliques])
    ej = np.concatenate([cl[loc_b] for cl in cliques] + [head[np.tril_indices(h)[1]]]) if h > 0 else \
        np.concatenate([cl[loc_b] for cl in cliques])
    return n, cliques, ei.astype(np.int32), ej.astype(np.int32)


def _finish(n, cliques, ei, ej, A_rows, rng, m, gram_rank=None, meta=None, A_sparse=None):
    """Draw X0, y0, Z0 and set b = A(X0), C = A*(y0) + Z0."""
    nU = ei.shape[0]
    w = np.where(ei == ej, 1.0, 2.0)
    lookup = _entry_lookup(n, ei, ej)
    # X0 = G G^T / r on the pattern entries (G is n x r)
    r = n if gram_rank is None else gram_rank
    G = rng.standard_normal((n, r))
    x0 = np.empty(nU)
    step = max(1, (1 << 24) // max(r, 1))
    for lo in range(0, nU, step):
        hi = min(nU, lo + step)
        x0[lo:hi] = np.einsum("ij,ij->i", G[ei[lo:hi]], G[ej[lo:hi]]) / r
    if gram_rank is not None:
        x0[ei == ej] += 1.0  # X0 = G G^T / r + I keeps a low-rank Gram PD
    del G
    y0 = rng.standard_normal(m)
    # Z0 = sum_k E_k^T (R_k R_k^T / s_k) E_k  (Agler form, Theorem 2)
    z0 = np.zeros(nU)
    for cl in cliques:
        s = cl.shape[0]
        R = rng.standard_normal((s, s))
        Zk = R @ R.T / s
        ia, ib = np.tril_indices(s)
        idx = _find_entries(n, lookup, cl[ia], cl[ib])
        np.add.at(z0, idx, Zk[ia, ib])
    if A_sparse is None:
        A = A_rows
        b = A @ (w * x0)             # <A_i, X0> = sum_e w_e A_ie X0_e
        c = A.T @ y0 + z0            # (A*(y0))_e = sum_i A_ie y0_i
    else:
        ptr, idx, val = A_sparse
        b = np.zeros(m)
        c = z0.copy()
        for i in range(m):
            lo, hi = ptr[i], ptr[i + 1]
            b[i] = np.dot(val[lo:hi], w[idx[lo:hi]] * x0[idx[lo:hi]])
            np.add.at(c, idx[lo:hi], val[lo:hi] * y0[i])
        A = None
    clique_ptr = np.zeros(len(cliques) + 1, dtype=np.int64)
    clique_ptr[1:] = np.cumsum([cl.shape[0] for cl in cliques])
    clique_vert = np.concatenate(cliques).astype(np.int32)
    prob = Problem(n=n, ei=ei, ej=ej, clique_ptr=clique_ptr, clique_vert=clique_vert,
                   b=b, c=c, A=A, meta=dict(meta or {}))
    if A_sparse is not None:
        prob.A_ptr, prob.A_idx, prob.A_val = A_sparse
    prob.meta.update({"x0": x0, "y0": y0, "z0": z0})
    return prob


def _symmetrised_normal(rng, m, ei, ej):
    """A_i = (R + R^T)/2 restricted to the pattern, R ~ N(0, 1) entrywise."""
    nU = ei.shape[0]
    out = np.empty((m, nU))
    diag = ei == ej
    chunk = max(1, (1 << 24) // max(nU, 1))
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        r1 = rng.standard_normal((hi - lo, nU))
        r2 = rng.standard_normal((hi - lo, nU))
        out[lo:hi] = np.where(diag[None, :], r1, 0.5 * (r1 + r2))
    return _f32(out)


def block_arrow(l: int, d: int, h: int, m: int, seed: int) -> Problem:
    """Random block-arrow SDP (stand-in for the block-arrow benchmark of
    Section V-A): each A_i is a symmetrised N(0,1) matrix on the whole
    pattern, b = A(X0) with X0 = G G^T / n, C = A*(y0) + Z0."""
    rng = _rng(seed)
    n, cliques, ei, ej = _block_arrow_pattern(l, d, h)
    A = _symmetrised_normal(rng, m, ei, ej)
    return _finish(n, cliques, ei, ej, A, rng, m,
                   meta={"kind": "block_arrow", "l": l, "d": d, "h": h, "seed": seed})


def config_seed(config: int, instance: int = 0) -> int:
    return 1000 * config + instance


# The five workloads of the benchmark suite, by name.
C1 = dict(l=10, d=10, h=5, m=50)        # plain FP64 parity anchor, n = 105
C2 = dict(l=200, d=20, h=10, m=2000)    # headline: n = 4010, 200 cliques of 30
C5 = dict(l=100, d=16, h=8, m=800)      # differentiation workload
# uneven batching: 3000 cliques of 4..96 vertices, separators of 1..8, sparse A
C3 = dict(p=3000, smin=4, smax=96, omax=8, m=8000, nnz_row=20)
# the same generator at a size the oracle solves in seconds
C3_SMALL = dict(p=40, smin=4, smax=96, omax=8, m=150, nnz_row=20)


def c1(instance: int = 0) -> Problem:
    return block_arrow(seed=config_seed(1, instance), **C1)


def c2(instance: int = 0) -> Problem:
    return block_arrow(seed=config_seed(2, instance), **C2)


def c3(instance: int = 0) -> Problem:
    return peo_chordal(seed=config_seed(3, instance), **C3)


def c3_small(instance: int = 0) -> Problem:
    return peo_chordal(seed=config_seed(3, 100 + instance), **C3_SMALL)


# large cliques (the sizes of Table I's largest, 322/323): 40 cliques of
# 127..330 vertices, projected by the matrix sign function
C3_BIG = dict(p=40, smin=127, smax=330, omax=8, m=2000, nnz_row=20)


def c3_big(instance: int = 0) -> Problem:
    return peo_chordal(seed=config_seed(3, 200 + instance), **C3_BIG)


def c5(instance: int = 0) -> Problem:
    return block_arrow(seed=config_seed(5, instance), **C5)


def random_symmetric(k: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Symmetric k x k test matrix with N(0,1) entries (for projection tests)."""
    rng = _rng(seed)
    R = rng.standard_normal((k, k)) * scale
    return (R + R.T) / 2


def clique_batch(sizes, seed: int):
    """Packed batch of random symmetric clique matrices (float64, full k x k
    row-major per clique), plus offsets."""
    rng = _rng(seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.zeros(sizes.shape[0] + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes * sizes)
    W = np.empty(off[-1])
    for t, k in enumerate(sizes):
        R = rng.standard_normal((k, k))
        W[off[t]:off[t + 1]] = ((R + R.T) / 2).ravel()
    return sizes, off, W


def trace_problem(n_blocks: int, d: int, h: int, seed: int) -> Problem:
    """min <C, X> s.t. tr X = 1, X PSD, on a block-arrow pattern.
    The optimum is lambda_min(C) (Rayleigh), a closed form for tests."""
    rng = _rng(seed)
    n, cliques, ei, ej = _block_arrow_pattern(n_blocks, d, h)
    nU = ei.shape[0]
    A = np.where(ei == ej, 1.0, 0.0)[None, :]
    b = np.array([1.0])
    R = rng.standard_normal((n, n))
    Cfull = (R + R.T) / 2
    c = Cfull[ei, ej].copy()
    clique_ptr = np.zeros(len(cliques) + 1, dtype=np.int64)
    clique_ptr[1:] = np.cumsum([cl.shape[0] for cl in cliques])
    return Problem(n=n, ei=ei, ej=ej, clique_ptr=clique_ptr,
                   clique_vert=np.concatenate(cliques).astype(np.int32),
                   b=b, c=c, A=A, meta={"kind": "trace", "seed": seed})


def lambda_max_problem(k: int, seed: int) -> Problem:
    """Dual form max <b, y> s.t. A*(y) + Z = C, Z PSD, with m = 1, A_1 = -I,
    b = -1, C = -M for a random symmetric M on the full k x k pattern (one
    clique).  Then y = -t and the constraint reads t I - M PSD, so the optimal
    <b, y> = -min t = -lambda_max(M)."""
    rng = _rng(seed)
    R = rng.standard_normal((k, k))
    Mfull = (R + R.T) / 2
    ei, ej = np.tril_indices(k)
    ei = ei.astype(np.int32)
    ej = ej.astype(np.int32)
    A = np.where(ei == ej, -1.0, 0.0)[None, :]
    cl = np.arange(k, dtype=np.int32)
    return Problem(n=k, ei=ei, ej=ej, clique_ptr=np.array([0, k], dtype=np.int64),
                   clique_vert=cl, b=np.array([-1.0]), c=-Mfull[ei, ej].copy(), A=A,
                   meta={"kind": "lambda_max", "M": Mfull})


def with_cliques(prob: Problem, cliques: list[np.ndarray]) -> Problem:
    """The same SDP data posed over a different clique cover of a pattern that
    contains the original one (entries absent from the original pattern get
    zero data).  Used to compare the decomposed and undecomposed problems."""
    n = prob.n
    ei, ej = _pattern_from_cliques(n, cliques)
    lookup = _entry_lookup(n, ei, ej)
    pos = _find_entries(n, lookup, prob.ei, prob.ej)
    nU = ei.shape[0]
    c = np.zeros(nU)
    c[pos] = prob.c
    A = np.zeros((prob.m, nU))
    A[:, pos] = prob.A_dense()
    clique_ptr = np.zeros(len(cliques) + 1, dtype=np.int64)
    clique_ptr[1:] = np.cumsum([cl.shape[0] for cl in cliques])
    return Problem(n=n, ei=ei, ej=ej, clique_ptr=clique_ptr,
                   clique_vert=np.concatenate(cliques).astype(np.int32),
                   b=prob.b.copy(), c=c, A=A, meta=dict(prob.meta, recliqued=True))


def block_trace_problem(l: int, d: int, seed: int) -> Problem:
    """Block-diagonal pattern (block-arrow with h = 0) with one trace
    constraint per block: min <C, X> s.t. tr X_b = 1 for each block, X PSD.
    The problem decouples; the optimum is sum_b lambda_min(C_b)."""
    rng = _rng(seed)
    n, cliques, ei, ej = _block_arrow_pattern(l, d, 0)
    nU = ei.shape[0]
    A = np.zeros((l, nU))
    blk = ei // d
    A[blk, np.arange(nU)] = np.where(ei == ej, 1.0, 0.0)
    R = rng.standard_normal((n, n))
    Cfull = (R + R.T) / 2
    clique_ptr = np.zeros(len(cliques) + 1, dtype=np.int64)
    clique_ptr[1:] = np.cumsum([cl.shape[0] for cl in cliques])
    return Problem(n=n, ei=ei, ej=ej, clique_ptr=clique_ptr,
                   clique_vert=np.concatenate(cliques).astype(np.int32),
                   b=np.ones(l), c=Cfull[ei, ej].copy(), A=A,
                   meta={"kind": "block_trace", "C": Cfull, "l": l, "d": d})


def small_chordal(n: int, p: int, smax: int, m: int, seed: int) -> Problem:
    """Small random chordal instance built from a clique tree: clique k > 0
    takes a separator from a random earlier clique and adds new vertices.
    Dense symmetrised N(0,1) constraints on the pattern; vertex labels are
    randomly permuted.  n is the resulting vertex count (argument is a cap)."""
    rng = _rng(seed)
    cliques = []
    nv = 0
    for k in range(p):
        s = int(rng.integers(2, smax + 1))
        if k == 0:
            cl = list(range(nv, nv + s))
            nv += s
        else:
            par = cliques[int(rng.integers(0, k))]
            o = int(rng.integers(1, min(len(par), s - 1) + 1))
            sep = list(rng.choice(par, size=o, replace=False))
            new = list(range(nv, nv + s - o))
            nv += s - o
            cl = sep + new
        cliques.append(sorted(int(v) for v in cl))
        if nv >= n:
            break
    perm = rng.permutation(nv)
    cliques = [np.sort(perm[np.asarray(cl)]).astype(np.int32) for cl in cliques]
    ei, ej = _pattern_from_cliques(nv, cliques)
    A = _symmetrised_normal(rng, m, ei, ej)
    return _finish(nv, cliques, ei, ej, A, rng, m, meta={"kind": "small_chordal", "seed": seed})


def random_sparse(n: int, extra: int, m: int, seed: int) -> Problem:
    """SDP on a pattern that is not chordal and comes without cliques: the
    cycle 0-1-...-(n-1)-0 (chordless for n >= 4) plus `extra` random chords,
    diagonal included.  Dense symmetrised N(0,1) constraints on the pattern,
    b = A(X0) with X0 = G G^T / n + I, C = A*(y0) + Z0 with Z0 diagonally
    dominant on the pattern (so positive definite): strictly feasible.
    clique_ptr is None (the setup computes a chordal extension)."""
    rng = _rng(seed)
    edges = {(max(i, (i + 1) % n), min(i, (i + 1) % n)) for i in range(n)}
    while len(edges) < n + extra:
        i, j = (int(v) for v in rng.integers(0, n, size=2))
        if i != j:
            edges.add((max(i, j), min(i, j)))
    ent = sorted(edges) + [(i, i) for i in range(n)]
    ei = np.array([e[0] for e in ent], dtype=np.int32)
    ej = np.array([e[1] for e in ent], dtype=np.int32)
    nU = ei.shape[0]
    w = np.where(ei == ej, 1.0, 2.0)
    A = _symmetrised_normal(rng, m, ei, ej)
    G = rng.standard_normal((n, n))
    x0 = np.einsum("ij,ij->i", G[ei], G[ej]) / n + (ei == ej)
    z0 = np.where(ei == ej, 0.0, 0.5 * rng.standard_normal(nU))
    rowsum = np.zeros(n)
    np.add.at(rowsum, ei, np.abs(z0))
    np.add.at(rowsum, ej, np.abs(z0))
    z0[ei == ej] = 1.0 + rowsum[ei[ei == ej]]
    y0 = rng.standard_normal(m)
    return Problem(n=n, ei=ei, ej=ej, clique_ptr=None, clique_vert=None, b=A @ (w * x0), c=A.T @ y0 + z0, A=A,
                   meta={"kind": "random_sparse", "seed": seed, "x0": x0, "y0": y0, "z0": z0})


def _peo_cliques(p: int, smin: int, smax: int, omax: int, rng):
    """Clique tree grown in perfect-elimination order: clique 0 has s_0 fresh
    vertices; clique k > 0 draws s_k, a uniform parent j < k and a separator of
    min(U{1..omax}, s_k - 1, s_j - 1) vertices of C_j, then adds s_k - |sep|
    fresh vertices.  Every clique has a fresh vertex and no separator covers a
    whole clique, so the cliques are the maximal cliques of the chordal union
    (running-intersection property of a clique tree, Section II-B)."""
    sizes = rng.integers(smin, smax + 1, size=p)
    cliques, fresh_from, nv = [], [], 0
    for k in range(p):
        s = int(sizes[k])
        if k == 0:
            sep = np.empty(0, dtype=np.int64)
        else:
            par = cliques[int(rng.integers(0, k))]
            o = min(int(rng.integers(1, omax + 1)), s - 1, par.shape[0] - 1)
            sep = rng.choice(par, size=o, replace=False)
        new = np.arange(nv, nv + s - sep.shape[0], dtype=np.int64)
        nv += new.shape[0]
        cliques.append(np.concatenate([sep, new]))
        fresh_from.append(sep.shape[0])
    return cliques, fresh_from, nv


def peo_chordal(p: int, smin: int, smax: int, omax: int, m: int, nnz_row: int, seed: int,
                gram_rank: int = 64) -> Problem:
    """Random chordal SDP with uneven cliques (stand-in for the SDPLIB-like
    uneven-clique workloads of Section V-B).  Pattern: union of C_k x C_k over
    the clique tree of _peo_cliques, vertex labels randomly permuted.  Each A_i
    has nnz_row distinct pattern entries chosen uniformly with N(0,1) values
    (an off-diagonal entry stands for both mirrored positions), stored as CSR.
    b = A(X0) with X0 = G G^T / r + I (G is n x r), C = A*(y0) + Z0."""
    rng = _rng(seed)
    cliques, fresh_from, nv = _peo_cliques(p, smin, smax, omax, rng)
    perm = rng.permutation(nv).astype(np.int64)
    # Entries of clique k not met before are the pairs with a fresh vertex.
    ei_l, ej_l, sorted_cl = [], [], []
    for cl, f in zip(cliques, fresh_from):
        lab = perm[cl]
        s = lab.shape[0]
        ia, ib = np.tril_indices(s)
        keep = ia >= f  # local index a is fresh (fresh vertices come last)
        va, vb = lab[ia[keep]], lab[ib[keep]]
        ei_l.append(np.maximum(va, vb))
        ej_l.append(np.minimum(va, vb))
        sorted_cl.append(np.sort(lab).astype(np.int32))
    ei = np.concatenate(ei_l).astype(np.int32)
    ej = np.concatenate(ej_l).astype(np.int32)
    nU = ei.shape[0]
    ptr = np.arange(m + 1, dtype=np.int64) * nnz_row
    idx = np.empty(m * nnz_row, dtype=np.int32)
    for i in range(m):
        idx[i * nnz_row:(i + 1) * nnz_row] = np.sort(rng.choice(nU, size=nnz_row, replace=False))
    val = _f32(rng.standard_normal(m * nnz_row))
    return _finish(nv, sorted_cl, ei, ej, None, rng, m, gram_rank=gram_rank,
                   meta={"kind": "peo_chordal", "p": p, "smin": smin, "smax": smax, "omax": omax,
                         "nnz_row": nnz_row, "seed": seed},
                   A_sparse=(ptr, idx, val))


def unit_directions(dim: int, count: int, seed: int) -> np.ndarray:
    """count random unit vectors in R^dim (rows), for directional derivatives."""
    rng = _rng(seed)
    D = rng.standard_normal((count, dim))
    return D / np.linalg.norm(D, axis=1, keepdims=True)


def c4_params(count: int = 512, seed: int = 4000):
    """Per-instance (l, d, h, m) of the many-SDP workload: l in 5..40,
    d in 8..32, h in 2..12 drawn uniformly, m = 5 l."""
    rng = _rng(seed)
    out = []
    for _ in range(count):
        l = int(rng.integers(5, 41))
        d = int(rng.integers(8, 33))
        h = int(rng.integers(2, 13))
        out.append((l, d, h, 5 * l))
    return out


def c4(count: int = 512, first: int = 0):
    """The many-SDP workload: `count` independent block-arrow SDPs (instances
    first..first+count-1 of the seeded sequence), seed 1000*4 + instance."""
    params = c4_params(first + count)
    return [block_arrow(l, d, h, m, seed=config_seed(4, first + i))
            for i, (l, d, h, m) in enumerate(params[first:first + count])]


# --------------------------------------------------------------------------
# Vector cones (free, nonnegative orthant, second-order) beside the PSD
# cliques, and instances with a known status (infeasible / unbounded)
# --------------------------------------------------------------------------

def _append_vector_vertices(ei, ej, n0, kinds_sizes):
    """Diagonal entries of fresh vertices n0, n0+1, ... for each vector cone
    (kind, size); returns the new entry arrays, vertex count and the cone CSR."""
    kinds, ptr, vert = [], [0], []
    v = n0
    for kind, size in kinds_sizes:
        kinds.append(kind)
        vert.extend(range(v, v + size))
        v += size
        ptr.append(len(vert))
    nv = v - n0
    newv = np.arange(n0, v, dtype=np.int32)
    ei = np.concatenate([ei, newv]).astype(np.int32)
    ej = np.concatenate([ej, newv]).astype(np.int32)
    return (ei, ej, v, np.asarray(kinds, dtype=np.int32), np.asarray(ptr, dtype=np.int64),
            np.asarray(vert, dtype=np.int32), nv)


def _interior_vector_point(rng, kind, size, dual=False):
    """A point in the interior of a vector cone (or of its dual cone; the free
    cone's dual is {0})."""
    if kind == CONE_FREE:
        return np.zeros(size) if dual else rng.standard_normal(size)
    if kind == CONE_ORTHANT:
        return rng.uniform(0.5, 1.5, size)
    z = rng.standard_normal(size - 1)
    return np.concatenate([[np.linalg.norm(z) + rng.uniform(0.5, 1.5)], z])


def mixed_cones(l: int, d: int, h: int, m: int, cones, seed: int) -> Problem:
    """Block-arrow SDP part (as block_arrow) plus vector cones `cones`, a list
    of (kind, size), on fresh vertices (their diagonal entries).  Dense N(0,1)
    constraints over every entry (symmetrised on the PSD part); b = A(x0) and
    c = A*(y0) + z0 with x0 and z0 interior to the cone and its dual cone, so
    the instance is strictly feasible (and a free variable's dual slack is 0).
    l = 0 gives a problem with vector cones only (no cliques)."""
    rng = _rng(seed)
    if l > 0:
        n0, cliques, ei, ej = _block_arrow_pattern(l, d, h)
    else:
        n0, cliques, ei, ej = 0, [], np.empty(0, np.int32), np.empty(0, np.int32)
    npsd = ei.shape[0]
    ei, ej, n, kinds, cptr, cvert, nv = _append_vector_vertices(ei, ej, n0, cones)
    nU = ei.shape[0]
    w = np.where(ei == ej, 1.0, 2.0)
    A = _symmetrised_normal(rng, m, ei, ej)
    x0 = np.zeros(nU)
    z0 = np.zeros(nU)
    if l > 0:
        G = rng.standard_normal((n0, n0))
        x0[:npsd] = np.einsum("ij,ij->i", G[ei[:npsd]], G[ej[:npsd]]) / n0
        lookup = _entry_lookup(n, ei, ej)
        for cl in cliques:
            s = cl.shape[0]
            R = rng.standard_normal((s, s))
            Zk = R @ R.T / s
            ia, ib = np.tril_indices(s)
            np.add.at(z0, _find_entries(n, lookup, cl[ia], cl[ib]), Zk[ia, ib])
    # vector-cone vertices own the entries npsd + (vertex - n0)
    for q, kind in enumerate(kinds):
        ent = npsd + (cvert[cptr[q]:cptr[q + 1]] - n0)
        x0[ent] = _interior_vector_point(rng, int(kind), ent.shape[0])
        z0[ent] = _interior_vector_point(rng, int(kind), ent.shape[0], dual=True)
    y0 = rng.standard_normal(m)
    clique_ptr = np.zeros(len(cliques) + 1, dtype=np.int64)
    clique_ptr[1:] = np.cumsum([cl.shape[0] for cl in cliques])
    clique_vert = np.concatenate(cliques).astype(np.int32) if cliques else np.empty(0, np.int32)
    return Problem(n=n, ei=ei, ej=ej, clique_ptr=clique_ptr, clique_vert=clique_vert, b=A @ (w * x0),
                   c=A.T @ y0 + z0, A=A, cone_kind=kinds, cone_ptr=cptr, cone_vert=cvert,
                   meta={"kind": "mixed_cones", "l": l, "d": d, "h": h, "seed": seed, "x0": x0, "y0": y0,
                         "z0": z0})


def mixed_small(seed: int = 7001) -> Problem:
    """Small mixed-cone instance: block-arrow l=6, d=6, h=3 and a free cone
    of 5, an orthant of 12 and second-order cones of 6 and 9, m = 40."""
    return mixed_cones(6, 6, 3, 40, [(CONE_FREE, 5), (CONE_ORTHANT, 12), (CONE_SOC, 6), (CONE_SOC, 9)], seed)


def lp(nvar: int, m: int, seed: int, status: str = "feasible") -> Problem:
    """Linear program min c^T x, A x = b, x >= 0 (one orthant cone, no
    cliques).  status "feasible": strictly feasible primal and dual;
    "infeasible": A^T y1 <= -0.1 componentwise and b^T y1 > 0 for a drawn y1
    (Farkas: no x >= 0 has A x = b); "unbounded": a drawn ray r > 0 with
    A r = 0 and c^T r = -1, and a feasible x0 > 0 (the objective is unbounded
    below)."""
    rng = _rng(seed)
    A = rng.standard_normal((m, nvar))
    x0 = rng.uniform(0.5, 1.5, nvar)
    y0 = rng.standard_normal(m)
    z0 = rng.uniform(0.5, 1.5, nvar)
    meta = {"kind": "lp", "status": status, "seed": seed}
    if status == "infeasible":
        y1 = rng.standard_normal(m)
        v = np.maximum(A.T @ y1, 0.0) + 0.1
        A = A - np.outer(y1, v) / (y1 @ y1)
        A = _f32(A)
        b = rng.standard_normal(m)
        b = b + y1 * (1.0 + abs(b @ y1)) / (y1 @ y1)
        c = A.T @ y0 + z0
        meta["y1"] = y1
    elif status == "unbounded":
        r = rng.uniform(0.5, 1.5, nvar)
        A = A - np.outer(A @ r, r) / (r @ r)
        A = _f32(A)
        b = A @ x0
        c = rng.standard_normal(nvar)
        c = c - r * (c @ r + 1.0) / (r @ r)
        meta["ray"] = r
    else:
        A = _f32(A)
        b = A @ x0
        c = A.T @ y0 + z0
    v = np.arange(nvar, dtype=np.int32)
    return Problem(n=nvar, ei=v.copy(), ej=v.copy(), clique_ptr=np.zeros(1, np.int64),
                   clique_vert=np.empty(0, np.int32), b=b, c=c, A=A,
                   cone_kind=np.array([CONE_ORTHANT], np.int32), cone_ptr=np.array([0, nvar], np.int64),
                   cone_vert=v.copy(), meta={**meta, "x0": x0, "y0": y0, "z0": z0})


def socp_norm(a: np.ndarray) -> Problem:
    """min t s.t. z = a, (t, z) in the second-order cone: the optimum is
    ||a|| (primal t = ||a||, z = a; dual y = a / ||a||)."""
    q = a.shape[0]
    v = np.arange(q + 1, dtype=np.int32)
    A = np.zeros((q, q + 1))
    A[np.arange(q), np.arange(1, q + 1)] = 1.0
    c = np.zeros(q + 1)
    c[0] = 1.0
    return Problem(n=q + 1, ei=v.copy(), ej=v.copy(), clique_ptr=np.zeros(1, np.int64),
                   clique_vert=np.empty(0, np.int32), b=np.asarray(a, dtype=np.float64), c=c, A=A,
                   cone_kind=np.array([CONE_SOC], np.int32), cone_ptr=np.array([0, q + 1], np.int64),
                   cone_vert=v.copy(), meta={"kind": "socp_norm"})


def sdp_infeasible(seed: int = 7101) -> Problem:
    """The C1-shaped block-arrow SDP (l=10, d=10, h=5, m=50) with one more
    constraint trace(X) = -1, which no PSD X meets (primal infeasible)."""
    p = block_arrow(10, 10, 5, 50, seed)
    tr = np.where(p.ei == p.ej, 1.0, 0.0)
    A = np.vstack([p.A, tr[None, :]])
    b = np.concatenate([p.b, [-1.0]])
    out = Problem(**{**p.__dict__})
    out.A, out.b = A, b
    out.meta = {**p.meta, "kind": "sdp_infeasible"}
    return out


def sdp_unbounded(seed: int = 7102) -> Problem:
    """The C1-shaped block-arrow SDP with every constraint's coefficients on
    the diagonal entries of block 0's vertices (0..9) set to zero, C = -1 on
    those entries and C = A*(y0 / 20) + Z0 elsewhere: X0 + t D with D the
    identity on block 0's vertices stays feasible for every t >= 0 while
    <C, X> decreases without bound (dual infeasible).  The smaller y0 keeps
    the ray's cost (-10 for ||D||_F = sqrt(10)) a sizeable part of ||C||."""
    p = block_arrow(10, 10, 5, 50, seed)
    ray = np.nonzero((p.ei == p.ej) & (p.ei < 10))[0]
    A = p.A.copy()
    A[:, ray] = 0.0
    w = np.where(p.ei == p.ej, 1.0, 2.0)
    c = A.T @ (p.meta["y0"] / 20.0) + p.meta["z0"]
    c[ray] = -1.0
    out = Problem(**{**p.__dict__})
    out.A, out.b, out.c = A, A @ (w * p.meta["x0"]), c
    out.meta = {**p.meta, "kind": "sdp_unbounded", "ray_entries": ray}
    return out


def lp_sparse(nvar: int, m: int, nnz_row: int, seed: int, soc: int = 0, free: int = 0) -> Problem:
    """Strictly feasible conic program with a sparse A: an orthant of nvar,
    optionally a second-order cone of `soc` and a free cone of `free`
    variables (no cliques).  Each constraint has nnz_row distinct uniform
    variables with N(0,1) coefficients (FP32-representable, CSR); b = A x0,
    c = A^T y0 + z0 with x0, z0 interior (z0 = 0 on the free variables)."""
    rng = _rng(seed)
    cones = [(CONE_ORTHANT, nvar)] + ([(CONE_SOC, soc)] if soc else []) + ([(CONE_FREE, free)] if free else [])
    ei, ej, n, kinds, cptr, cvert, nv = _append_vector_vertices(np.empty(0, np.int32), np.empty(0, np.int32), 0,
                                                                cones)
    nU = ei.shape[0]
    ptr = np.arange(m + 1, dtype=np.int64) * nnz_row
    idx = np.empty(m * nnz_row, dtype=np.int32)
    for i in range(m):
        idx[i * nnz_row:(i + 1) * nnz_row] = np.sort(rng.choice(nU, size=nnz_row, replace=False))
    val = _f32(rng.standard_normal(m * nnz_row))
    x0 = np.empty(nU)
    z0 = np.empty(nU)
    for q, kind in enumerate(kinds):
        ent = np.arange(cptr[q], cptr[q + 1])
        x0[ent] = _interior_vector_point(rng, int(kind), ent.shape[0])
        z0[ent] = _interior_vector_point(rng, int(kind), ent.shape[0], dual=True)
    y0 = rng.standard_normal(m)
    b = np.add.reduceat(val * x0[idx], ptr[:-1]) if m > 0 else np.empty(0)
    c = z0.copy()
    np.add.at(c, idx, val * np.repeat(y0, nnz_row))
    return Problem(n=n, ei=ei, ej=ej, clique_ptr=np.zeros(1, np.int64), clique_vert=np.empty(0, np.int32), b=b,
                   c=c, A=None, A_ptr=ptr, A_idx=idx, A_val=val, cone_kind=kinds, cone_ptr=cptr, cone_vert=cvert,
                   meta={"kind": "lp_sparse", "seed": seed, "x0": x0, "y0": y0, "z0": z0})


# a large conic program with vector cones only: 4 M orthant variables, a
# second-order cone of 100,000 and 10,000 free variables, m = 8,000 sparse
# constraints of 20 coefficients (few constraints share a variable, so the
# factor stays sparse)
LP_BIG = dict(nvar=4_000_000, m=8_000, nnz_row=20, soc=100_000, free=10_000)


def lp_big(instance: int = 0) -> Problem:
    return lp_sparse(seed=config_seed(6, instance), **LP_BIG)
