"""Chordal extension and maximal-clique extraction (host code of the library,
no GPU): cdcs_chordal_extension (paper Sec. II-A, Definition 1) checked
against independent characterisations on small graphs:
  * the extended graph is chordal: repeatedly deleting simplicial vertices
    (vertices whose neighbours form a clique) empties it (Dirac / Fulkerson-
    Gross);
  * it contains the pattern, and a chordal pattern gets no fill;
  * the returned cliques are exactly the maximal cliques of the extended
    graph (brute-force Bron-Kerbosch enumeration);
  * a chordless cycle of length n needs n - 3 fill edges, which minimum-degree
    elimination attains;
  * malformed patterns are rejected.
"""
import itertools

import numpy as np
import pytest

from paper_1609_06068_amd import cdcs, synth


def _adj(n, ei, ej):
    A = [set() for _ in range(n)]
    for i, j in zip(ei, ej):
        if i != j:
            A[int(i)].add(int(j))
            A[int(j)].add(int(i))
    return A


def _is_chordal(n, adj, verts):
    adj = {v: set(adj[v]) & verts for v in verts}
    left = set(verts)
    while left:
        simp = next((v for v in sorted(left)
                     if all(b in adj[a] for a, b in itertools.combinations(sorted(adj[v] & left), 2))), None)
        if simp is None:
            return False
        left.remove(simp)
    return True


def _maximal_cliques(adj, verts):
    out = []

    def bk(R, P, X):
        if not P and not X:
            out.append(frozenset(R))
            return
        for v in sorted(P):
            bk(R | {v}, P & adj[v], X & adj[v])
            P = P - {v}
            X = X | {v}

    bk(set(), set(verts), set())
    return set(out)


def _extend(n, ei, ej):
    fi, fj, cptr, cvert = cdcs.chordal_extension(n, ei, ej)
    cliques = [cvert[cptr[k]:cptr[k + 1]] for k in range(len(cptr) - 1)]
    return fi, fj, cliques


def _check(n, ei, ej):
    fi, fj, cliques = _extend(n, ei, ej)
    pat = set(zip(ei.tolist(), ej.tolist()))
    fill = list(zip(fi.tolist(), fj.tolist()))
    assert len(set(fill)) == len(fill) and not (set(fill) & pat)
    assert all(i >= j for i, j in fill)
    verts = {int(v) for v in np.concatenate([ei, ej])}
    adj = _adj(n, np.concatenate([ei, fi]), np.concatenate([ej, fj]))
    assert _is_chordal(n, adj, verts)
    for cl in cliques:
        assert np.all(np.diff(cl) > 0)
    got = {frozenset(int(v) for v in cl) for cl in cliques}
    assert len(got) == len(cliques)
    assert got == _maximal_cliques(adj, verts)
    # the union of C_k x C_k is exactly pattern + fill
    cover = {(max(a, b), min(a, b)) for cl in cliques for a in cl.tolist() for b in cl.tolist()}
    assert cover == pat | set(fill)
    return fill, cliques


def _cycle(n):
    ent = [(max(i, (i + 1) % n), min(i, (i + 1) % n)) for i in range(n)] + [(i, i) for i in range(n)]
    return np.array([e[0] for e in ent], np.int32), np.array([e[1] for e in ent], np.int32)


@pytest.mark.parametrize("n", [4, 5, 9, 20])
def test_chordless_cycle_gets_minimum_fill(n):
    ei, ej = _cycle(n)
    fill, cliques = _check(n, ei, ej)
    assert len(fill) == n - 3
    assert len(cliques) == n - 2 and all(len(c) == 3 for c in cliques)


@pytest.mark.parametrize("seed", range(6))
def test_random_patterns(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 13))
    prob = synth.random_sparse(n, extra=int(rng.integers(0, n)), m=3, seed=seed)
    _check(n, prob.ei, prob.ej)


def test_chordal_patterns_get_no_fill():
    for prob in (synth.c1(), synth.small_chordal(n=25, p=8, smax=6, m=3, seed=2)):
        fill, cliques = _check(prob.n, prob.ei, prob.ej)
        assert not fill
        given = {frozenset(int(v) for v in prob.clique(k)) for k in range(prob.p)}
        given = {g for g in given if not any(g < h for h in given)}  # a generator clique may lie in a later one
        assert {frozenset(int(v) for v in cl) for cl in cliques} == given


def test_uneven_clique_tree_at_scale():
    """The 3000-clique workload's pattern (chordal by construction): the
    extension finds no fill and exactly the generator's cliques."""
    prob = synth.c3()
    fi, _, cliques = _extend(prob.n, prob.ei, prob.ej)
    assert fi.shape[0] == 0 and len(cliques) == prob.p
    given = sorted(tuple(int(v) for v in prob.clique(k)) for k in range(prob.p))
    assert sorted(tuple(int(v) for v in cl) for cl in cliques) == given


def test_vertices_without_entries_and_isolated_diagonals():
    # vertex 3 has no entry at all; vertex 4 only its diagonal
    ei = np.array([1, 2, 2, 4, 0, 1, 2], np.int32)
    ej = np.array([0, 0, 1, 4, 0, 1, 2], np.int32)
    fill, cliques = _check(5, ei, ej)
    assert not fill
    assert sorted(tuple(int(v) for v in c) for c in cliques) == [(0, 1, 2), (4,)]


def test_malformed_patterns_are_rejected():
    with pytest.raises(cdcs.CdcsError) as e:
        cdcs.chordal_extension(3, np.array([1, 1], np.int32), np.array([0, 0], np.int32))
    assert e.value.status == cdcs.E_PATTERN
    with pytest.raises(cdcs.CdcsError) as e:
        cdcs.chordal_extension(3, np.array([0], np.int32), np.array([1], np.int32))
    assert e.value.status == cdcs.E_PATTERN
    with pytest.raises(cdcs.CdcsError) as e:
        cdcs.chordal_extension(3, np.array([5], np.int32), np.array([0], np.int32))
    assert e.value.status == cdcs.E_PATTERN
