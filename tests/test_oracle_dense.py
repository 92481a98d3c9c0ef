"""Pins for the oracle's dense kernels (CPU only).

The Jacobi eigensolver, the PSD-cone projection and the Cholesky factor are
checked against library routines (numpy.linalg), closed forms and the
invariants the projection must satisfy (Sec. III-B.2: P_k is the projection
onto the PSD cone)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1609_06068_amd import synth

SIZES = [1, 2, 3, 5, 8, 15, 24, 30, 41]


def _proj_eigh(W):
    lam, Q = np.linalg.eigh(W)
    return (Q * np.maximum(lam, 0)) @ Q.T


@pytest.mark.parametrize("k", SIZES)
def test_jacobi_matches_eigvalsh(k):
    W = synth.random_symmetric(k, seed=100 + k)
    ev, V, sweeps = O.jacobi_eigh(W)
    ref = np.linalg.eigvalsh(W)
    assert np.allclose(np.sort(ev), ref, atol=1e-12 * max(1, np.abs(ref).max()))
    assert np.allclose(V.T @ V, np.eye(k), atol=1e-13 * k)
    assert np.allclose(W @ V, V * ev, atol=1e-12 * max(1, np.linalg.norm(W)))
    assert sweeps <= 15


def test_jacobi_two_by_two_closed_form():
    a, b, c = 1.5, -0.75, 0.25
    W = np.array([[a, b], [b, c]])
    ev, V, _ = O.jacobi_eigh(W)
    mid, rad = (a + c) / 2, np.hypot((a - c) / 2, b)
    assert np.allclose(np.sort(ev), [mid - rad, mid + rad], atol=1e-15)


def test_jacobi_diagonal_needs_no_sweep():
    d = np.array([3.0, -1.0, 0.5, 2.0])
    ev, V, sweeps = O.jacobi_eigh(np.diag(d))
    assert sweeps == 0
    assert np.array_equal(ev, d)
    assert np.array_equal(V, np.eye(4))


def test_jacobi_repeated_eigenvalues():
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    lam = np.array([2.0] * 5 + [-1.0] * 4 + [0.0] * 3)
    W = (Q * lam) @ Q.T
    ev, V, _ = O.jacobi_eigh(W)
    assert np.allclose(np.sort(ev), np.sort(lam), atol=1e-12)


@pytest.mark.parametrize("k", SIZES)
def test_projection_matches_eigh_and_is_psd(k):
    W = synth.random_symmetric(k, seed=200 + k)
    P = O.psd_project(W)
    assert np.allclose(P, _proj_eigh(W), atol=1e-12 * max(1, np.linalg.norm(W)))
    assert np.array_equal(P, P.T)
    assert np.linalg.eigvalsh(P).min() >= -1e-12 * np.linalg.norm(W)


@pytest.mark.parametrize("k", [3, 15, 30])
def test_projection_idempotent_and_moreau(k):
    W = synth.random_symmetric(k, seed=300 + k, scale=3.0)
    P = O.psd_project(W)
    assert np.allclose(O.psd_project(P), P, atol=1e-12 * np.linalg.norm(W))
    N = O.psd_project(-W)
    # Moreau: W = P+(W) - P+(-W), and the two parts are orthogonal
    assert np.allclose(P - N, W, atol=1e-12 * np.linalg.norm(W))
    assert abs(np.sum(P * N)) <= 1e-11 * np.linalg.norm(W) ** 2


def test_projection_is_nearest_psd():
    W = synth.random_symmetric(10, seed=4)
    P = O.psd_project(W)
    lam = np.linalg.eigvalsh(W)
    dist = np.linalg.norm(W - P)
    assert np.isclose(dist, np.sqrt(np.sum(np.minimum(lam, 0) ** 2)), rtol=1e-12)
    rng = np.random.default_rng(9)
    for _ in range(50):
        G = rng.standard_normal((10, 10))
        Y = P + 0.1 * G @ G.T / 10  # other PSD matrices near P
        assert np.linalg.norm(W - Y) >= dist - 1e-12


def test_projection_special_cases():
    rng = np.random.default_rng(1)
    G = rng.standard_normal((7, 7))
    S = G @ G.T
    assert np.allclose(O.psd_project(S), S, atol=1e-12 * np.linalg.norm(S))
    assert np.allclose(O.psd_project(-S), 0, atol=1e-12 * np.linalg.norm(S))
    d = np.array([1.0, -2.0, 0.0, 3.0])
    assert np.array_equal(O.psd_project(np.diag(d)), np.diag(np.maximum(d, 0)))
    assert np.array_equal(O.psd_project(np.zeros((5, 5))), np.zeros((5, 5)))
    assert O.psd_project(np.array([[-4.0]]))[0, 0] == 0.0
    assert O.psd_project(np.array([[4.0]]))[0, 0] == 4.0


def test_projection_batch_equals_single():
    sizes, off, W = synth.clique_batch([3, 7, 1, 12], seed=8)
    blocks = [W[off[t]:off[t + 1]].reshape(k, k) for t, k in enumerate(sizes)]
    Ps = O.psd_project_batch(blocks)
    for B, P in zip(blocks, Ps):
        assert np.array_equal(P, O.psd_project(B))
    Ps2, evs, Vs = O.psd_project_batch_eig(blocks)
    for B, P, ev, V in zip(blocks, Ps2, evs, Vs):
        assert np.array_equal(P, O.psd_project(B))
        assert np.allclose((V * ev) @ V.T, B, atol=1e-12)


@pytest.mark.parametrize("m", [1, 4, 33, 120])
def test_cholesky_matches_numpy(m):
    rng = np.random.default_rng(m)
    G = rng.standard_normal((m, m + 5))
    M = G @ G.T
    L = O.cholesky(M)
    assert np.allclose(L, np.linalg.cholesky(M), atol=1e-10 * np.abs(M).max())
    assert np.allclose(L @ L.T, M, atol=1e-11 * np.abs(M).max())
    assert np.all(np.triu(L, 1) == 0)
    t = rng.standard_normal(m)
    assert np.allclose(O.chol_solve(L, t), np.linalg.solve(M, t), rtol=1e-9, atol=1e-9)


def test_cholesky_rejects_indefinite():
    M = np.array([[1.0, 2.0], [2.0, 1.0]])
    with pytest.raises(O.OracleError) as e:
        O.cholesky(M)
    assert e.value.status == O.E_RANK
    with pytest.raises(O.OracleError):
        O.cholesky(np.zeros((3, 3)))
