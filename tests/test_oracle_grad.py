"""Pins for the oracle's reverse-mode derivative of unrolled Algorithm 1.

The adjoint (FP64) is checked against central finite differences of the
oracle's own forward iteration, and the projection adjoint against the
Frechet derivative of P(W) = V max(L,0) V^T computed by finite differences."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1609_06068_amd import synth


def _losses(o, prob, x, xt, which):
    if which == "linear":
        L, g = O.loss_linear(prob, o.dec, x)
        return L, g, o.dec.w * x          # direct dL/dc of <C, X>
    L, g = O.loss_target(o.dec, x, xt)
    return L, g, np.zeros_like(x)


def test_projection_adjoint_is_the_frechet_derivative():
    rng = np.random.default_rng(0)
    W = synth.random_symmetric(9, seed=2)
    ev, V, _ = O.jacobi_eigh(W)
    for _ in range(5):
        H = rng.standard_normal((9, 9))
        H = H + H.T
        G = rng.standard_normal((9, 9))
        G = G + G.T
        h = 1e-6
        dP = (O.psd_project(W + h * H) - O.psd_project(W - h * H)) / (2 * h)
        # <G, DP[H]> = <DP*[G], H> with DP* the Daleckii-Krein form
        assert np.isclose(np.sum(G * dP), np.sum(O.psd_project_vjp(ev, V, G) * H), rtol=1e-6, atol=1e-8)


def test_dk_gamma_cases():
    lam = np.array([2.0, 1.0, -1.0, 0.0])
    g = O.dk_gamma(lam)
    assert g[0, 1] == 1.0 and g[2, 3] == 0.0 and g[3, 3] == 0.0
    assert np.isclose(g[0, 2], 2.0 / 3.0) and np.isclose(g[2, 0], 2.0 / 3.0)
    assert np.isclose(g[0, 3], 1.0)


@pytest.mark.parametrize("which", ["linear", "target"])
def test_unrolled_adjoint_matches_central_differences(which):
    prob = synth.block_arrow(l=4, d=4, h=2, m=6, seed=3)
    o = O.Oracle(prob)
    K = 15
    U = O.Unrolled(o, K=K, rho=1.0)
    xt = prob.meta["x0"]
    x = U.forward(prob.c, prob.b)
    L, g, direct = _losses(o, prob, x, xt, which)
    cbar, bbar = U.backward(g)
    cbar = cbar + direct
    rng = np.random.default_rng(11)
    h = 1e-6
    for _ in range(4):
        dc = rng.standard_normal(prob.nU)
        dc /= np.linalg.norm(dc)
        db = rng.standard_normal(prob.m)
        db /= np.linalg.norm(db)
        for (c1, b1, c2, b2, ana) in [(prob.c + h * dc, prob.b, prob.c - h * dc, prob.b, np.dot(cbar, dc)),
                                      (prob.c, prob.b + h * db, prob.c, prob.b - h * db, np.dot(bbar, db))]:
            pr = synth.Problem(**{**prob.__dict__})
            pr.c, pr.b = c1, b1
            Lp = _losses(o, pr, O.Unrolled(o, K=K).forward(c1, b1), xt, which)[0]
            pr.c, pr.b = c2, b2
            Lm = _losses(o, pr, O.Unrolled(o, K=K).forward(c2, b2), xt, which)[0]
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - ana) <= 1e-5 * max(1.0, abs(ana)), (which, fd, ana)
