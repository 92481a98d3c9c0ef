"""Differentiable building blocks over the gfx950 library (torch.autograd).

Each Function's forward and backward call library kernels: the batched PSD
projection and its Daleckii-Krein adjoint, the entry selectors H_k (gather)
and sum_k H_k^T (scatter), which are each other's transposes, and the affine
projection.  The affine map x = F(r1, b) of the KKT system
(E:OptCondMinYPrimal) satisfies (dF/dr1)^T = W (dF/dr1) W^-1 with W = diag(w)
(w = 1 on diagonal entries, 2 off-diagonal), and (dF/db)^T xbar is the y of
that same solve, so its adjoint is the cached-factor solve applied to the
cotangent.

`unrolled_x` runs K iterations of Algorithm 1 from zero state as a function of
(c, b) with per-iteration checkpointing (only the state entering each
iteration is kept; the backward recomputes one iteration at a time).
"""
from __future__ import annotations

import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

from . import cdcs


class PSDProject(torch.autograd.Function):
    """P(W_k) for packed FP32 clique blocks; backward by Daleckii-Krein."""

    @staticmethod
    def forward(ctx, W, geo):
        P, ev, V, eoff, voff = cdcs.psd_project_batched(W, geo["sizes_h"], geo["off_d"], smax=geo["smax"], eig=True)
        ctx.save_for_backward(ev, V, eoff, voff)
        ctx.geo = geo
        return P

    @staticmethod
    def backward(ctx, gP):
        ev, V, eoff, voff = ctx.saved_tensors
        g = ctx.geo
        gW = cdcs.psd_project_vjp(gP.float(), ev, V, eoff, voff, g["sizes_d"], g["off_d"], g["smax"])
        return gW, None


class Gather(torch.autograd.Function):
    """x (entries) -> H_k x packed; adjoint sum_k H_k^T."""

    @staticmethod
    def forward(ctx, x, sol):
        ctx.sol = sol
        return sol.gather(x)

    @staticmethod
    def backward(ctx, g):
        return ctx.sol.scatter(g.double()), None


class Scatter(torch.autograd.Function):
    """packed clique blocks -> sum_k H_k^T (entries); adjoint H_k."""

    @staticmethod
    def forward(ctx, packed, sol):
        ctx.sol = sol
        return sol.scatter(packed)

    @staticmethod
    def backward(ctx, g):
        return ctx.sol.gather(g.double()), None


class Affine(torch.autograd.Function):
    """x = F(r1, b): the x part of the KKT solve with right-hand side (r1, b)."""

    @staticmethod
    def forward(ctx, r1, b, sol, w):
        ctx.sol, ctx.w = sol, w
        x, _ = sol.affine_project(r1, b)
        return x

    @staticmethod
    def backward(ctx, gx):
        w = ctx.w
        xo, yo = ctx.sol.affine_project(gx.double() / w, torch.zeros(ctx.sol.m, dtype=torch.float64,
                                                                        device=gx.device))
        return w * xo, yo, None, None


def geometry(sol):
    """Device-side size/offset tables of the solver's cliques."""
    sizes = np.asarray(sol.sizes, dtype=np.int64)
    return {"sizes_h": sizes, "sizes_d": torch.as_tensor(sizes.astype(np.int32), device="cuda"),
            "off_d": torch.as_tensor(sol.offsets, device="cuda"), "smax": int(sizes.max())}


def entry_weights(prob, device="cuda"):
    return torch.as_tensor(np.where(prob.ei == prob.ej, 1.0, 2.0), dtype=torch.float64, device=device)


def unrolled_x(sol, prob, c, b, K: int, rho: float = 1.0, use_checkpoint: bool = True):
    """x after K iterations of Algorithm 1 from zero state, differentiable in (c, b)."""
    geo = geometry(sol)
    w = entry_weights(prob, c.device)
    xk = torch.zeros(sol.nslots, dtype=torch.float64, device=c.device)
    lam = torch.zeros_like(xk)

    def step(xk, lam, c, b):
        r1 = Scatter.apply(xk + lam / rho, sol) - c / rho           # (E:OptCondMinYPrimal) rhs
        x = Affine.apply(r1, b, sol, w)
        h = Gather.apply(x, sol)
        P = PSDProject.apply((h - lam / rho).float(), geo).double()  # (E:XkUpdate)
        lam_new = lam + rho * (P - h)                                # (E:LambdakUpdate)
        return x, P, lam_new

    x = None
    for _ in range(K):
        if use_checkpoint:
            x, xk, lam = checkpoint(step, xk, lam, c, b, use_reentrant=False)
        else:
            x, xk, lam = step(xk, lam, c, b)
    return x
