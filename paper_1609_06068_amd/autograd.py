"""Differentiable entry points over the gfx950 library (torch.autograd).

Every forward and backward is a library call; PyTorch only supplies device
memory, the stream and the autograd bookkeeping.

* `UnrolledADMM` / `unrolled_x`: x after K iterations of Algorithm 1 from
  zero state as a function of (c, b).  The forward runs the library's own
  iteration (cdcs_unrolled_step: the kernels of cdcs_admm_step, with the
  caller's c and b) and keeps, per iteration, the eigenpairs of every
  clique's projection (the per-iteration checkpoint: the adjoint of an
  iteration needs nothing else, since the rest of the iteration is linear).
  The backward runs the library's adjoint of one iteration
  (cdcs_unrolled_step_vjp: Daleckii-Krein adjoint of the projection, the
  gather/scatter transposes and the cached KKT solve) from the last
  iteration to the first.
* `PSDProject`: P(W_k) for packed FP32 clique blocks, backward by
  cdcs_psd_project_vjp.
* `Gather` / `Scatter`: the entry selectors H_k and sum_k H_k^T, each other's
  transposes.
* `Affine`: x = F(r1, b) of the KKT system (E:OptCondMinYPrimal), backward by
  cdcs_affine_project_adjoint.
"""
from __future__ import annotations

import numpy as np
import torch

from . import cdcs


class UnrolledADMM(torch.autograd.Function):
    """x_K(c, b) of K Algorithm-1 iterations from zero state."""

    @staticmethod
    def forward(ctx, c, b, sol, K, rho):
        st = sol.new_state("primal")
        c = c.detach().contiguous()
        b = b.detach().contiguous()
        evals = torch.empty((K, sol.nevals), dtype=torch.float32, device=c.device)
        evecs = torch.empty((K, sol.nwarm), dtype=torch.float32, device=c.device)
        for n in range(K):
            sol.unrolled_step(st, c, b, rho, evals[n], evecs[n])
        ctx.save_for_backward(evals, evecs)
        ctx.sol, ctx.K, ctx.rho = sol, K, rho
        return st["x"]

    @staticmethod
    def backward(ctx, xbar):
        evals, evecs = ctx.saved_tensors
        sol, K, rho = ctx.sol, ctx.K, ctx.rho
        dev = xbar.device
        cbar = torch.zeros(sol.nnz, dtype=torch.float64, device=dev)
        bbar = torch.zeros(sol.m, dtype=torch.float64, device=dev)
        blkbar = torch.zeros(sol.nslots, dtype=torch.float64, device=dev)
        lambar = torch.zeros(sol.nslots, dtype=torch.float64, device=dev)
        xbar = xbar.contiguous().to(torch.float64)
        for n in range(K - 1, -1, -1):
            sol.unrolled_step_vjp(evals[n], evecs[n], xbar if n == K - 1 else None, blkbar, lambar, cbar, bbar,
                                  rho=rho)
        return cbar, bbar, None, None, None


def unrolled_x(sol, c, b, K: int, rho: float = 1.0):
    """x after K iterations of Algorithm 1 from zero state, differentiable in (c, b)."""
    return UnrolledADMM.apply(c, b, sol, K, rho)


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
        gW = cdcs.psd_project_vjp(gP.contiguous(), ev, V, eoff, voff, g["sizes_d"], g["off_d"], g["smax"])
        return gW, None


class Gather(torch.autograd.Function):
    """x (entries) -> H_k x packed; adjoint sum_k H_k^T."""

    @staticmethod
    def forward(ctx, x, sol):
        ctx.sol = sol
        return sol.gather(x)

    @staticmethod
    def backward(ctx, g):
        return ctx.sol.scatter(g), None


class Scatter(torch.autograd.Function):
    """packed clique blocks -> sum_k H_k^T (entries); adjoint H_k."""

    @staticmethod
    def forward(ctx, packed, sol):
        ctx.sol = sol
        return sol.scatter(packed)

    @staticmethod
    def backward(ctx, g):
        return ctx.sol.gather(g), None


class Affine(torch.autograd.Function):
    """x = F(r1, b): the x part of the KKT solve with right-hand side (r1, b)."""

    @staticmethod
    def forward(ctx, r1, b, sol):
        ctx.sol = sol
        x, _ = sol.affine_project(r1, b)
        return x

    @staticmethod
    def backward(ctx, gx):
        r1bar, bbar = ctx.sol.affine_project_adjoint(gx)
        return r1bar, bbar, None


def geometry(sol):
    """Device-side size/offset tables of the solver's cliques."""
    sizes = np.asarray(sol.sizes, dtype=np.int64)
    return {"sizes_h": sizes, "sizes_d": torch.as_tensor(sizes.astype(np.int32), device="cuda"),
            "off_d": torch.as_tensor(sol.offsets, device="cuda"), "smax": int(sizes.max())}


def entry_weights(prob, device="cuda"):
    """w_e = 1 on diagonal pattern entries, 2 off the diagonal (vec inner products)."""
    return torch.as_tensor(np.where(prob.ei == prob.ej, 1.0, 2.0), dtype=torch.float64, device=device)
