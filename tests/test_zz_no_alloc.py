"""The allocation-free affine adjoint (needs a GPU): through the C-ABI,
cdcs_affine_project_adjoint_noalloc against cdcs_affine_project_adjoint on
two calls in a row, the second on a smaller handle (the fixed device array
keeps the first call's contents), for dense and sparse A and a batch handle;
and a handle above the array's limit is rejected."""
import ctypes

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


def _noalloc(torch, sol, xbar):
    L = cdcs.load_library()
    r1 = torch.full((sol.nnz,), float("nan"), dtype=torch.float64, device="cuda")
    r2 = torch.full((sol.m,), float("nan"), dtype=torch.float64, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = L.cdcs_affine_project_adjoint_noalloc(sol._h, ctypes.c_void_p(xbar.data_ptr()),
                                               ctypes.c_void_p(r1.data_ptr()), ctypes.c_void_p(r2.data_ptr()), s)
    return st, r1, r2


def _compare(torch, sol, seed):
    rng = np.random.default_rng(seed)
    xbar = torch.as_tensor(rng.standard_normal(sol.nnz), device="cuda")
    st, r1, r2 = _noalloc(torch, sol, xbar)
    assert st == cdcs.OK, cdcs.load_library().cdcs_last_error()
    e1, e2 = sol.affine_project_adjoint(xbar)
    torch.cuda.synchronize()
    # the same kernels on the same inputs: the same bits
    assert torch.equal(r1, e1) and torch.equal(r2, e2)
    assert torch.isfinite(r1).all() and torch.isfinite(r2).all()


@pytest.mark.parametrize("pair", ["dense", "sparse", "batch"])
def test_noalloc_matches_the_allocating_entry_point(torch, pair):
    if pair == "dense":
        big, small = cdcs.Solver(synth.c1()), cdcs.Solver(synth.block_arrow(3, 4, 2, 6, seed=11))
    elif pair == "sparse":
        big, small = cdcs.Solver(synth.c3_small()), cdcs.Solver(synth.block_arrow(2, 3, 1, 4, seed=12))
    else:
        big = cdcs.BatchSolver([synth.block_arrow(6, 8, 3, 30, seed=13), synth.block_arrow(4, 6, 2, 20, seed=14)])
        small = cdcs.BatchSolver([synth.block_arrow(2, 3, 1, 4, seed=15)])
    assert small.nnz < big.nnz and small.m < big.m
    _compare(torch, big, 1)
    _compare(torch, small, 2)  # second call, smaller input
    big.close()
    small.close()


def test_noalloc_rejects_handles_above_the_limit(torch):
    prob = synth.c3()  # 4.9 M pattern entries > 2^20
    sol = cdcs.Solver(prob)
    xbar = torch.zeros(sol.nnz, dtype=torch.float64, device="cuda")
    st, _, _ = _noalloc(torch, sol, xbar)
    assert st == cdcs.E_ARG
    assert b"scratch" in cdcs.load_library().cdcs_last_error()
    sol.close()
