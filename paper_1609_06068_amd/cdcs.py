"""Python binding of libcdcs.so (the gfx950 library declared in include/cdcs.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  Importing this
module does not load the library; the first call does, and it fails loudly
(CdcsLibraryMissing) when libcdcs.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcdcs.so")

OK, E_ARG, E_PATTERN, E_RANK, E_DEVICE, E_NOMEM, E_NOT_CONVERGED, E_NUMERIC = range(8)
PRIMAL_INFEASIBLE, DUAL_INFEASIBLE = 8, 9
K_PROJECT, K_GEMV_AU, K_TRMV, K_GEMV_ATY, K_SCATTER = range(5)
PRIMAL, DUAL = 0, 1
MAX_CLIQUE = 1024
MAX_BATCHED_CLIQUE = 126
STATUS_NAMES = {0: "CDCS_OK", 1: "CDCS_E_ARG", 2: "CDCS_E_PATTERN", 3: "CDCS_E_RANK", 4: "CDCS_E_DEVICE",
                5: "CDCS_E_NOMEM", 6: "CDCS_E_NOT_CONVERGED", 7: "CDCS_E_NUMERIC", 8: "CDCS_PRIMAL_INFEASIBLE",
                9: "CDCS_DUAL_INFEASIBLE"}

# Every symbol include/cdcs.h declares.
EXPORTS = ["cdcs_setup", "cdcs_setup_batch", "cdcs_batch_info", "cdcs_get_sizes", "cdcs_clique_offsets", "cdcs_psd_project_batched",
           "cdcs_psd_project_vjp", "cdcs_gather", "cdcs_scatter", "cdcs_affine_project", "cdcs_admm_solve",
           "cdcs_admm_step", "cdcs_admm_solve_timed", "cdcs_profile_kernel", "cdcs_get_tuning", "cdcs_set_projection_plan",
           "cdcs_residual_history", "cdcs_warm_reset", "cdcs_destroy", "cdcs_last_error", "cdcs_admm_prepare",
           "cdcs_psd_project_cliques", "cdcs_unrolled_step", "cdcs_unrolled_step_vjp",
           "cdcs_affine_project_adjoint", "cdcs_chordal_extension", "cdcs_affine_project_adjoint_noalloc",
           "cdcs_setup_cones", "cdcs_hsde_init", "cdcs_hsde_solve", "cdcs_hsde_solution", "cdcs_hsde_history",
           "cdcs_hsde_solve_timed"]


class CdcsLibraryMissing(ImportError):
    pass


class CdcsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Pattern(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("i", ctypes.c_void_p), ("j", ctypes.c_void_p)]


class _Cliques(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("ptr", ctypes.c_void_p), ("vert", ctypes.c_void_p)]


class _Constraints(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("dense", ctypes.c_int32), ("ptr", ctypes.c_void_p),
                ("idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("form", ctypes.c_int32), ("check_every", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("jacobi_cap_hits", ctypes.c_int32), ("eps_p", ctypes.c_double), ("eps_d", ctypes.c_double),
                ("obj_primal", ctypes.c_double), ("obj_dual", ctypes.c_double), ("loop_s", ctypes.c_double),
                ("jacobi_sweeps", ctypes.c_int64)]


class _State(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("blk", ctypes.c_void_p),
                ("lam", ctypes.c_void_p), ("v", ctypes.c_void_p), ("vw", ctypes.c_void_p)]


class _Problem(ctypes.Structure):
    _fields_ = [("pattern", ctypes.POINTER(_Pattern)), ("A", ctypes.POINTER(_Constraints)),
                ("b", ctypes.c_void_p), ("c", ctypes.c_void_p), ("cliques", ctypes.POINTER(_Cliques))]


class _InstanceInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("eps_p", ctypes.c_double),
                ("eps_d", ctypes.c_double), ("obj_primal", ctypes.c_double), ("obj_dual", ctypes.c_double),
                ("time_to_tol_s", ctypes.c_double)]


class _Tuning(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int32), ("threads", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("nbuckets", ctypes.c_int32), ("bucket_size", ctypes.c_int32 * 8),
                ("bucket_threads", ctypes.c_int32 * 8), ("bucket_count", ctypes.c_int32 * 8),
                ("bucket_us", ctypes.c_float * 8), ("queue_us", ctypes.c_float), ("buckets_us", ctypes.c_float),
                ("parallel_us", ctypes.c_float)]


class _Sizes(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("p", ctypes.c_int32), ("smax", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("nslots", ctypes.c_int64), ("sparse_a", ctypes.c_int32),
                ("sparse_factor", ctypes.c_int32), ("nnz_a", ctypes.c_int64), ("nnz_factor", ctypes.c_int64),
                ("nwarm", ctypes.c_int64), ("nnz_l", ctypes.c_int64), ("nvcones", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("nslots_psd", ctypes.c_int64)]


class _Vcones(ctypes.Structure):
    _fields_ = [("ncones", ctypes.c_int32), ("kind", ctypes.c_void_p), ("ptr", ctypes.c_void_p),
                ("vert", ctypes.c_void_p)]


class _HsdeState(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("s", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("tk", ctypes.c_void_p), ("vw", ctypes.c_void_p)]


class _HsdeInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("jacobi_cap_hits", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("res_pri", ctypes.c_double), ("res_dual", ctypes.c_double),
                ("gap", ctypes.c_double), ("obj_primal", ctypes.c_double), ("obj_dual", ctypes.c_double),
                ("tau", ctypes.c_double), ("kappa", ctypes.c_double), ("loop_s", ctypes.c_double),
                ("jacobi_sweeps", ctypes.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcdcs.so and declare the C signatures (no device work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise CdcsLibraryMissing(f"{path} is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.cdcs_setup.argtypes = [P(_Pattern), P(_Constraints), vp, vp, P(_Cliques), vp, vp, P(vp)]
    L.cdcs_setup_cones.argtypes = [P(_Pattern), P(_Constraints), vp, vp, P(_Cliques), P(_Vcones), vp, vp, P(vp)]
    L.cdcs_hsde_init.argtypes = [vp, P(_HsdeState), vp]
    L.cdcs_hsde_solve.argtypes = [vp, P(_HsdeState), P(_Options), P(_HsdeInfo), vp]
    L.cdcs_hsde_solution.argtypes = [vp, P(_HsdeState), i32, vp, vp, vp]
    L.cdcs_hsde_history.argtypes = [vp, vp, i32]
    L.cdcs_hsde_solve_timed.argtypes = [vp, P(_HsdeState), P(_Options), P(_HsdeInfo), vp, vp, vp]
    L.cdcs_setup_batch.argtypes = [i32, P(_Problem), vp, vp, P(vp)]
    L.cdcs_batch_info.argtypes = [vp, i32, P(_InstanceInfo)]
    L.cdcs_get_sizes.argtypes = [vp, P(_Sizes)]
    L.cdcs_get_tuning.argtypes = [vp, P(_Tuning)]
    L.cdcs_set_projection_plan.argtypes = [vp, i32, i32, i32]
    L.cdcs_admm_prepare.argtypes = [vp, P(_State), P(_Options), vp]
    L.cdcs_psd_project_cliques.argtypes = [vp, vp, vp, vp]
    L.cdcs_unrolled_step.argtypes = [vp, P(_State), vp, vp, dbl, vp, vp, vp]
    L.cdcs_unrolled_step_vjp.argtypes = [vp, dbl, vp, vp, vp, vp, vp, vp, vp, vp]
    L.cdcs_affine_project_adjoint.argtypes = [vp, vp, vp, vp, vp]
    L.cdcs_chordal_extension.argtypes = [P(_Pattern), P(i64), P(i32), P(i64), vp, vp, vp, vp]
    L.cdcs_affine_project_adjoint_noalloc.argtypes = [vp, vp, vp, vp, vp]
    L.cdcs_clique_offsets.argtypes = [vp, vp]
    L.cdcs_psd_project_batched.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.cdcs_psd_project_vjp.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.cdcs_gather.argtypes = [vp, vp, vp, vp]
    L.cdcs_scatter.argtypes = [vp, vp, vp, vp]
    L.cdcs_affine_project.argtypes = [vp, vp, vp, vp, vp, vp]
    L.cdcs_admm_solve.argtypes = [vp, P(_State), P(_Options), P(_Info), vp]
    L.cdcs_admm_step.argtypes = [vp, P(_State), i32, dbl, vp]
    L.cdcs_warm_reset.argtypes = [vp, vp, vp]
    L.cdcs_admm_solve_timed.argtypes = [vp, P(_State), P(_Options), P(_Info), vp, vp, vp]
    L.cdcs_profile_kernel.argtypes = [vp, P(_State), i32, dbl, i32, i32, vp]
    L.cdcs_residual_history.argtypes = [vp, vp, i32]
    L.cdcs_destroy.argtypes = [vp]
    L.cdcs_last_error.argtypes = []
    L.cdcs_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "cdcs_last_error":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st: int, what: str):
    if st != OK:
        msg = load_library().cdcs_last_error().decode(errors="replace")
        raise CdcsError(st, f"{what}: {msg}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the cdcs library needs a HIP device (torch.cuda.is_available() is False)")
    return torch


def _stream(torch, stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


@dataclass
class SolveInfo:
    iters: int
    status: int
    converged: bool
    jacobi_cap_hits: int
    eps_p: float
    eps_d: float
    obj_primal: float
    obj_dual: float
    loop_s: float
    jacobi_sweeps: int


def _marshal(prob):
    """C structs describing one problem (host arrays kept alive in the tuple)."""
    ei = np.ascontiguousarray(prob.ei, dtype=np.int32)
    ej = np.ascontiguousarray(prob.ej, dtype=np.int32)
    b = np.ascontiguousarray(prob.b, dtype=np.float64)
    c = np.ascontiguousarray(prob.c, dtype=np.float64)
    pat = _Pattern(int(prob.n), int(ei.shape[0]), _np_ptr(ei), _np_ptr(ej))
    if prob.clique_ptr is None:
        # no cliques given: setup computes a chordal extension and its cliques
        cptr = cvert = cl = None
    else:
        cptr = np.ascontiguousarray(prob.clique_ptr, dtype=np.int64)
        cvert = np.ascontiguousarray(prob.clique_vert, dtype=np.int32)
        cl = _Cliques(int(cptr.shape[0] - 1), _np_ptr(cptr), _np_ptr(cvert))
    if prob.A is not None:
        aval = np.ascontiguousarray(prob.A, dtype=np.float64)
        cons = _Constraints(int(b.shape[0]), 1, None, None, _np_ptr(aval))
        keep = (aval,)
    else:
        aptr = np.ascontiguousarray(prob.A_ptr, dtype=np.int64)
        aidx = np.ascontiguousarray(prob.A_idx, dtype=np.int32)
        aval = np.ascontiguousarray(prob.A_val, dtype=np.float64)
        cons = _Constraints(int(b.shape[0]), 0, _np_ptr(aptr), _np_ptr(aidx), _np_ptr(aval))
        keep = (aptr, aidx, aval)
    return pat, cons, b, c, cl, (ei, ej, cptr, cvert, b, c) + keep


def _marshal_cones(prob):
    """The vector cones of a problem as a C struct (None without cones)."""
    if getattr(prob, "cone_kind", None) is None or len(prob.cone_kind) == 0:
        return None, ()
    kind = np.ascontiguousarray(prob.cone_kind, dtype=np.int32)
    ptr = np.ascontiguousarray(prob.cone_ptr, dtype=np.int64)
    vert = np.ascontiguousarray(prob.cone_vert, dtype=np.int32)
    return _Vcones(int(kind.shape[0]), _np_ptr(kind), _np_ptr(ptr), _np_ptr(vert)), (kind, ptr, vert)


@dataclass
class HsdeInfo:
    iters: int
    status: int
    jacobi_cap_hits: int
    res_pri: float
    res_dual: float
    gap: float
    obj_primal: float
    obj_dual: float
    tau: float
    kappa: float
    loop_s: float
    jacobi_sweeps: int


class Solver:
    """One SDP set up on the device (cdcs_setup) and its ADMM entry points."""

    def __init__(self, prob, _handle=None):
        L = load_library()
        torch = _torch()
        self._torch = torch
        if _handle is None:
            pat, cons, b, c, cl, keep = _marshal(prob)
            vc, keep_vc = _marshal_cones(prob)
            h = ctypes.c_void_p()
            if vc is None:
                st = L.cdcs_setup(ctypes.byref(pat), ctypes.byref(cons), _np_ptr(b), _np_ptr(c),
                                  ctypes.byref(cl) if cl is not None else None, None, _stream(torch), ctypes.byref(h))
            else:
                st = L.cdcs_setup_cones(ctypes.byref(pat), ctypes.byref(cons), _np_ptr(b), _np_ptr(c),
                                        ctypes.byref(cl) if cl is not None else None, ctypes.byref(vc), None,
                                        _stream(torch), ctypes.byref(h))
            del keep, keep_vc
            _check(st, "cdcs_setup")
        else:
            h = _handle
        self._h = h
        sz = _Sizes()
        _check(L.cdcs_get_sizes(h, ctypes.byref(sz)), "cdcs_get_sizes")
        self.n, self.m, self.p, self.smax = sz.n, sz.m, sz.p, sz.smax
        self.nnz, self.nslots = sz.nnz, sz.nslots
        self.sparse_a, self.nnz_a = bool(sz.sparse_a), sz.nnz_a
        self.sparse_factor, self.nnz_factor = bool(sz.sparse_factor), sz.nnz_factor
        self.nwarm = sz.nwarm
        self.nnz_l = sz.nnz_l  # > 0: sparse Cholesky factor of A D^-1 A^T
        self.nvcones, self.nslots_psd = sz.nvcones, sz.nslots_psd
        off = np.empty(self.p + 1, dtype=np.int64)
        _check(L.cdcs_clique_offsets(h, _np_ptr(off)), "cdcs_clique_offsets")
        self.offsets = off
        self.sizes = np.diff(off)
        # packed offsets are prefix sums of s(s+1)/2: recover s
        self.sizes = ((np.sqrt(8 * self.sizes + 1) - 1) // 2).astype(np.int64)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().cdcs_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_state(self, form: str = "primal") -> dict:
        torch = self._torch
        dev = torch.device("cuda")
        st = {
            "x": torch.zeros(self.nnz, dtype=torch.float64, device=dev),
            "y": torch.zeros(self.m, dtype=torch.float64, device=dev),
            "blk": torch.zeros(self.nslots, dtype=torch.float32, device=dev),
            "lam": torch.zeros(self.nslots, dtype=torch.float32, device=dev),
            "v": torch.zeros(self.nslots, dtype=torch.float32, device=dev) if form == "dual" else None,
            # eigenvector warm start carried from one solve call to the next
            "vw": torch.empty(max(self.nwarm, 1), dtype=torch.float32, device=dev),
        }
        _check(load_library().cdcs_warm_reset(self._h, _ptr(st["vw"]), _stream(torch, None)), "cdcs_warm_reset")
        return st

    @staticmethod
    def _cstate(st: dict) -> _State:
        return _State(_ptr(st["x"]), _ptr(st["y"]), _ptr(st["blk"]), _ptr(st["lam"]), _ptr(st.get("v")),
                      _ptr(st.get("vw")))

    def solve(self, state: dict, form: str = "primal", rho: float = 1.0, tol: float = 1e-4,
              max_iter: int = 500, check_every: int = 50, stream=None, raise_on_cap: bool = False,
              raise_on_numeric: bool = True) -> SolveInfo:
        """cdcs_admm_solve.  Raises CdcsError on failure; CDCS_E_NOT_CONVERGED
        only with raise_on_cap, CDCS_E_NUMERIC unless raise_on_numeric is
        False (then SolveInfo.status carries it)."""
        L = load_library()
        f = PRIMAL if form == "primal" else DUAL
        opts = _Options(float(rho), float(tol), int(max_iter), f, int(check_every))
        info = _Info()
        cs = self._cstate(state)
        st = L.cdcs_admm_solve(self._h, ctypes.byref(cs), ctypes.byref(opts), ctypes.byref(info),
                               _stream(self._torch, stream))
        allowed = (OK, E_NOT_CONVERGED) if raise_on_numeric else (OK, E_NOT_CONVERGED, E_NUMERIC)
        if st not in allowed or (raise_on_cap and st == E_NOT_CONVERGED):
            _check(st, "cdcs_admm_solve")
        return SolveInfo(info.iters, info.status, bool(info.converged), info.jacobi_cap_hits, info.eps_p,
                         info.eps_d, info.obj_primal, info.obj_dual, info.loop_s, info.jacobi_sweeps)

    def solve_timed(self, state: dict, form: str = "primal", rho: float = 1.0, tol: float = 0.0,
                    max_iter: int = 500, stream=None):
        """cdcs_admm_solve with eager launches and events around every kernel:
        returns (SolveInfo, {kernel name: (total ms, launches)})."""
        L = load_library()
        f = PRIMAL if form == "primal" else DUAL
        opts = _Options(float(rho), float(tol), int(max_iter), f, 0)
        info = _Info()
        cs = self._cstate(state)
        ms = np.zeros(5, dtype=np.float64)
        n = np.zeros(5, dtype=np.int64)
        st = L.cdcs_admm_solve_timed(self._h, ctypes.byref(cs), ctypes.byref(opts), ctypes.byref(info),
                                     ms.ctypes.data, n.ctypes.data, _stream(self._torch, stream))
        if st not in (OK, E_NOT_CONVERGED):
            _check(st, "cdcs_admm_solve_timed")
        names = ("project", "gemv_Au", "trmv", "gemv_ATy", "scatter")
        times = {names[k]: (float(ms[k]), int(n[k])) for k in range(5)}
        return SolveInfo(info.iters, info.status, bool(info.converged), info.jacobi_cap_hits, info.eps_p,
                         info.eps_d, info.obj_primal, info.obj_dual, info.loop_s, info.jacobi_sweeps), times

    def step(self, state: dict, form: str = "primal", rho: float = 1.0, stream=None):
        L = load_library()
        cs = self._cstate(state)
        _check(L.cdcs_admm_step(self._h, ctypes.byref(cs), PRIMAL if form == "primal" else DUAL, float(rho),
                                _stream(self._torch, stream)), "cdcs_admm_step")

    # ---- homogeneous self-dual embedding ----------------------------------
    def new_hsde_state(self) -> dict:
        """HSDE state buffers at the starting point (cdcs_hsde_init)."""
        torch = self._torch
        dev = torch.device("cuda")
        st = {
            "x": torch.empty(self.nnz, dtype=torch.float64, device=dev),
            "y": torch.empty(self.m, dtype=torch.float64, device=dev),
            "s": torch.empty(self.nslots, dtype=torch.float32, device=dev),
            "z": torch.empty(self.nslots, dtype=torch.float32, device=dev),
            "tk": torch.empty(2, dtype=torch.float64, device=dev),
            "vw": torch.empty(max(self.nwarm, 1), dtype=torch.float32, device=dev),
        }
        self.hsde_init(st)
        return st

    @staticmethod
    def _hstate(st: dict) -> _HsdeState:
        return _HsdeState(_ptr(st["x"]), _ptr(st["y"]), _ptr(st["s"]), _ptr(st["z"]), _ptr(st["tk"]),
                          _ptr(st.get("vw")))

    def hsde_init(self, st: dict, stream=None):
        hs = self._hstate(st)
        _check(load_library().cdcs_hsde_init(self._h, ctypes.byref(hs), _stream(self._torch, stream)),
               "cdcs_hsde_init")

    def hsde_solve(self, st: dict, tol: float = 1e-4, max_iter: int = 2000, check_every: int = 50,
                   stream=None) -> HsdeInfo:
        """cdcs_hsde_solve.  The outcome (solved, infeasible, unbounded, cap,
        numeric) is HsdeInfo.status; other failures raise CdcsError."""
        opts = _Options(1.0, float(tol), int(max_iter), 0, int(check_every))
        info = _HsdeInfo()
        hs = self._hstate(st)
        r = load_library().cdcs_hsde_solve(self._h, ctypes.byref(hs), ctypes.byref(opts), ctypes.byref(info),
                                           _stream(self._torch, stream))
        if r not in (OK, E_NOT_CONVERGED, E_NUMERIC, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE):
            _check(r, "cdcs_hsde_solve")
        return HsdeInfo(info.iters, info.status, info.jacobi_cap_hits, info.res_pri, info.res_dual, info.gap,
                        info.obj_primal, info.obj_dual, info.tau, info.kappa, info.loop_s, info.jacobi_sweeps)

    def hsde_solve_timed(self, st: dict, tol: float = 0.0, max_iter: int = 500, stream=None):
        """cdcs_hsde_solve_timed: (HsdeInfo, {kernel name: (total ms, launches)})."""
        opts = _Options(1.0, float(tol), int(max_iter), 0, 0)
        info = _HsdeInfo()
        hs = self._hstate(st)
        ms = np.zeros(5, dtype=np.float64)
        n = np.zeros(5, dtype=np.int64)
        r = load_library().cdcs_hsde_solve_timed(self._h, ctypes.byref(hs), ctypes.byref(opts), ctypes.byref(info),
                                                 ms.ctypes.data, n.ctypes.data, _stream(self._torch, stream))
        if r not in (OK, E_NOT_CONVERGED, E_NUMERIC, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE):
            _check(r, "cdcs_hsde_solve_timed")
        names = ("project", "gemv_Au", "trmv", "gemv_ATy", "scatter")
        return (HsdeInfo(info.iters, info.status, info.jacobi_cap_hits, info.res_pri, info.res_dual, info.gap,
                         info.obj_primal, info.obj_dual, info.tau, info.kappa, info.loop_s, info.jacobi_sweeps),
                {names[k]: (float(ms[k]), int(n[k])) for k in range(5)})

    def hsde_solution(self, st: dict, which: int = 0, stream=None):
        """(X, y_sdp) for which=0, the Farkas y for which=1, the ray X for which=2
        (cdcs_hsde_solution; X in pattern order)."""
        torch = self._torch
        X = torch.empty(self.nnz, dtype=torch.float64, device="cuda") if which != 1 else None
        y = torch.empty(self.m, dtype=torch.float64, device="cuda") if which != 2 else None
        hs = self._hstate(st)
        _check(load_library().cdcs_hsde_solution(self._h, ctypes.byref(hs), int(which), _ptr(X), _ptr(y),
                                                  _stream(torch, stream)), "cdcs_hsde_solution")
        return X, y

    def hsde_history(self, n: int) -> np.ndarray:
        """(res_pri, res_dual, gap) of the last HSDE solve's first n iterations."""
        out = np.zeros((n, 3))
        _check(load_library().cdcs_hsde_history(self._h, _np_ptr(out), int(n)), "cdcs_hsde_history")
        return out

    def profile_kernel(self, state: dict, kernel: int, reps: int = 1, form: str = "primal", rho: float = 1.0,
                       stream=None):
        """Enqueue `reps` launches of one kernel of an iteration (for event timing)."""
        cs = self._cstate(state)
        _check(load_library().cdcs_profile_kernel(self._h, ctypes.byref(cs), PRIMAL if form == "primal" else DUAL,
                                                   float(rho), int(kernel), int(reps), _stream(self._torch, stream)),
               "cdcs_profile_kernel")

    def tuning(self) -> dict:
        """The projection launch plan chosen at setup (cdcs_get_tuning)."""
        t = _Tuning()
        _check(load_library().cdcs_get_tuning(self._h, ctypes.byref(t)), "cdcs_get_tuning")
        nb = t.nbuckets
        return {"persistent": t.persistent == 1, "parallel_buckets": t.persistent == 2, "threads": t.threads,
                "grid": t.grid,
                "buckets": [{"size": t.bucket_size[q], "threads": t.bucket_threads[q], "count": t.bucket_count[q],
                             "us": t.bucket_us[q]} for q in range(nb)],
                "queue_us": t.queue_us, "buckets_us": t.buckets_us, "parallel_us": t.parallel_us}

    def set_projection_plan(self, persistent: bool, threads: int = 0, grid: int = 0, parallel: bool = False):
        """Override the tuned plan (cdcs_set_projection_plan); parallel: the
        per-bucket launches on parallel streams."""
        mode = 1 if persistent else (2 if parallel else 0)
        _check(load_library().cdcs_set_projection_plan(self._h, mode, int(threads), int(grid)),
               "cdcs_set_projection_plan")

    def prepare(self, state: dict, form: str = "primal", rho: float = 1.0, tol: float = 1e-4,
                max_iter: int = 500, check_every: int = 50, stream=None):
        """Capture the graphs solve() with these arguments launches (cdcs_admm_prepare)."""
        opts = _Options(float(rho), float(tol), int(max_iter), PRIMAL if form == "primal" else DUAL,
                        int(check_every))
        cs = self._cstate(state)
        _check(load_library().cdcs_admm_prepare(self._h, ctypes.byref(cs), ctypes.byref(opts),
                                                _stream(self._torch, stream)), "cdcs_admm_prepare")

    def project_cliques(self, W, P=None, stream=None):
        """P(W_k) for this handle's cliques with the tuned launch plan, cold start
        (cdcs_psd_project_cliques).  W: packed FP32 device tensor of nslots."""
        torch = self._torch
        W = W.contiguous()
        P = torch.empty_like(W) if P is None else P
        _check(load_library().cdcs_psd_project_cliques(self._h, _ptr(W), _ptr(P), _stream(torch, stream)),
               "cdcs_psd_project_cliques")
        return P

    def history(self, n: int) -> np.ndarray:
        out = np.zeros((n, 2))
        _check(load_library().cdcs_residual_history(self._h, _np_ptr(out), int(n)), "cdcs_residual_history")
        return out

    def gather(self, x, stream=None):
        """H_k x for every clique, packed (FP64)."""
        torch = self._torch
        x = x.contiguous()
        out = torch.empty(self.nslots, dtype=torch.float64, device=x.device)
        _check(load_library().cdcs_gather(self._h, _ptr(x), _ptr(out), _stream(torch, stream)), "cdcs_gather")
        return out

    def scatter(self, packed, stream=None):
        """sum_k H_k^T of packed clique blocks (FP64), on the pattern entries."""
        torch = self._torch
        packed = packed.contiguous()
        out = torch.empty(self.nnz, dtype=torch.float64, device=packed.device)
        _check(load_library().cdcs_scatter(self._h, _ptr(packed), _ptr(out), _stream(torch, stream)),
               "cdcs_scatter")
        return out

    @property
    def nevals(self) -> int:
        return int(np.sum(self.sizes))

    def unrolled_step(self, state: dict, c, b, rho: float = 1.0, evals=None, evecs=None, stream=None):
        """One Algorithm-1 iteration with the given c and b (device FP64),
        saving the projections' eigenpairs (cdcs_unrolled_step)."""
        cs = self._cstate(state)
        c = c.contiguous()
        b = b.contiguous()
        st = load_library().cdcs_unrolled_step(self._h, ctypes.byref(cs), _ptr(c), _ptr(b), float(rho),
                                               _ptr(evals), _ptr(evecs), _stream(self._torch, stream))
        if st not in (OK, E_NOT_CONVERGED):
            _check(st, "cdcs_unrolled_step")

    def unrolled_step_vjp(self, evals, evecs, xbar, blkbar, lambar, cbar, bbar, rho: float = 1.0, stream=None):
        """Adjoint of unrolled_step (cdcs_unrolled_step_vjp): blkbar, lambar
        (FP64 packed) are updated in place, cbar and bbar accumulate."""
        _check(load_library().cdcs_unrolled_step_vjp(self._h, float(rho), _ptr(evals), _ptr(evecs),
                                                     _ptr(xbar.contiguous() if xbar is not None else None),
                                                     _ptr(blkbar), _ptr(lambar), _ptr(cbar), _ptr(bbar),
                                                     _stream(self._torch, stream)), "cdcs_unrolled_step_vjp")

    def affine_project_adjoint(self, xbar, stream=None):
        """Cotangents (r1bar, r2bar) of cdcs_affine_project's inputs from the
        cotangent of its x (cdcs_affine_project_adjoint)."""
        torch = self._torch
        xbar = xbar.contiguous()
        r1bar = torch.empty(self.nnz, dtype=torch.float64, device=xbar.device)
        r2bar = torch.empty(self.m, dtype=torch.float64, device=xbar.device)
        _check(load_library().cdcs_affine_project_adjoint(self._h, _ptr(xbar), _ptr(r1bar), _ptr(r2bar),
                                                          _stream(torch, stream)), "cdcs_affine_project_adjoint")
        return r1bar, r2bar

    def affine_project(self, r1, r2, stream=None):
        torch = self._torch
        x = torch.empty(self.nnz, dtype=torch.float64, device=r1.device)
        y = torch.empty(self.m, dtype=torch.float64, device=r1.device)
        r1 = r1.contiguous()
        r2 = r2.contiguous()
        _check(load_library().cdcs_affine_project(self._h, _ptr(r1), _ptr(r2), _ptr(x), _ptr(y),
                                                   _stream(torch, stream)), "cdcs_affine_project")
        return x, y


@dataclass
class InstanceInfo:
    iters: int
    status: int
    eps_p: float
    eps_d: float
    obj_primal: float
    obj_dual: float
    time_to_tol_s: float


class BatchSolver(Solver):
    """Many independent SDPs in one handle (cdcs_setup_batch): one projection
    launch over every instance's cliques, one factor per instance, per-instance
    stopping.  State buffers are the concatenations of the per-instance ones."""

    def __init__(self, probs):
        L = load_library()
        torch = _torch()
        marsh = [_marshal(p) for p in probs]
        arr = (_Problem * len(probs))()
        for q, (pat, cons, b, c, cl, keep) in enumerate(marsh):
            arr[q] = _Problem(ctypes.pointer(pat), ctypes.pointer(cons), _np_ptr(b), _np_ptr(c), ctypes.pointer(cl))
        h = ctypes.c_void_p()
        st = L.cdcs_setup_batch(len(probs), arr, None, _stream(torch), ctypes.byref(h))
        del marsh, arr
        _check(st, "cdcs_setup_batch")
        super().__init__(None, _handle=h)
        self.nprob = len(probs)
        self.entry_off = np.concatenate([[0], np.cumsum([p.nU for p in probs])]).astype(np.int64)
        self.row_off = np.concatenate([[0], np.cumsum([p.m for p in probs])]).astype(np.int64)
        self.clique_off = np.concatenate([[0], np.cumsum([p.p for p in probs])]).astype(np.int64)

    def instance_info(self) -> list:
        out = (_InstanceInfo * self.nprob)()
        _check(load_library().cdcs_batch_info(self._h, self.nprob, out), "cdcs_batch_info")
        return [InstanceInfo(o.iters, o.status, o.eps_p, o.eps_d, o.obj_primal, o.obj_dual, o.time_to_tol_s)
                for o in out]


def chordal_extension(n: int, ei, ej):
    """Chordal extension of the pattern (ei, ej) of an n x n matrix and its
    maximal cliques (cdcs_chordal_extension, host code: no device needed).
    Returns (fill_i, fill_j, clique_ptr, clique_vert)."""
    L = load_library()
    ei = np.ascontiguousarray(ei, dtype=np.int32)
    ej = np.ascontiguousarray(ej, dtype=np.int32)
    pat = _Pattern(int(n), int(ei.shape[0]), _np_ptr(ei), _np_ptr(ej))
    nfill, p, nvert = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    _check(L.cdcs_chordal_extension(ctypes.byref(pat), ctypes.byref(nfill), ctypes.byref(p), ctypes.byref(nvert),
                                    None, None, None, None), "cdcs_chordal_extension")
    fi = np.empty(nfill.value, dtype=np.int32)
    fj = np.empty(nfill.value, dtype=np.int32)
    cptr = np.empty(p.value + 1, dtype=np.int64)
    cvert = np.empty(nvert.value, dtype=np.int32)
    _check(L.cdcs_chordal_extension(ctypes.byref(pat), ctypes.byref(nfill), ctypes.byref(p), ctypes.byref(nvert),
                                    _np_ptr(fi), _np_ptr(fj), _np_ptr(cptr), _np_ptr(cvert)),
           "cdcs_chordal_extension")
    return fi, fj, cptr, cvert


def packed_offsets(sizes) -> np.ndarray:
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.zeros(sizes.shape[0] + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes * (sizes + 1) // 2)
    return off


def psd_project_batched(W, sizes, offsets=None, smax=None, eig: bool = False, stream=None):
    """P(W_k) for a packed batch of symmetric blocks (device tensors).

    W: float32 cuda tensor of packed lower triangles; sizes: int32 cuda tensor
    (or host array); offsets: int64 cuda tensor of nb+1 packed offsets.
    Returns P (and eigenvalues / eigenvector matrices when eig=True)."""
    torch = _torch()
    dev = W.device
    if isinstance(sizes, torch.Tensor) and sizes.is_cuda and not eig:
        # device-resident sizes/offsets: no host round trip (smax and offsets required)
        if smax is None or offsets is None:
            raise CdcsError(E_ARG, "device sizes need smax and device offsets")
        sizes_d = sizes
        nb = int(sizes.shape[0])
    else:
        sizes_h = np.asarray(sizes.cpu() if hasattr(sizes, "cpu") else sizes, dtype=np.int64)
        nb = int(sizes_h.shape[0])
        if smax is None:
            smax = int(sizes_h.max()) if nb else 1
        if nb and (sizes_h.min() < 1 or sizes_h.max() > MAX_BATCHED_CLIQUE):
            raise CdcsError(E_ARG, f"block sizes must lie in 1..{MAX_BATCHED_CLIQUE}")
        sizes_d = torch.as_tensor(sizes_h.astype(np.int32), device=dev)
        if offsets is None:
            offsets = torch.as_tensor(packed_offsets(sizes_h), device=dev)
    W = W.contiguous()
    P = torch.empty_like(W)
    evals = evecs = eoff = voff = None
    if eig:
        eo = np.zeros(nb + 1, dtype=np.int64)
        eo[1:] = np.cumsum(sizes_h)
        vo = np.zeros(nb + 1, dtype=np.int64)
        vo[1:] = np.cumsum(sizes_h * sizes_h)
        eoff = torch.as_tensor(eo, device=dev)
        voff = torch.as_tensor(vo, device=dev)
        evals = torch.empty(int(eo[-1]), dtype=torch.float32, device=dev)
        evecs = torch.empty(int(vo[-1]), dtype=torch.float32, device=dev)
    st = load_library().cdcs_psd_project_batched(nb, int(smax), _ptr(sizes_d), _ptr(offsets), _ptr(W), _ptr(P),
                                                 _ptr(evals), _ptr(eoff), _ptr(evecs), _ptr(voff),
                                                 _stream(torch, stream))
    _check(st, "cdcs_psd_project_batched")
    if eig:
        return P, evals, evecs, eoff, voff
    return P


def psd_project_vjp(gP, evals, evecs, eoff, voff, sizes_d, offsets_d, smax: int, stream=None):
    """Cotangent of W from the cotangent of P (Daleckii-Krein), packed FP32."""
    torch = _torch()
    gP = gP.contiguous()
    gW = torch.empty_like(gP)
    st = load_library().cdcs_psd_project_vjp(int(sizes_d.shape[0]), int(smax), _ptr(sizes_d), _ptr(offsets_d),
                                             _ptr(evals), _ptr(eoff), _ptr(evecs), _ptr(voff), _ptr(gP),
                                             _ptr(gW), _stream(torch, stream))
    _check(st, "cdcs_psd_project_vjp")
    return gW


def psd_project_plain(W, sizes_d, offsets_d, sizes_h, P=None, stream=None):
    """The clique-per-launch form: the same projection kernel launched once per
    block with a one-workgroup grid of the block's own size bucket (no
    graph).  Baseline for the batched form."""
    torch = _torch()
    L = load_library()
    P = torch.empty_like(W) if P is None else P
    s = _stream(torch, stream)
    sizes_h = np.asarray(sizes_h, dtype=np.int64)
    nb = int(sizes_d.shape[0])
    sp, op, wp, pp = sizes_d.data_ptr(), offsets_d.data_ptr(), W.data_ptr(), P.data_ptr()
    fn = L.cdcs_psd_project_batched
    for t in range(nb):
        st = fn(1, int(sizes_h[t]), ctypes.c_void_p(sp + 4 * t), ctypes.c_void_p(op + 8 * t), ctypes.c_void_p(wp),
                ctypes.c_void_p(pp), None, None, None, None, s)
        if st != OK:
            _check(st, "cdcs_psd_project_batched")
    return P


def pack_blocks(blocks) -> np.ndarray:
    """Full symmetric blocks -> packed lower triangles (row-major), layout only."""
    out = []
    for B in blocks:
        ia, ib = np.tril_indices(B.shape[0])
        out.append(np.asarray(B)[ia, ib])
    return np.concatenate(out) if out else np.zeros(0)


def unpack_blocks(packed, sizes, offsets=None):
    """Packed lower triangles -> list of full symmetric numpy blocks, layout only."""
    packed = np.asarray(packed)
    sizes = np.asarray(sizes, dtype=np.int64)
    if offsets is None:
        offsets = packed_offsets(sizes)
    blocks = []
    for t, s in enumerate(sizes):
        s = int(s)
        B = np.zeros((s, s), dtype=packed.dtype)
        ia, ib = np.tril_indices(s)
        vals = packed[offsets[t]:offsets[t] + s * (s + 1) // 2]
        B[ia, ib] = vals
        B[ib, ia] = vals
        blocks.append(B)
    return blocks
