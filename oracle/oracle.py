"""CPU FP64 oracle for chordally decomposed ADMM on sparse SDPs.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library: the index maps, the KKT factor, the eigensolver and the
iteration are all re-derived here from the paper (Zheng, Fantuzzi,
Papachristodoulou, Goulart, Wynn, "Fast ADMM for Semidefinite Programs with
Chordal Sparsity", arXiv:1609.06068).

Coordinates.  A symmetric matrix X on the aggregate pattern is held by its
values on the lower-triangular pattern entries e = (i, j), i >= j.  The paper's
vec(X) holds every off-diagonal value twice, so with w_e = 1 (diagonal) or 2
(off-diagonal) every vec inner product <u, v> equals sum_e w_e u_e v_e, and the
vec norm is the w-weighted norm.  H_k x (= vec(E_k X E_k^T), Sec. III-A) is the
|C_k| x |C_k| submatrix; H_k^T applied to a clique matrix adds each of its
lower-triangular values to the matching entry; D = sum_k H_k^T H_k is the
per-entry count of cliques covering the entry (Sec. III-B.1).  A brute-force
test checks this against the literal vec/Kronecker form on small instances.

Floating point: FP64 throughout.  Own cyclic Jacobi eigensolver and own dense
Cholesky (C, no LAPACK); numpy matrix products serve as plain library steps.

Readings of the paper taken here (each is also listed in the design notes):
  * A is the m x n^2 matrix with rows vec(A_1) .. vec(A_m) (the printed A_0 is
    a typo: the operators use A_1..A_m);
  * the relative residuals (the paper defers to Boyd et al. 2011, Sec. 3.3):
      Alg. 1: eps_p = ||x_k - H_k x|| / max(||H_k x||, ||x_k||),
              eps_d = rho ||sum_k H_k^T (x_k - x_k^prev)|| / ||sum_k H_k^T lam_k||;
      Alg. 2: eps_p = ||z_k - v_k|| / max(||z_k||, ||v_k||),
              eps_d = rho ||v_k - v_k^prev|| / ||lam_k||;
    norms over all cliques stacked; a zero denominator leaves the numerator;
  * fixed rho (default 1), zero initial guesses (also v_k = 0 in Alg. 2);
  * Alg. 2 uses the unsubstituted multiplier update lam += rho (z - v); the
    printed shortcut lam = rho H_k x has the wrong sign (it is -rho H_k x,
    checked by a test).

Vector cones (CDCS's other cone types, Sec. IV: free, nonnegative orthant,
second-order cone) sit on the diagonal entries of vertices that lie in no
clique; each is one more block of the decomposition with H_k selecting its
entries (D_e = 1 on them).  Algorithm 1 projects onto the cones, Algorithm 2
onto their dual cones (the free cone's dual cone is {0}).  The homogeneous
self-dual embedding (the variant the paper names as future work, Sec. VI) is
the class Hsde below; its readings are in its docstring.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "cdcs_oracle.c")

OK, E_ARG, E_RANK, E_NUMERIC = 0, 1, 3, 7


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (-O3, OpenMP over independent
    cliques and Cholesky rows; no -march=native, because the library built
    here also runs on other hosts)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-std=c99", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_int64)
        L.oracle_jacobi_eigh.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, ip]
        L.oracle_psd_project.argtypes = [ctypes.c_int, dp, dp, dp, dp]
        L.oracle_psd_project_batch.argtypes = [ctypes.c_int, lp, lp, dp, dp, ip]
        L.oracle_psd_project_batch_eig.argtypes = [ctypes.c_int, lp, lp, lp, dp, dp, dp, dp]
        L.oracle_cholesky.argtypes = [ctypes.c_int, dp, dp]
        L.oracle_chol_solve.argtypes = [ctypes.c_int, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _lp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


class OracleError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


# --------------------------------------------------------------------------
# Dense kernels (C): eigendecomposition, PSD projection, Cholesky
# --------------------------------------------------------------------------

def jacobi_eigh(W: np.ndarray, max_sweeps: int = 100):
    """W = V diag(evals) V^T by cyclic-by-row Jacobi.  Returns (evals, V, sweeps)."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    k = W.shape[0]
    ev = np.empty(k)
    V = np.empty((k, k))
    sw = ctypes.c_int(0)
    st = lib().oracle_jacobi_eigh(k, _dp(W), _dp(ev), _dp(V), max_sweeps, ctypes.byref(sw))
    if st != OK:
        raise OracleError(st, "Jacobi did not converge")
    return ev, V, sw.value


def psd_project(W: np.ndarray) -> np.ndarray:
    """Projection onto the PSD cone, P(W) = V max(Lambda, 0) V^T
    (equations (E:XkUpdate), (E:zkUpdate))."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    k = W.shape[0]
    P = np.empty((k, k))
    st = lib().oracle_psd_project(k, _dp(W), _dp(P), None, None)
    if st != OK:
        raise OracleError(st, "Jacobi did not converge")
    return P


def psd_project_batch(blocks: list[np.ndarray]) -> list[np.ndarray]:
    """Independent projections of a list of symmetric matrices (one per clique)."""
    sizes = np.array([b.shape[0] for b in blocks], dtype=np.int64)
    off = np.zeros(len(blocks) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes * sizes)
    W = np.empty(off[-1])
    for t, b in enumerate(blocks):
        W[off[t]:off[t + 1]] = b.ravel()
    P = np.empty_like(W)
    status = np.zeros(len(blocks), dtype=np.int32)
    st = lib().oracle_psd_project_batch(len(blocks), _lp(sizes), _lp(off), _dp(W), _dp(P), _ip(status))
    if st != OK:
        raise OracleError(st, "Jacobi did not converge")
    return [P[off[t]:off[t + 1]].reshape(sizes[t], sizes[t]) for t in range(len(blocks))]


def psd_project_batch_eig(blocks: list[np.ndarray]):
    """As psd_project_batch, also returning each block's eigenvalues and
    eigenvectors (columns of V)."""
    sizes = np.array([b.shape[0] for b in blocks], dtype=np.int64)
    off = np.zeros(len(blocks) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes * sizes)
    eoff = np.zeros(len(blocks) + 1, dtype=np.int64)
    eoff[1:] = np.cumsum(sizes)
    W = np.empty(off[-1])
    for t, b in enumerate(blocks):
        W[off[t]:off[t + 1]] = b.ravel()
    P = np.empty_like(W)
    V = np.empty_like(W)
    ev = np.empty(eoff[-1])
    st = lib().oracle_psd_project_batch_eig(len(blocks), _lp(sizes), _lp(off), _lp(eoff),
                                            _dp(W), _dp(P), _dp(ev), _dp(V))
    if st != OK:
        raise OracleError(st, "Jacobi did not converge")
    Ps = [P[off[t]:off[t + 1]].reshape(sizes[t], sizes[t]) for t in range(len(blocks))]
    evs = [ev[eoff[t]:eoff[t + 1]] for t in range(len(blocks))]
    Vs = [V[off[t]:off[t + 1]].reshape(sizes[t], sizes[t]) for t in range(len(blocks))]
    return Ps, evs, Vs


def soc_project(v: np.ndarray) -> np.ndarray:
    """Euclidean projection onto the second-order cone {(t, z): ||z|| <= t}:
    v itself inside the cone, 0 inside its polar (||z|| <= -t), otherwise
    ((t + ||z||) / 2) (1, z / ||z||) (Boyd and Vandenberghe, Convex
    Optimization, Exercise 8.3(c))."""
    v = np.asarray(v, dtype=np.float64)
    t, z = v[0], v[1:]
    nz = float(np.sqrt(np.sum(z * z)))
    if nz <= t:
        return v.copy()
    if nz <= -t:
        return np.zeros_like(v)
    a = 0.5 * (t + nz)
    return np.concatenate([[a], (a / nz) * z])


def vector_cone_project(kind: int, v: np.ndarray) -> np.ndarray:
    """Projection onto a vector cone: free (R^n: identity), nonnegative
    orthant (entrywise max(., 0)) or second-order cone (CDCS's cone types
    besides PSD, Sec. IV)."""
    if kind == 0:
        return np.asarray(v, dtype=np.float64).copy()
    if kind == 1:
        return np.maximum(v, 0.0)
    return soc_project(v)


def cholesky(M: np.ndarray) -> np.ndarray:
    """M = L L^T (lower L).  Raises OracleError(E_RANK) if M is not PD."""
    M = np.ascontiguousarray(M, dtype=np.float64)
    m = M.shape[0]
    L = np.empty((m, m))
    st = lib().oracle_cholesky(m, _dp(M), _dp(L))
    if st != OK:
        raise OracleError(st, "KKT Schur complement is not positive definite (A rank deficient)")
    return L


def chol_solve(L: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Solve L L^T y = t by forward then backward substitution."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    y = np.empty_like(t)
    lib().oracle_chol_solve(L.shape[0], _dp(L), _dp(t), _dp(y))
    return y


# --------------------------------------------------------------------------
# Chordal decomposition: E_k, H_k and D (Sections II-B, III-A, III-B.1)
# --------------------------------------------------------------------------

class Decomposition:
    """Entry selectors for each clique.

    idx[k] is the |C_k| x |C_k| table of entry positions of the submatrix
    E_k X E_k^T (both triangles point to the same lower-triangular entry).
    D[e] counts the cliques whose C_k x C_k contains e.
    """

    def __init__(self, prob):
        n = prob.n
        ei = np.asarray(prob.ei, dtype=np.int64)
        ej = np.asarray(prob.ej, dtype=np.int64)
        if np.any(ei < ej):
            raise OracleError(2, "pattern entries must be lower triangular")
        key = ei * n + ej
        if np.unique(key).shape[0] != key.shape[0]:
            raise OracleError(2, "duplicate pattern entry")
        order = np.argsort(key)
        skey = key[order]
        self.nU = key.shape[0]
        self.w = np.where(ei == ej, 1.0, 2.0)
        self.idx = []
        self.tril = []
        D = np.zeros(self.nU)
        for k in range(prob.p):
            cl = np.asarray(prob.clique(k), dtype=np.int64)
            if cl.shape[0] == 0 or np.any(np.diff(cl) <= 0) or cl[0] < 0 or cl[-1] >= n:
                raise OracleError(2, f"clique {k} not sorted / out of range")
            s = cl.shape[0]
            I = np.maximum(cl[:, None], cl[None, :])
            J = np.minimum(cl[:, None], cl[None, :])
            q = (I * n + J).ravel()
            pos = np.searchsorted(skey, q)
            pos = np.minimum(pos, self.nU - 1)
            if np.any(skey[pos] != q):
                raise OracleError(2, f"clique {k} pair missing from the pattern")
            tab = order[pos].reshape(s, s)
            self.idx.append(tab)
            ia, ib = np.tril_indices(s)
            self.tril.append((ia, ib))
            np.add.at(D, tab[ia, ib], 1.0)
        # vector cones: each covers the diagonal entries of its vertices, which
        # lie in no clique and in no other cone and have no off-diagonal entry
        self.p = prob.p
        self.vidx, self.vkind = [], []
        in_clique = np.zeros(n, dtype=bool)
        if prob.p > 0:
            in_clique[np.asarray(prob.clique_vert, dtype=np.int64)] = True
        offdiag_v = np.zeros(n, dtype=bool)
        offdiag_v[ei[ei != ej]] = True
        offdiag_v[ej[ei != ej]] = True
        for q in range(prob.ncones):
            vs = np.asarray(prob.cone(q), dtype=np.int64)
            kind = int(prob.cone_kind[q])
            if vs.shape[0] == 0 or kind not in (0, 1, 2) or (kind == 2 and vs.shape[0] < 2):
                raise OracleError(2, f"vector cone {q}: empty, unknown kind or a one-vertex second-order cone")
            if np.any(vs < 0) or np.any(vs >= n) or np.any(in_clique[vs]) or np.any(offdiag_v[vs]):
                raise OracleError(2, f"vector cone {q}: vertex out of range, in a clique or with off-diagonal entries")
            pos = np.minimum(np.searchsorted(skey, vs * n + vs), self.nU - 1)
            if np.any(skey[pos] != vs * n + vs):
                raise OracleError(2, f"vector cone {q}: diagonal entry missing from the pattern")
            ent = order[pos]
            if np.any(D[ent] != 0):
                raise OracleError(2, f"vector cone {q}: entry already covered")
            D[ent] = 1.0
            self.vidx.append(ent)
            self.vkind.append(kind)
        self.ncones = self.p + len(self.vidx)
        if np.any(D == 0):
            raise OracleError(2, "pattern entry covered by no clique or cone")
        self.D = D

    def gather(self, x: np.ndarray, k: int) -> np.ndarray:
        """H_k x: the clique submatrix E_k X E_k^T (k < p), or the vector of a
        vector cone's entries (k >= p)."""
        if k >= self.p:
            return x[self.vidx[k - self.p]]
        return x[self.idx[k]]

    def scatter(self, blocks) -> np.ndarray:
        """sum_k H_k^T vec(B_k) in entry coordinates (cliques, then vector cones)."""
        out = np.zeros(self.nU)
        for k, B in enumerate(blocks):
            if k >= self.p:
                np.add.at(out, self.vidx[k - self.p], B)
                continue
            ia, ib = self.tril[k]
            np.add.at(out, self.idx[k][ia, ib], B[ia, ib])
        return out

    def zero_blocks(self):
        return ([np.zeros(t.shape) for t in self.idx] + [np.zeros(v.shape[0]) for v in self.vidx])

    def project(self, W: list, dual: bool = False) -> list:
        """Projection of every cone block onto its cone (dual=False) or onto
        its dual cone (dual=True): the PSD projection for cliques (self-dual),
        the vector cones' own projections after them (the free cone's dual
        cone is {0}; the orthant and the second-order cone are self-dual)."""
        out = psd_project_batch(W[:self.p]) if self.p > 0 else []
        for q, kind in enumerate(self.vkind):
            if dual and kind == 0:
                out.append(np.zeros_like(W[self.p + q]))
            else:
                out.append(vector_cone_project(kind, W[self.p + q]))
        return out

    def wdot(self, u, v) -> float:
        return float(np.sum(self.w * u * v))

    def wnorm(self, u) -> float:
        return float(np.sqrt(np.sum(self.w * u * u)))


def _stack_norm(blocks) -> float:
    return float(np.sqrt(sum(float(np.sum(B * B)) for B in blocks)))


def _rel(num, den):
    return num / den if den > 0 else num


# --------------------------------------------------------------------------
# Affine projection: the KKT systems (E:OptCondMinYPrimal) / (E:OptCondMinYDual)
# --------------------------------------------------------------------------

class KKT:
    """Solve [D A^T; A 0][x; y] = [r1; r2] by block elimination with a cached
    Cholesky factor (Sec. III-B.1; the same matrix serves Alg. 2).

    In entry coordinates the first block row reads D_e x_e + (A^T y)_e = r1_e
    and the second sum_e w_e A_ie x_e = r2_i, so
        M = A diag(w / D) A^T,  M y = A (w * r1 / D) - r2,  x = (r1 - A^T y) / D.
    """

    def __init__(self, prob, dec: Decomposition):
        if prob.A is not None:
            self.A = np.asarray(prob.A, dtype=np.float64)
        else:
            import scipy.sparse as sp
            self.A = sp.csr_matrix((prob.A_val, prob.A_idx.astype(np.int64), prob.A_ptr),
                                   shape=(prob.m, dec.nU))
        self.D = dec.D
        self.w = dec.w
        sc = self.w / self.D
        if isinstance(self.A, np.ndarray):
            M = (self.A * sc[None, :]) @ self.A.T
        else:
            import scipy.sparse as sp
            M = (self.A @ sp.diags(sc) @ self.A.T).toarray()
        self.M = 0.5 * (M + M.T)
        self.L = cholesky(self.M)

    def solve(self, r1: np.ndarray, r2: np.ndarray):
        t = self.A @ (self.w * r1 / self.D) - r2
        y = chol_solve(self.L, t)
        x = (r1 - self.A.T @ y) / self.D
        return x, y


# --------------------------------------------------------------------------
# Algorithms 1 and 2
# --------------------------------------------------------------------------

@dataclass
class Result:
    form: str
    iters: int
    converged: bool
    x: np.ndarray            # global x (entry coordinates)
    y: np.ndarray            # KKT multiplier y of the last affine step
    blocks: list             # x_k (Alg. 1) or z_k (Alg. 2), full clique matrices
    lam: list                # lambda_k
    v: list | None           # v_k (Alg. 2)
    eps_p: list = field(default_factory=list)
    eps_d: list = field(default_factory=list)
    X_sdp: np.ndarray | None = None   # primal SDP variable on the entries
    y_sdp: np.ndarray | None = None   # dual SDP multiplier
    Z_sdp: np.ndarray | None = None   # dual slack on the entries
    obj_primal: float = 0.0
    obj_dual: float = 0.0


class Oracle:
    def __init__(self, prob):
        self.prob = prob
        self.dec = Decomposition(prob)
        self.kkt = KKT(prob, self.dec)
        self.sizes = [int(s) for s in prob.clique_sizes()]

    def zero_blocks(self):
        return self.dec.zero_blocks()

    # ---- Algorithm 1: decomposed primal form ------------------------------
    def admm_primal(self, rho=1.0, max_iter=200, tol=0.0, xk=None, lam=None, callback=None) -> Result:
        dec, kkt, prob = self.dec, self.kkt, self.prob
        c, b = prob.c, prob.b
        xk = self.zero_blocks() if xk is None else [B.copy() for B in xk]
        lam = self.zero_blocks() if lam is None else [B.copy() for B in lam]
        res = Result("primal", 0, False, None, None, xk, lam, None)
        nc = dec.ncones
        for it in range(1, max_iter + 1):
            # X-block: (E:OptCondMinYPrimal)
            r1 = dec.scatter([xk[k] + lam[k] / rho for k in range(nc)]) - c / rho
            x, y = kkt.solve(r1, b)
            # Y-block: (E:XkUpdate), one PSD projection per clique (and one
            # projection per vector cone)
            Hx = [dec.gather(x, k) for k in range(nc)]
            W = [Hx[k] - lam[k] / rho for k in range(nc)]
            xk_new = dec.project(W)
            # Z-block: (E:LambdakUpdate)
            lam = [lam[k] + rho * (xk_new[k] - Hx[k]) for k in range(nc)]
            # relative residuals
            rp = _stack_norm([xk_new[k] - Hx[k] for k in range(nc)])
            eps_p = _rel(rp, max(_stack_norm(Hx), _stack_norm(xk_new)))
            s = rho * dec.scatter([xk_new[k] - xk[k] for k in range(nc)])
            eps_d = _rel(dec.wnorm(s), dec.wnorm(dec.scatter(lam)))
            xk = xk_new
            res.eps_p.append(eps_p)
            res.eps_d.append(eps_d)
            res.iters = it
            if callback is not None:
                callback(it, x, y, xk, lam)
            if max(eps_p, eps_d) <= tol:
                res.converged = True
                break
        res.x, res.y, res.blocks, res.lam = x, y, xk, lam
        res.X_sdp = x
        res.y_sdp = -rho * y
        res.Z_sdp = dec.scatter(lam)
        res.obj_primal = dec.wdot(c, x)
        res.obj_dual = float(np.dot(b, res.y_sdp))
        return res

    # ---- Algorithm 2: decomposed dual form --------------------------------
    def admm_dual(self, rho=1.0, max_iter=200, tol=0.0, z=None, v=None, lam=None, callback=None) -> Result:
        dec, kkt, prob = self.dec, self.kkt, self.prob
        c, b = prob.c, prob.b
        z = self.zero_blocks() if z is None else [B.copy() for B in z]
        v = self.zero_blocks() if v is None else [B.copy() for B in v]
        lam = self.zero_blocks() if lam is None else [B.copy() for B in lam]
        res = Result("dual", 0, False, None, None, z, lam, v)
        nc = dec.ncones
        for it in range(1, max_iter + 1):
            # Y-block first: (E:zkUpdate)
            z = dec.project([v[k] - lam[k] / rho for k in range(nc)], dual=True)
            # X-block: (E:OptCondMinYDual), then (E:vkEqn)
            r1 = c - dec.scatter([z[k] + lam[k] / rho for k in range(nc)])
            x, y = kkt.solve(r1, -b / rho)
            v_new = [z[k] + lam[k] / rho + dec.gather(x, k) for k in range(nc)]
            # Z-block: (E:MultUpdateDualSDP)
            lam = [lam[k] + rho * (z[k] - v_new[k]) for k in range(nc)]
            rp = _stack_norm([z[k] - v_new[k] for k in range(nc)])
            eps_p = _rel(rp, max(_stack_norm(z), _stack_norm(v_new)))
            eps_d = _rel(rho * _stack_norm([v_new[k] - v[k] for k in range(nc)]), _stack_norm(lam))
            v = v_new
            res.eps_p.append(eps_p)
            res.eps_d.append(eps_d)
            res.iters = it
            if callback is not None:
                callback(it, x, y, z, lam)
            if max(eps_p, eps_d) <= tol:
                res.converged = True
                break
        res.x, res.y, res.blocks, res.lam, res.v = x, y, z, lam, v
        res.y_sdp = y
        res.Z_sdp = dec.scatter(z)
        res.X_sdp = -rho * x
        res.obj_dual = float(np.dot(b, y))
        res.obj_primal = dec.wdot(c, res.X_sdp)
        return res

    def solve(self, form="primal", **kw) -> Result:
        return self.admm_primal(**kw) if form == "primal" else self.admm_dual(**kw)

    # ---- optimality measures of the original SDP (Sec. I) -----------------
    def sdp_kkt_residuals(self, res: Result):
        """Relative primal infeasibility, dual infeasibility and duality gap of
        (X_sdp, y_sdp, Z_sdp) for the SDP pair (E:PrimalSDP)/(E:DualSDP), plus
        the smallest clique eigenvalue of X and of the Z_k blocks."""
        dec, prob = self.dec, self.prob
        A = self.kkt.A
        X, y, Z = res.X_sdp, res.y_sdp, res.Z_sdp
        AX = A @ (dec.w * X)
        pinf = np.linalg.norm(AX - prob.b) / (1.0 + np.linalg.norm(prob.b))
        dres = A.T @ y + Z - prob.c
        dinf = dec.wnorm(dres) / (1.0 + dec.wnorm(prob.c))
        pobj = dec.wdot(prob.c, X)
        dobj = float(np.dot(prob.b, y))
        gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
        zblocks = res.lam if res.form == "primal" else res.blocks
        xmin = min(cone_margin(dec, k, dec.gather(X, k)) for k in range(dec.ncones))
        zmin = min(cone_margin(dec, k, zblocks[k], dual=True) for k in range(dec.ncones))
        return dict(pinf=pinf, dinf=dinf, gap=gap, pobj=pobj, dobj=dobj, xmin=xmin, zmin=zmin)


def cone_margin(dec: Decomposition, k: int, B, dual: bool = False) -> float:
    """How far B lies inside cone k (negative: outside): the smallest
    eigenvalue (PSD), the smallest entry (orthant), t - ||z|| (second-order
    cone); the free cone always holds (+inf) and its dual cone {0} holds to
    -max |B|."""
    if k < dec.p:
        return float(np.linalg.eigvalsh(B).min())
    kind = dec.vkind[k - dec.p]
    B = np.asarray(B, dtype=np.float64)
    if kind == 0:
        return -float(np.abs(B).max()) if dual else float("inf")
    if kind == 1:
        return float(B.min())
    return float(B[0] - np.linalg.norm(B[1:]))


# --------------------------------------------------------------------------
# Homogeneous self-dual embedding of the decomposed problem (the HSDE variant
# the paper names as future work, Sec. VI, following O'Donoghue, Chu, Parikh
# and Boyd 2016, "Conic optimization via operator splitting and homogeneous
# self-dual embedding")
# --------------------------------------------------------------------------

HSDE_SOLVED, HSDE_MAXIT, HSDE_NUMERIC, HSDE_INFEASIBLE, HSDE_UNBOUNDED = 1, 2, 3, 4, 5


@dataclass
class HsdeResult:
    iters: int
    status: int              # 0 running (max_iter not reached), 1 solved, 2 cap, 4 primal infeasible, 5 dual infeasible
    x: np.ndarray            # u_x (entries)
    y: np.ndarray            # u_y on the equality rows
    z: list                  # u_y on the cone rows (one block per cone)
    s: list                  # v_s on the cone rows
    tau: float
    kappa: float
    res_pri: list = field(default_factory=list)
    res_dual: list = field(default_factory=list)
    gap: list = field(default_factory=list)
    X_sdp: np.ndarray | None = None
    y_sdp: np.ndarray | None = None
    Z_sdp: np.ndarray | None = None
    obj_primal: float = 0.0
    obj_dual: float = 0.0
    cert_y: np.ndarray | None = None   # primal infeasible: A*(y) in -K*, b^T y = 1
    cert_x: np.ndarray | None = None   # dual infeasible: A(x) = 0, x in K, <c, x> = -1


class Hsde:
    """The decomposed primal problem min <c, x>_w s.t. A(x) = b, H_k x = x_k in
    K_k, written as the conic program min <c, x> s.t. Ahat x + s = bhat,
    s in {0}^m x K_1 x ... x K_p with Ahat = [A; -H_1; ...; -H_p] and
    bhat = (b, 0, ..., 0), and embedded homogeneously:
        Q = [[0, Ahat^T, c], [-Ahat, 0, bhat], [-c^T, -bhat^T, 0]],
        u = (x, y, z, tau) in R^nU x (R^m x K*) x R_+,  v = Q u = (0, 0, s, kappa).
    The iteration (no over-relaxation) is
        ut = (I + Q)^-1 (u + v),  u = Pi(ut - v),  v = v - ut + u.
    All inner products on the entries are w-weighted (vec coordinates), so
    the adjoint of A is (A^T y)_e = sum_i A_ie y_i and H_k^T H_k sums to D.

    The linear system: with M = [[I, Ahat^T], [-Ahat, I]] and h = (c, bhat),
    (I + Q) ut = w splits into M zeta = w_xy, M g = h (g cached) and
    ut_tau = (w_tau + h^T zeta) / (1 + h^T g), ut_xy = zeta - ut_tau g.
    M (a, b) = (r_x, r_y) is solved by eliminating b = r_y + Ahat a:
    (I + D + A^T A) a = r_x - Ahat^T r_y, and with E = 1 + D that system is
    solved through the m x m matrix M' = I + A diag(w / E) A^T (cached
    Cholesky factor): p = r_x + sum_k H_k^T r_k, t = A(w p / E) + r_0,
    y' = M'^-1 t, a = (p - A^T y') / E, b_0 = y', b_k = r_k - H_k a.

    Termination (readings: the paper gives none for this variant; these are
    the scaled residuals of the reference above, relative to 1 + ||b|| and
    1 + ||c||), at an iterate with tau > 0:
        res_pri  = ||(A(x) - tau b, s_k - H_k x)|| / (tau (1 + ||b||)),
        res_dual = ||A^T y - sum_k H_k^T z_k + tau c||_w / (tau (1 + ||c||_w)),
        gap      = |<c, x>_w + b^T y| / (tau + |<c, x>_w| + |b^T y|),
    solved when all three are <= tol; primal infeasible (certificate
    -y / (-b^T y)) when b^T y < 0 and ||A^T y - sum_k H_k^T z_k||_w ||b|| <=
    tol (-b^T y); dual infeasible (certificate x / (-<c, x>_w)) when
    <c, x>_w < 0 and ||(A(x), s_k - H_k x)|| ||c||_w <= tol (-<c, x>_w).
    Checked in that order after every iteration.
    """

    def __init__(self, prob):
        self.prob = prob
        self.dec = dec = Decomposition(prob)
        if prob.A is not None:
            self.A = np.asarray(prob.A, dtype=np.float64)
        else:
            import scipy.sparse as sp
            self.A = sp.csr_matrix((prob.A_val, prob.A_idx.astype(np.int64), prob.A_ptr), shape=(prob.m, dec.nU))
        self.E = 1.0 + dec.D
        sc = dec.w / self.E
        if isinstance(self.A, np.ndarray):
            Mp = (self.A * sc[None, :]) @ self.A.T
        else:
            import scipy.sparse as sp
            Mp = (self.A @ sp.diags(sc) @ self.A.T).toarray()
        Mp = 0.5 * (Mp + Mp.T) + np.eye(prob.m)
        self.L = cholesky(Mp)
        self.gx, self.gy, self.gz = self.solve_m(prob.c, prob.b, dec.zero_blocks())
        self.hg = dec.wdot(prob.c, self.gx) + float(np.dot(prob.b, self.gy))
        self.nb = float(np.linalg.norm(prob.b))
        self.nc = dec.wnorm(prob.c)

    def A_op(self, x):
        """A(x) = [<A_i, X>] = sum_e w_e A_ie x_e."""
        return self.A @ (self.dec.w * x)

    def AT_op(self, y):
        """The adjoint: (A^T y)_e = sum_i A_ie y_i."""
        return self.A.T @ y

    def solve_m(self, rx, ry, rz):
        """(a, b_0, b_k) with M (a, b) = (rx, (ry, rz))."""
        dec = self.dec
        p = rx + dec.scatter(rz)
        t = self.A_op(p / self.E) + ry
        y1 = chol_solve(self.L, t)
        a = (p - self.AT_op(y1)) / self.E
        bz = [rz[k] - dec.gather(a, k) for k in range(dec.ncones)]
        return a, y1, bz

    def solve_iq(self, wx, wy, wz, wt):
        """ut = (I + Q)^-1 w for w = (wx, wy, wz, wt)."""
        dec, prob = self.dec, self.prob
        za, zy, zz = self.solve_m(wx, wy, wz)
        ut = (wt + dec.wdot(prob.c, za) + float(np.dot(prob.b, zy))) / (1.0 + self.hg)
        return (za - ut * self.gx, zy - ut * self.gy, [zz[k] - ut * self.gz[k] for k in range(dec.ncones)], ut)

    def step(self, x, y, z, s, tau, kappa):
        """One iteration; returns the new (x, y, z, s, tau, kappa) and ut_tau."""
        dec = self.dec
        nc = dec.ncones
        # ut = (I + Q)^-1 (u + v); v is zero on the x and y rows
        ux, uy, uz, ut = self.solve_iq(x, y, [z[k] + s[k] for k in range(nc)], tau + kappa)
        # u = Pi_C(ut - v): x and y free, z onto the dual cones, tau >= 0
        z_new = dec.project([uz[k] - s[k] for k in range(nc)], dual=True)
        tau_new = max(ut - kappa, 0.0)
        # v = v - ut + u
        s_new = [s[k] - uz[k] + z_new[k] for k in range(nc)]
        kappa_new = kappa - ut + tau_new
        return ux, uy, z_new, s_new, tau_new, kappa_new, ut

    def initial(self):
        """u = (0, 0, 0, 1), v = (0, 0, 0, 1)."""
        dec = self.dec
        return (np.zeros(dec.nU), np.zeros(self.prob.m), dec.zero_blocks(), dec.zero_blocks(), 1.0, 1.0)

    def residuals(self, x, y, z, s, tau):
        dec, prob = self.dec, self.prob
        nc = dec.ncones
        Ax = self.A_op(x)
        cons = [s[k] - dec.gather(x, k) for k in range(nc)]
        r_cone = _stack_norm(cons)
        pri_nt = float(np.sqrt(np.sum((Ax - tau * prob.b) ** 2) + r_cone ** 2))
        ray_nt = float(np.sqrt(np.sum(Ax ** 2) + r_cone ** 2))
        aty = self.AT_op(y) - dec.scatter(z)
        dual_nt = dec.wnorm(aty + tau * prob.c)
        aty_n = dec.wnorm(aty)
        cx = dec.wdot(prob.c, x)
        by = float(np.dot(prob.b, y))
        return pri_nt, dual_nt, ray_nt, aty_n, cx, by

    def solve(self, max_iter=2000, tol=1e-6, state=None, callback=None) -> HsdeResult:
        dec, prob = self.dec, self.prob
        nc = dec.ncones
        x, y, z, s, tau, kappa = self.initial() if state is None else state
        z = [B.copy() for B in z]
        s = [B.copy() for B in s]
        res = HsdeResult(0, 0, x, y, z, s, tau, kappa)
        for it in range(1, max_iter + 1):
            x, y, z, s, tau, kappa, _ = self.step(x, y, z, s, tau, kappa)
            pri_nt, dual_nt, ray_nt, aty_n, cx, by = self.residuals(x, y, z, s, tau)
            if tau > 0:
                rp = pri_nt / (tau * (1.0 + self.nb))
                rd = dual_nt / (tau * (1.0 + self.nc))
            else:
                rp = rd = float("inf")
            gp = abs(cx + by) / (tau + abs(cx) + abs(by)) if tau + abs(cx) + abs(by) > 0 else 0.0
            res.res_pri.append(rp)
            res.res_dual.append(rd)
            res.gap.append(gp)
            res.iters = it
            if callback is not None:
                callback(it, x, y, z, s, tau, kappa)
            if not all(np.isfinite(v) for v in (pri_nt, dual_nt, cx, by, tau, kappa)):
                res.status = HSDE_NUMERIC
                break
            if tau > 0 and max(rp, rd, gp) <= tol:
                res.status = HSDE_SOLVED
                break
            if by < 0 and aty_n * self.nb <= tol * (-by):
                res.status = HSDE_INFEASIBLE
                break
            if cx < 0 and ray_nt * self.nc <= tol * (-cx):
                res.status = HSDE_UNBOUNDED
                break
        else:
            res.status = HSDE_MAXIT
        res.x, res.y, res.z, res.s, res.tau, res.kappa = x, y, z, s, tau, kappa
        if res.status == HSDE_INFEASIBLE:
            res.cert_y = y / float(np.dot(prob.b, y))
        elif res.status == HSDE_UNBOUNDED:
            res.cert_x = x / (-dec.wdot(prob.c, x))
        elif tau > 0:
            res.X_sdp = x / tau
            res.y_sdp = -y / tau
            res.Z_sdp = dec.scatter(z) / tau
            res.obj_primal = dec.wdot(prob.c, res.X_sdp)
            res.obj_dual = float(np.dot(prob.b, res.y_sdp))
        return res


# --------------------------------------------------------------------------
# Differentiating unrolled Algorithm 1 (reverse mode, FP64)
# --------------------------------------------------------------------------

def dk_gamma(lam: np.ndarray) -> np.ndarray:
    """First divided differences of f(t) = max(t, 0) at the eigenvalues
    (Daleckii-Krein): Gamma_ij = (f(l_i) - f(l_j)) / (l_i - l_j), with
    f'(l) = 1 for l > 0 and 0 for l <= 0 on ties (the derivative at 0 is taken
    as 0)."""
    li = lam[:, None]
    lj = lam[None, :]
    pi = np.maximum(li, 0.0)
    pj = np.maximum(lj, 0.0)
    both_pos = (li > 0) & (lj > 0)
    both_non = (li <= 0) & (lj <= 0)
    den = li - lj
    with np.errstate(divide="ignore", invalid="ignore"):
        mixed = (pi - pj) / den
    return np.where(both_pos, 1.0, np.where(both_non, 0.0, mixed))


def psd_project_vjp(lam: np.ndarray, V: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Adjoint of the Frechet derivative of P(W) = V max(L, 0) V^T at W (self-
    adjoint in the Frobenius product): V (Gamma o (V^T G V)) V^T, G symmetric."""
    B = V.T @ G @ V
    return V @ (dk_gamma(lam) * B) @ V.T


class Unrolled:
    """K iterations of Algorithm 1 from zero state, x_K as a function of
    (c, b), with its reverse-mode derivative.

    The forward keeps the state (x_k, lambda_k) before each iteration (the
    per-iteration checkpoint); the backward recomputes one iteration at a time.
    Coordinates are plain (unweighted) on the entry vectors and on full clique
    blocks; a loss L(x_K) supplies dL/dx_K in the same coordinates.
    """

    def __init__(self, orc: Oracle, K: int, rho: float = 1.0):
        self.o, self.K, self.rho = orc, K, rho

    def _iteration(self, xk, lam, c, b):
        o, rho, p = self.o, self.rho, self.o.prob.p
        r1 = o.dec.scatter([xk[k] + lam[k] / rho for k in range(p)]) - c / rho
        x, y = o.kkt.solve(r1, b)
        h = [o.dec.gather(x, k) for k in range(p)]
        W = [h[k] - lam[k] / rho for k in range(p)]
        P, evs, Vs = psd_project_batch_eig(W)
        lam_new = [lam[k] + rho * (P[k] - h[k]) for k in range(p)]
        return x, P, lam_new, (evs, Vs)

    def forward(self, c, b):
        p = self.o.prob.p
        xk = self.o.zero_blocks()
        lam = self.o.zero_blocks()
        self.ckpt = []
        self.min_abs_eig = np.inf
        x = None
        for _ in range(self.K):
            self.ckpt.append((xk, lam))
            x, xk, lam, (evs, Vs) = self._iteration(xk, lam, c, b)
            for k in range(p):
                nrm = np.linalg.norm(np.concatenate([xk[k].ravel(), lam[k].ravel()])) + 1e-300
                self.min_abs_eig = min(self.min_abs_eig, float(np.abs(evs[k]).min()) / nrm)
        self.c, self.b = c, b
        return x

    def _affine_adjoint(self, xbar):
        """(d x / d r1)^T xbar and (d x / d b)^T xbar via the same KKT solve:
        x = F(r1, b) gives r1bar = w F(xbar / w, 0) and bbar = y of that solve."""
        w = self.o.dec.w
        xo, yo = self.o.kkt.solve(xbar / w, np.zeros(self.o.prob.m))
        return w * xo, yo

    def backward(self, xbar_K):
        o, rho, p = self.o, self.rho, self.o.prob.p
        dec = o.dec
        cbar = np.zeros(dec.nU)
        bbar = np.zeros(o.prob.m)
        xkbar = [np.zeros_like(B) for B in self.ckpt[0][0]]
        lambar = [np.zeros_like(B) for B in self.ckpt[0][0]]
        for n in range(self.K - 1, -1, -1):
            xk_prev, lam_prev = self.ckpt[n]
            x, P, _, (evs, Vs) = self._iteration(xk_prev, lam_prev, self.c, self.b)
            # lambda_new = lambda + rho (P - h)
            Pbar = [xkbar[k] + rho * lambar[k] for k in range(p)]
            hbar = [-rho * lambar[k] for k in range(p)]
            lam_prev_bar = [lambar[k].copy() for k in range(p)]
            # P = proj(W), W = h - lambda / rho
            for k in range(p):
                G = 0.5 * (Pbar[k] + Pbar[k].T)
                Wbar = psd_project_vjp(evs[k], Vs[k], G)
                hbar[k] = hbar[k] + Wbar
                lam_prev_bar[k] = lam_prev_bar[k] - Wbar / rho
            # h = H_k x  (gather); its adjoint adds both triangles of each block
            xbar = np.zeros(dec.nU)
            for k in range(p):
                np.add.at(xbar, dec.idx[k].ravel(), hbar[k].ravel())
            if n == self.K - 1:
                xbar = xbar + xbar_K
            # x = F(r1, b)
            r1bar, bb = self._affine_adjoint(xbar)
            bbar += bb
            cbar += -r1bar / rho
            # r1 = sum_k H_k^T (x_k + lambda_k / rho) - c / rho (lower triangles)
            q = [np.zeros_like(B) for B in xk_prev]
            for k in range(p):
                ia, ib = dec.tril[k]
                q[k][ia, ib] = r1bar[dec.idx[k][ia, ib]]
            xkbar = q
            lambar = [lam_prev_bar[k] + q[k] / rho for k in range(p)]
        return cbar, bbar


def loss_linear(prob, dec, x):
    """<C, X> on the pattern (vec inner product) and its gradient in x."""
    return float(np.sum(dec.w * prob.c * x)), dec.w * prob.c


def loss_target(dec, x, xt):
    """||X - X_target||_F^2 on the pattern and its gradient in x."""
    d = x - xt
    return float(np.sum(dec.w * d * d)), 2.0 * dec.w * d
