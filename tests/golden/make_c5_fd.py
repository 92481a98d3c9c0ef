"""Write c5_fd.json: FP64 central finite differences of the oracle's unrolled
Algorithm 1 (block-arrow l=100, d=16, h=8, m=800; K = 100 iterations from zero
state, rho = 1) for the losses <C, X_K> and ||X_K - X_target||_F^2
(X_target = X0 of the generator), along 20 unit directions in c and 20 in b,
steps 1e-6 and 1e-5, together with the oracle's reverse-mode directional
derivatives.  The difference between the two steps bounds the FD error: the
FP64 forward carries ~5e-13 relative noise (iterative eigensolver), which at
step 1e-6 is comparable to the small directional derivatives of <C, X_K>.

Calls only oracle/ and the seeded input generators.
usage: python tests/golden/make_c5_fd.py [workers]
"""
import json
import os
import sys
import time
from multiprocessing import get_context

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1609_06068_amd import synth  # noqa: E402

K, RHO, NDIR = 100, 1.0, 20
STEPS = (1e-6, 1e-5)
SEED_C, SEED_B = 5001, 5002

_o = None


def _init():
    global _o
    _o = O.Oracle(synth.c5())


def _losses(c, b):
    prob = _o.prob
    x = O.Unrolled(_o, K=K, rho=RHO).forward(c, b)
    d = x - prob.meta["x0"]
    return float(np.sum(_o.dec.w * c * x)), float(np.sum(_o.dec.w * d * d))


def _fd(job):
    kind, i, vec, H = job
    prob = _o.prob
    vec = np.asarray(vec)
    if kind == "c":
        lp = _losses(prob.c + H * vec, prob.b)
        lm = _losses(prob.c - H * vec, prob.b)
    else:
        lp = _losses(prob.c, prob.b + H * vec)
        lm = _losses(prob.c, prob.b - H * vec)
    return kind, i, H, [(lp[0] - lm[0]) / (2 * H), (lp[1] - lm[1]) / (2 * H)]


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    t0 = time.time()
    prob = synth.c5()
    dc = synth.unit_directions(prob.nU, NDIR, SEED_C)
    db = synth.unit_directions(prob.m, NDIR, SEED_B)
    o = O.Oracle(prob)
    U = O.Unrolled(o, K=K, rho=RHO)
    x = U.forward(prob.c, prob.b)
    adj = {}
    for name, (L, g) in {"linear": O.loss_linear(prob, o.dec, x),
                         "target": O.loss_target(o.dec, x, prob.meta["x0"])}.items():
        cbar, bbar = U.backward(g)
        if name == "linear":
            cbar = cbar + o.dec.w * x
        adj[name] = {"loss": L, "dc": (dc @ cbar).tolist(), "db": (db @ bbar).tolist()}
    jobs = [(kd, i, (dc if kd == "c" else db)[i].tolist(), H) for H in STEPS for kd in ("c", "b")
            for i in range(NDIR)]
    fd = {H: {"c": [None] * NDIR, "b": [None] * NDIR} for H in STEPS}
    with get_context("fork").Pool(workers, initializer=_init) as pool:
        for kind, i, H, vals in pool.imap_unordered(_fd, jobs):
            fd[H][kind][i] = vals
    out = {"workload": "block-arrow l=100 d=16 h=8 m=800, Algorithm 1, K=100, rho=1, zero start",
           "steps": list(STEPS), "directions": NDIR, "seed_c": SEED_C, "seed_b": SEED_B,
           "min_abs_eig_over_norm": U.min_abs_eig,
           "fd": {f"{H:g}": {"linear": {"dc": [v[0] for v in fd[H]["c"]], "db": [v[0] for v in fd[H]["b"]]},
                             "target": {"dc": [v[1] for v in fd[H]["c"]], "db": [v[1] for v in fd[H]["b"]]}}
                  for H in STEPS},
           "oracle_adjoint": adj, "seconds": time.time() - t0}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_fd.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k in ("seconds", "min_abs_eig_over_norm")}))


if __name__ == "__main__":
    main()
