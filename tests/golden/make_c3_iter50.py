"""Write c3_iter50.json: the oracle's iterates after 50 iterations of
Algorithm 1 and of Algorithm 2 (rho = 1, zero start) on the uneven-clique
workload (clique tree of 3000 cliques of 4..96 vertices, separators of 1..8,
m = 8000 sparse constraints of 20 coefficients), sampled: the global x on
1024 pattern entries and the clique blocks (x_k or z_k, lambda_k, and v_k for
Algorithm 2) on 1024 packed slots (clique k, row a >= column b), plus the RMS
of every sampled vector over all of its entries (the scale of the element-wise
tolerance), the residual histories and the objectives.  Samples are drawn
uniformly with a fixed seed.

Calls only oracle/ and the seeded input generators.
usage: python tests/golden/make_c3_iter50.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1609_06068_amd import synth  # noqa: E402

ITERS, RHO, NSAMP, SEED = 50, 1.0, 1024, 3050


def block_rms(blocks):
    return float(np.sqrt(sum(float(np.sum(B * B)) for B in blocks) / sum(B.size for B in blocks)))


def main():
    t0 = time.time()
    prob = synth.c3()
    o = O.Oracle(prob)
    print(f"oracle setup {time.time() - t0:.1f}s", flush=True)
    rng = np.random.default_rng(SEED)
    ents = np.sort(rng.choice(o.dec.nU, size=NSAMP, replace=False))
    sizes = np.asarray(o.sizes, dtype=np.int64)
    off = np.zeros(prob.p + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes * (sizes + 1) // 2)
    g = np.sort(rng.choice(int(off[-1]), size=NSAMP, replace=False))
    ks = np.searchsorted(off, g, side="right") - 1
    loc = g - off[ks]
    a = ((np.sqrt(8 * loc + 1) - 1) // 2).astype(np.int64)
    a -= (a * (a + 1) // 2 > loc)
    a += ((a + 1) * (a + 2) // 2 <= loc)
    b = loc - a * (a + 1) // 2
    assert np.all((b >= 0) & (b <= a) & (a < sizes[ks]))
    w = o.dec.w
    out = {"workload": "clique tree p=3000, sizes 4..96, separators 1..8, m=8000 sparse A (20 per row), "
                       "rho=1, zero start",
           "iterations": ITERS, "seed": SEED, "entries": ents.tolist(),
           "slots": {"clique": ks.tolist(), "a": a.tolist(), "b": b.tolist()}}
    for form in ("primal", "dual"):
        t1 = time.time()
        r = o.solve(form, rho=RHO, max_iter=ITERS)
        print(f"{form}: {ITERS} iterations in {time.time() - t1:.1f}s", flush=True)
        rec = {"x": r.x[ents].tolist(),
               "x_rms": float(np.sqrt(np.sum(w * r.x * r.x) / np.sum(w))),
               "blk": [float(r.blocks[k][i, j]) for k, i, j in zip(ks, a, b)],
               "blk_rms": block_rms(r.blocks),
               "lam": [float(r.lam[k][i, j]) for k, i, j in zip(ks, a, b)],
               "lam_rms": block_rms(r.lam),
               "eps_p": r.eps_p, "eps_d": r.eps_d,
               "obj_primal": r.obj_primal, "obj_dual": r.obj_dual}
        if form == "dual":
            rec["v"] = [float(r.v[k][i, j]) for k, i, j in zip(ks, a, b)]
            rec["v_rms"] = block_rms(r.v)
        out[form] = rec
    out["seconds"] = time.time() - t0
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_iter50.json"), "w") as fh:
        json.dump(out, fh)
    print(f"done in {out['seconds']:.0f}s")


if __name__ == "__main__":
    main()
