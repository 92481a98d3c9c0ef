#!/usr/bin/env python
"""Benchmark of the hot path: ADMM iterations/s and clique projections/s at
1e-4 relative accuracy, batched vs plain, on one MI355X.

Workload: random block-arrow SDP with l = 200 blocks of size d = 20 and an
arrow head of h = 10 (n = 4010), 200 cliques of size 30, m = 2000 dense
symmetrised N(0,1) constraints (seeded synthetic data standing in for the
paper's block-arrow benchmark), rho = 1, Algorithm 1 by default.

A step is one ADMM iteration (scatter -> affine projection -> batched PSD
projection with multiplier epilogue -> residuals), replayed from captured
HIP graphs of 50 iterations.  The timed region runs exactly --steps
iterations with the early exit disabled, on inputs already resident in HBM.
A separate cold-start solve reports the iterations needed for
max(eps_p, eps_d) <= 1e-4.

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
GRAPH_CHUNK = 50
METRIC = "ADMM iterations/sec and clique projections/sec at 1e-4 rel. accuracy, batched vs plain"


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1609_06068_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1609_06068_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def time_events(torch, fn, reps_outer=1):
    """Average milliseconds of fn() between two events on the current stream."""
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps_outer):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps_outer


def algorithmic_bytes(sol, prob):
    """Bytes each kernel must move per launch (method data only; index maps,
    padding and partial sums are implementation traffic)."""
    m, nU, ns, p = sol.m, sol.nnz, sol.nslots, sol.p
    return {
        "gemv_Au": m * nU * 4 + nU * 8 + 2 * m * 8,           # A (FP32), u, b, t
        "gemv_ATy": nU * m * 4 + m * 8 + 3 * nU * 8,          # A^T, y, u, 1/(wD), x
        "trmv": 2 * (m * (m + 1) // 2) * 8 + 4 * m * 8,      # L^-1 and L^-T triangles, vectors
        "project": nU * 8 + ns * (4 + 4 + 4) + p * 24,        # x, lam in/out, x_k out, partials
        "scatter": ns * 8 + nU * (8 * 3 + 8 * 2),             # x_k, lam; c, 1/D, w; S_prev in, u and S out
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--form", default="primal", choices=["primal", "dual"])
    ap.add_argument("--cpu-iters", type=int, default=50, help="oracle iterations timed for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB elementwise kernel (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--print-hash", action="store_true", help="print the kernel source hash and exit")
    args = ap.parse_args()
    if args.print_hash:
        print(kernel_source_hash())
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1609_06068_amd import cdcs, synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    form = args.form
    rho = 1.0
    if args.copy_probe:
        xp = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        yp = torch.empty_like(xp)
        for _ in range(3):
            torch.mul(xp, 2.0, out=yp)
        torch.cuda.synchronize()
        del xp, yp
    _log("generating workload")
    prob = synth.c2()
    t0 = time.perf_counter()
    sol = cdcs.Solver(prob)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    _log(f"setup {setup_s:.2f}s  nnz={sol.nnz} m={sol.m} p={sol.p} slots={sol.nslots}")

    # Accuracy: cold start, stop at max(eps_p, eps_d) <= 1e-4 (500-iteration cap).
    st = sol.new_state(form)
    acc = sol.solve(st, form=form, rho=rho, tol=1e-4, max_iter=500, check_every=GRAPH_CHUNK)
    torch.cuda.synchronize()
    _log(f"to 1e-4: {acc.iters} iterations, converged={acc.converged}, {acc.loop_s:.4f}s")
    converged_state = st

    # Timed region: warmup, then exactly K iterations (no early exit).
    K, W = args.steps, args.warmup
    stt = sol.new_state(form)
    if W > 0:
        sol.solve(stt, form=form, rho=rho, tol=0.0, max_iter=W, check_every=min(GRAPH_CHUNK, W))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = sol.solve(stt, form=form, rho=rho, tol=0.0, max_iter=K, check_every=GRAPH_CHUNK)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert info.iters == K, info
    sweeps_per_solve = info.jacobi_sweeps / (K * sol.p)
    ips = K / elapsed
    _log(f"timed: {K} iterations in {elapsed:.4f}s -> {ips:.1f} it/s, {sweeps_per_solve:.2f} sweeps/eigensolve")

    # Per-kernel average durations with HIP events (same arguments as in the loop).
    # (The solve's graphs replay after each warmup; profile_kernel graphs read the same state.)
    R = args.kernel_reps
    names = {cdcs.K_GEMV_AU: "gemv_Au", cdcs.K_GEMV_ATY: "gemv_ATy", cdcs.K_TRMV: "trmv",
             cdcs.K_PROJECT: "project", cdcs.K_SCATTER: "scatter"}
    kern_ms = {}
    for kid, name in names.items():
        # R launches captured in one graph (the solve's launch mode), replayed between events
        sol.profile_kernel(stt, kid, reps=2, form=form, rho=rho)  # warm
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            sol.profile_kernel(stt, kid, reps=R, form=form, rho=rho)
        g.replay()
        kern_ms[name] = time_events(torch, g.replay, reps_outer=3) / R
        del g
    abytes = algorithmic_bytes(sol, prob)
    kern = {n: {"us": kern_ms[n] * 1e3, "GB_s": abytes[n] / (kern_ms[n] * 1e-3) / 1e9} for n in names.values()}
    _log("kernels: " + ", ".join(f"{n} {v['us']:.1f}us {v['GB_s']:.0f}GB/s" for n, v in kern.items()))

    # Batched vs plain projection on the converged iterate's clique matrices W_k
    # (input preparation: W = x_k - lam_k / rho, which is the projection's argument).
    sizes_h = sol.sizes
    sizes_d = torch.as_tensor(sizes_h.astype(np.int32), device="cuda")
    off_d = torch.as_tensor(sol.offsets, device="cuda")
    Wp = (converged_state["blk"] - converged_state["lam"] / rho).contiguous()
    smax = int(sizes_h.max())
    P1 = cdcs.psd_project_batched(Wp, sizes_d, off_d, smax=smax)
    t_batched = time_events(torch, lambda: cdcs.psd_project_batched(Wp, sizes_d, off_d, smax=smax), reps_outer=10)
    P2 = cdcs.psd_project_plain(Wp, sizes_d, off_d, smax)
    t_plain = time_events(torch, lambda: cdcs.psd_project_plain(Wp, sizes_d, off_d, smax, P=P2),
                          reps_outer=3)
    assert torch.equal(P1, P2), "plain and batched projections differ"
    batched = {"batched_clique_proj_per_s": sol.p / (t_batched * 1e-3),
               "plain_clique_proj_per_s": sol.p / (t_plain * 1e-3),
               "batched_ms": t_batched, "plain_ms": t_plain, "speedup": t_plain / t_batched}
    _log(f"projection batched {t_batched:.3f}ms vs plain {t_plain:.3f}ms ({t_plain / t_batched:.1f}x)")

    dom = max(("gemv_Au", "gemv_ATy"), key=lambda n: kern_ms[n])
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic_c2.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tj = json.load(fh)
        if tj.get("source_hash") == kernel_source_hash() and dom in tj.get("kernels", {}):
            traffic = tj["kernels"][dom]["bytes_per_launch"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": kern[dom]["GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": kern[dom]["GB_s"] / HBM_PEAK_GBS, "traffic": traffic,
                "algorithmic_bytes": abytes[dom], "avg_us": kern[dom]["us"]}

    result = {
        "metric": METRIC,
        "value": ips,
        "unit": "ADMM iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 eig + f64 affine",
        "data": "synthetic",
        "config": {"workload": "block-arrow SDP l=200 d=20 h=10 (n=4010), 200 cliques of 30, m=2000, "
                               f"{'Alg. 1 (primal)' if form == 'primal' else 'Alg. 2 (dual)'}, rho=1",
                   "graph_chunk": GRAPH_CHUNK, "setup_s": setup_s},
        "clique_projections_per_s": ips * sol.p,
        "jacobi_sweeps_per_eigensolve": sweeps_per_solve,
        "accuracy": {"tol": 1e-4, "converged": acc.converged, "iters_to_tol": acc.iters,
                     "time_to_tol_s": acc.loop_s, "eps_p": acc.eps_p, "eps_d": acc.eps_d,
                     "obj_primal": acc.obj_primal, "obj_dual": acc.obj_dual},
        "batched_vs_plain": batched,
        "kernels": kern,
        "roofline": roofline,
    }

    if not args.no_cpu:
        from threadpoolctl import threadpool_limits

        from oracle import oracle as orc
        _log("oracle leg")
        o = orc.Oracle(prob)
        n_cpu = args.cpu_iters
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            ref = o.solve(form, rho=rho, max_iter=n_cpu)
            cpu_s = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": n_cpu / cpu_s, "unit": "ADMM iterations/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"first {n_cpu} iterations of the same solve (setup excluded), "
                                            f"FP64, one thread ({cpu_s:.1f}s)"}
        # parity at the same iteration count (cold start)
        sp = sol.new_state(form)
        sol.solve(sp, form=form, rho=rho, tol=0.0, max_iter=n_cpu, check_every=GRAPH_CHUNK)
        xg = sp["x"].cpu().numpy()
        lam_g = np.concatenate([B.ravel() for B in cdcs.unpack_blocks(sp["lam"].cpu().numpy().astype(np.float64),
                                                                       sol.sizes, sol.offsets)])
        lam_r = np.concatenate([B.ravel() for B in ref.lam])
        result["parity"] = {"iterations": n_cpu,
                            "x_rel": float(np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)),
                            "lam_rel": float(np.linalg.norm(lam_g - lam_r) / np.linalg.norm(lam_r)),
                            "tol": 1e-4}
        _log(f"oracle {n_cpu / cpu_s:.2f} it/s; parity {result['parity']}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
