#!/usr/bin/env python
"""Benchmark of the hot path: ADMM iterations/s and clique projections/s at
1e-4 relative accuracy, batched vs plain, on one MI355X.

Default workload (--workload c2): random block-arrow SDP with l = 200 blocks
of size d = 20 and an arrow head of h = 10 (n = 4010), 200 cliques of size
30, m = 2000 dense symmetrised N(0,1) constraints (seeded synthetic data
standing in for the paper's block-arrow benchmark), rho = 1, Algorithm 1.

A step is one ADMM iteration (scatter -> affine projection -> batched PSD
projection with multiplier epilogue -> residuals), replayed from captured
HIP graphs of 50 iterations.  The timed region runs exactly --steps
iterations with the early exit disabled, on inputs already resident in HBM.
A separate cold-start solve reports the iterations needed for
max(eps_p, eps_d) <= 1e-4.  Per-kernel durations (and the roofline figure)
are averages over the timed iterations themselves: they are run again from a
copy of their starting state with eager launches and HIP events around every
kernel; the JSON line reports whether the replay ended on the timed run's iterate
bit for bit (kernels_replay_bitwise).

Other workloads (each prints its own JSON line; not part of the default run):
  c3  uneven cliques: clique tree of 3000 cliques of 4..96 vertices with
      separators of 1..8, m = 8000 sparse constraints (20 coefficients each);
  c4  512 independent block-arrow SDPs in one handle, per-instance stopping,
      p50/p99 of the per-instance time to tolerance;
  c5  gradient of <C, X_K> through K = 100 unrolled iterations (l = 100,
      d = 16, h = 8, m = 800) with per-iteration checkpointing.

--gpus N with N > 1 exits: this build runs on one GPU.
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
FP32_VALU_PEAK_TFLOPS = 157.3
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
    padding and partial sums are implementation traffic).  For a sparse A the
    coefficient arrays count (4 B index + 8 B value) and each gathered vector
    element 8 B."""
    import numpy as np
    m, nU, ns, p = sol.m, sol.nnz, sol.nslots, sol.p
    out = {
        # L^-1 and L^-T (dense triangles, or CSR: 4 B column + 8 B value + 8 B gathered element), vectors
        "trmv": (2 * sol.nnz_factor * (4 + 8 + 8) if sol.sparse_factor else 2 * (m * (m + 1) // 2) * 8) + 4 * m * 8,
        "project": nU * 8 + ns * (4 + 4 + 4) + p * 24,        # x, lam in/out, x_k out, partials
        "scatter": ns * 8 + nU * (8 * 3 + 8 * 2),             # x_k, lam; c, 1/D, w; S_prev in, u and S out
    }
    if sol.sparse_a:
        nnz = sol.nnz_a
        ntc = int(np.unique(prob.A_idx).shape[0])
        out["gemv_Au"] = nnz * (4 + 8 + 8) + 2 * m * 8         # coefficients, u gathers, b, t
        # coefficients, y gathers; x = u on every entry, then u, s2 in and x out on the touched ones
        out["gemv_ATy"] = nnz * (4 + 8 + 8) + nU * 16 + ntc * (4 + 8 * 3)
    else:
        out["gemv_Au"] = m * nU * 4 + nU * 8 + 2 * m * 8        # A (FP32), u, b, t
        out["gemv_ATy"] = nU * m * 4 + m * 8 + 3 * nU * 8       # A^T, y, u, 1/(wD), x
    return out


def projection_model_flops(sizes):
    """Symmetric eigendecomposition with vectors (9 k^3) plus the rebuild
    V max(L, 0) V^T (k^3) per clique."""
    import numpy as np
    k = np.asarray(sizes, dtype=np.float64)
    return float(np.sum(10.0 * k ** 3))


def snapshot(state):
    return {k: (v.clone() if v is not None else None) for k, v in state.items()}


def replay_kernel_ms(torch, sol, start, final, form, rho, K):
    """Average duration (ms) of each kernel over the timed iterations.  A solve
    is a function of (problem, state, options), so the K timed iterations are
    run again from a copy of their starting state with eager launches and HIP
    events around every kernel (cdcs_admm_solve_timed).  Returns the averages
    and whether the replay ended on the timed run's iterate bit for bit (it
    should; a mismatch is reported in the JSON line, not fatal, so the line
    keeps its other figures)."""
    st = snapshot(start)
    info, times = sol.solve_timed(st, form=form, rho=rho, tol=0.0, max_iter=K)
    same = info.iters == K and all(torch.equal(st[k], final[k]) for k in ("x", "y", "blk", "lam"))
    if not same:
        _log("warning: the replay did not reproduce the timed iterations bit for bit")
    return {n: ms / cnt for n, (ms, cnt) in times.items() if cnt > 0}, same


def batched_vs_plain(torch, sol, state, rho):
    """The batched projection (one launch per size bucket) against the
    clique-per-launch form on the same clique matrices W_k = x_k - lam_k / rho."""
    import numpy as np
    from paper_1609_06068_amd import cdcs
    sizes_h = sol.sizes
    sizes_d = torch.as_tensor(sizes_h.astype(np.int32), device="cuda")
    off_d = torch.as_tensor(sol.offsets, device="cuda")
    Wp = (state["blk"] - state["lam"] / rho).contiguous()
    smax = int(sizes_h.max())
    P1 = cdcs.psd_project_batched(Wp, sizes_d, off_d, smax=smax)
    t_batched = time_events(torch, lambda: cdcs.psd_project_batched(Wp, sizes_d, off_d, smax=smax), reps_outer=10)
    P2 = cdcs.psd_project_plain(Wp, sizes_d, off_d, smax)
    t_plain = time_events(torch, lambda: cdcs.psd_project_plain(Wp, sizes_d, off_d, smax, P=P2), reps_outer=3)
    assert torch.equal(P1, P2), "plain and batched projections differ"
    _log(f"projection batched {t_batched:.3f}ms vs plain {t_plain:.3f}ms ({t_plain / t_batched:.1f}x)")
    return {"batched_clique_proj_per_s": sol.p / (t_batched * 1e-3),
            "plain_clique_proj_per_s": sol.p / (t_plain * 1e-3),
            "batched_ms": t_batched, "plain_ms": t_plain, "speedup": t_plain / t_batched}


def roofline_for(kern_ms, abytes, sizes, traffic_file):
    """Roofline of the kernel that takes the most time per iteration; `traffic`
    is its counter-measured HBM bytes per launch while the counters were taken
    on the current kernel sources."""
    dom = max(kern_ms, key=lambda n: kern_ms[n])
    traffic = None
    if traffic_file and os.path.exists(traffic_file):
        with open(traffic_file) as fh:
            tj = json.load(fh)
        if tj.get("source_hash") == kernel_source_hash() and dom in tj.get("kernels", {}):
            traffic = tj["kernels"][dom]["bytes_per_launch"]
    if dom == "project":
        fl = projection_model_flops(sizes)
        ach = fl / (kern_ms[dom] * 1e-3) / 1e12
        return {"bound": "alu", "kernel": dom, "achieved": ach, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP32_VALU_PEAK_TFLOPS, "traffic": traffic, "algorithmic_flops": fl,
                "avg_us": kern_ms[dom] * 1e3}
    gbs = abytes[dom] / (kern_ms[dom] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes": abytes[dom],
            "avg_us": kern_ms[dom] * 1e3}


def base_result(value, unit, K, W, ms_per_step, workload, extra_config=None):
    cfg = {"workload": workload}
    cfg.update(extra_config or {})
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": K, "warmup": W,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 eig + f64 affine", "data": "synthetic", "config": cfg}


# --------------------------------------------------------------------------
# One SDP: the block-arrow headline workload (c2) and the uneven one (c3)
# --------------------------------------------------------------------------

SINGLE = {
    "c2": dict(desc="block-arrow SDP l=200 d=20 h=10 (n=4010), 200 cliques of 30, m=2000 dense A",
               acc_cap=500, cpu_iters=100, traffic="traffic_c2.json"),
    "c3": dict(desc="clique-tree SDP, 3000 cliques of 4..96 (separators 1..8), m=8000 sparse A "
                    "(20 coefficients per constraint)",
               acc_cap=6000, cpu_iters=2, traffic="traffic_c3.json"),
}


def run_single(args, torch, workload):
    import numpy as np
    from paper_1609_06068_amd import cdcs, synth
    spec = SINGLE[workload]
    form, rho = args.form, 1.0
    _log(f"generating workload {workload}")
    prob = synth.c2() if workload == "c2" else synth.c3()
    t0 = time.perf_counter()
    sol = cdcs.Solver(prob)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    _log(f"setup {setup_s:.2f}s  n={sol.n} nnz={sol.nnz} m={sol.m} p={sol.p} slots={sol.nslots} "
         f"sparse_a={sol.sparse_a}")

    # Accuracy: cold start, stop at max(eps_p, eps_d) <= 1e-4.
    st = sol.new_state(form)
    acc = sol.solve(st, form=form, rho=rho, tol=1e-4, max_iter=1 if args.profile else spec["acc_cap"],
                    check_every=GRAPH_CHUNK)
    torch.cuda.synchronize()
    _log(f"to 1e-4: {acc.iters} iterations, converged={acc.converged}, {acc.loop_s:.4f}s")
    tuning = sol.tuning()
    _log(f"projection plan: {tuning}")

    # Timed region: warmup, then exactly K iterations (no early exit).
    K, W = args.steps, args.warmup
    stt = sol.new_state(form)
    if W > 0:
        sol.solve(stt, form=form, rho=rho, tol=0.0, max_iter=W, check_every=min(GRAPH_CHUNK, W))
    start = snapshot(stt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = sol.solve(stt, form=form, rho=rho, tol=0.0, max_iter=K, check_every=GRAPH_CHUNK)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert info.iters == K, info
    sweeps_per_solve = info.jacobi_sweeps / (K * sol.p)
    ips = K / elapsed
    _log(f"timed: {K} iterations in {elapsed:.4f}s -> {ips:.1f} it/s, {sweeps_per_solve:.2f} sweeps/eigensolve")

    kern_ms, replay_same = replay_kernel_ms(torch, sol, start, stt, form, rho, K)
    abytes = algorithmic_bytes(sol, prob)
    kern = {n: {"us": kern_ms[n] * 1e3, "GB_s": abytes[n] / (kern_ms[n] * 1e-3) / 1e9} for n in kern_ms}
    _log("kernels: " + ", ".join(f"{n} {v['us']:.1f}us {v['GB_s']:.0f}GB/s" for n, v in kern.items()))
    batched = None if args.profile else batched_vs_plain(torch, sol, st, rho)
    tfile = os.path.join(ROOT, "profiles", spec["traffic"])
    roofline = roofline_for(kern_ms, abytes, sol.sizes, tfile)
    result = base_result(ips, "ADMM iterations/s", K, W, 1e3 * elapsed / K,
                         spec["desc"] + (", Alg. 1 (primal)" if form == "primal" else ", Alg. 2 (dual)") + ", rho=1",
                         {"graph_chunk": GRAPH_CHUNK, "setup_s": setup_s, "n": sol.n, "nnz": sol.nnz,
                          "p": sol.p, "m": sol.m})
    result.update({
        "clique_projections_per_s": ips * sol.p,
        "jacobi_sweeps_per_eigensolve": sweeps_per_solve,
        "accuracy": {"tol": 1e-4, "cap": spec["acc_cap"], "converged": acc.converged, "iters_to_tol": acc.iters,
                     "time_to_tol_s": acc.loop_s, "eps_p": acc.eps_p, "eps_d": acc.eps_d,
                     "obj_primal": acc.obj_primal, "obj_dual": acc.obj_dual},
        "batched_vs_plain": batched,
        "projection_plan": tuning,
        "kernels": kern,
        "kernels_replay_bitwise": replay_same,
        "roofline": roofline,
    })
    if workload == "c3":
        result["projection_model_tflops"] = projection_model_flops(sol.sizes) / (kern_ms["project"] * 1e-3) / 1e12

    if not (args.no_cpu or args.profile):
        from threadpoolctl import threadpool_limits

        from oracle import oracle as orc
        n_cpu = args.cpu_iters if args.cpu_iters is not None else spec["cpu_iters"]
        _log(f"oracle leg ({n_cpu} iterations)")
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            o = orc.Oracle(prob)
            cpu_setup = time.perf_counter() - t0
            t0 = time.perf_counter()
            ref = o.solve(form, rho=rho, max_iter=n_cpu)
            cpu_s = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": n_cpu / cpu_s, "unit": "ADMM iterations/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"first {n_cpu} iterations of the same solve, FP64, one thread "
                                            f"({cpu_s:.1f}s; oracle setup {cpu_setup:.1f}s excluded)"}
        # parity at the same iteration count (cold start)
        sp = sol.new_state(form)
        sol.solve(sp, form=form, rho=rho, tol=0.0, max_iter=n_cpu, check_every=min(GRAPH_CHUNK, n_cpu))
        xg = sp["x"].cpu().numpy()
        lam_g = np.concatenate([B.ravel() for B in cdcs.unpack_blocks(sp["lam"].cpu().numpy().astype(np.float64),
                                                                       sol.sizes, sol.offsets)])
        lam_r = np.concatenate([B.ravel() for B in ref.lam])
        result["parity"] = {"iterations": n_cpu,
                            "x_rel": float(np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)),
                            "lam_rel": float(np.linalg.norm(lam_g - lam_r) / np.linalg.norm(lam_r)),
                            "tol": 1e-4}
        _log(f"oracle {n_cpu / cpu_s:.3f} it/s; parity {result['parity']}")
    sol.close()
    return result


# --------------------------------------------------------------------------
# Many SDPs in one handle (c4)
# --------------------------------------------------------------------------

def run_many(args, torch):
    import numpy as np
    from paper_1609_06068_amd import cdcs, synth
    rho = 1.0
    _log("generating 512 block-arrow instances")
    probs = synth.c4()
    t0 = time.perf_counter()
    sol = cdcs.BatchSolver(probs)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    _log(f"setup {setup_s:.2f}s  nnz={sol.nnz} m={sol.m} p={sol.p}")
    # cold solves to 1e-4, every instance stopping on its own
    cap = 1 if args.profile else 3000
    st = sol.new_state("primal")
    sol.solve(st, form="primal", rho=rho, tol=1e-4, max_iter=cap, check_every=GRAPH_CHUNK)  # warm graphs
    st = sol.new_state("primal")
    acc = sol.solve(st, form="primal", rho=rho, tol=1e-4, max_iter=cap, check_every=GRAPH_CHUNK)
    torch.cuda.synchronize()
    inst = sol.instance_info()
    t2t = np.array([i.time_to_tol_s for i in inst])
    its = np.array([i.iters for i in inst])
    conv = np.array([i.status == cdcs.OK for i in inst])
    _log(f"batch solve: {acc.iters} iterations, {conv.sum()}/{len(inst)} converged, {acc.loop_s:.3f}s")
    if conv.any():
        _log(f"time to tol p50 {np.percentile(t2t[conv], 50) * 1e3:.2f}ms p99 {np.percentile(t2t[conv], 99) * 1e3:.2f}ms")
    tuning = sol.tuning()
    _log(f"projection plan: {tuning}")
    # Timed region: exactly K whole-batch iterations (no early exit).
    K, W = args.steps, args.warmup
    stt = sol.new_state("primal")
    if W > 0:
        sol.solve(stt, form="primal", rho=rho, tol=0.0, max_iter=W, check_every=min(GRAPH_CHUNK, W))
    start = snapshot(stt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = sol.solve(stt, form="primal", rho=rho, tol=0.0, max_iter=K, check_every=GRAPH_CHUNK)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert info.iters == K
    ips = K / elapsed
    _log(f"timed: {K} batch iterations in {elapsed:.4f}s -> {ips:.1f} it/s")
    result = base_result(ips, "ADMM iterations/s (all 512 instances)", K, W, 1e3 * elapsed / K,
                         "512 independent block-arrow SDPs, l in 5..40, d in 8..32, h in 2..12, m = 5 l, "
                         "one handle, Alg. 1, rho=1",
                         {"graph_chunk": GRAPH_CHUNK, "setup_s": setup_s, "p": sol.p, "m": sol.m, "nnz": sol.nnz})
    result.update({
        "clique_projections_per_s": ips * sol.p,
        "instance_iterations_per_s": ips * len(probs),
        "accuracy": {"tol": 1e-4, "converged": int(conv.sum()), "instances": len(inst),
                     "iters_p50": float(np.percentile(its, 50)), "iters_max": int(its.max()),
                     "time_to_tol_p50_ms": float(np.percentile(t2t[conv], 50) * 1e3) if conv.any() else None,
                     "time_to_tol_p99_ms": float(np.percentile(t2t[conv], 99) * 1e3) if conv.any() else None,
                     "batch_solve_s": acc.loop_s},
        "batched_vs_plain": None if args.profile else batched_vs_plain(torch, sol, st, rho),
        "projection_plan": tuning,
    })
    # per-kernel averages over the timed iterations: projection, scatter, whole
    # affine step (the gemv_Au kind of a batch handle)
    kms, replay_same = replay_kernel_ms(torch, sol, start, stt, "primal", rho, K)
    kern = {"project": {"us": kms["project"] * 1e3}, "scatter": {"us": kms["scatter"] * 1e3},
            "affine": {"us": kms["gemv_Au"] * 1e3}}
    # algorithmic bytes of the affine step: A_q read twice (FP32, rows of ld_q),
    # the triangular factors (FP64 triangles) and the vectors u, x, t, y
    a_bytes = 0
    f_bytes = 0
    for pr in probs:
        ld = (pr.nU + 3) // 4 * 4
        a_bytes += 2 * pr.m * ld * 4
        f_bytes += 2 * (pr.m * (pr.m + 1) // 2) * 8
    aff_bytes = a_bytes + f_bytes + sol.nnz * 8 * 4 + sol.m * 8 * 4
    kern["affine"]["GB_s"] = aff_bytes / (kern["affine"]["us"] * 1e-6) / 1e9
    result["kernels"] = kern
    result["kernels_replay_bitwise"] = replay_same
    _log("kernels: " + ", ".join(f"{n} {v['us']:.1f}us" for n, v in kern.items()))
    if kern["affine"]["us"] >= kern["project"]["us"]:
        gbs = kern["affine"]["GB_s"]
        result["roofline"] = {"bound": "hbm", "kernel": "affine (4 kernels)", "achieved": gbs, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                              "algorithmic_bytes": aff_bytes, "avg_us": kern["affine"]["us"]}
    else:
        fl = projection_model_flops(sol.sizes)
        ach = fl / (kern["project"]["us"] * 1e-6) / 1e12
        result["roofline"] = {"bound": "alu", "kernel": "project", "achieved": ach, "peak": FP32_VALU_PEAK_TFLOPS,
                              "unit": "TFLOP/s", "frac": ach / FP32_VALU_PEAK_TFLOPS, "traffic": None,
                              "algorithmic_flops": fl, "avg_us": kern["project"]["us"]}
    if not (args.no_cpu or args.profile):
        from threadpoolctl import threadpool_limits

        from oracle import oracle as orc
        sample = list(range(0, len(probs), len(probs) // 40))[:40]  # about 10 s of oracle work
        n_cpu = 50
        _log(f"oracle leg ({len(sample)} instances x {n_cpu} iterations)")
        cpu_s = 0.0
        with threadpool_limits(limits=1):
            for q in sample:
                o = orc.Oracle(probs[q])
                t0 = time.perf_counter()
                o.solve("primal", rho=rho, max_iter=n_cpu)
                cpu_s += time.perf_counter() - t0
        per_batch_iter = cpu_s / n_cpu * len(probs) / len(sample)
        result["cpu_baseline"] = {"value": 1.0 / per_batch_iter, "unit": "ADMM iterations/s (all 512 instances)",
                                  "cores": 1, "kind": "oracle",
                                  "sample": f"{n_cpu} iterations of instances {sample} ({cpu_s:.1f}s), scaled to "
                                            f"all 512 instances, FP64, one thread"}
    sol.close()
    return result


# --------------------------------------------------------------------------
# Differentiation through unrolled iterations (c5)
# --------------------------------------------------------------------------

def run_grad(args, torch):
    from paper_1609_06068_amd import autograd as ag
    from paper_1609_06068_amd import cdcs, synth
    prob = synth.c5()
    sol = cdcs.Solver(prob)
    Kun = 100
    w = ag.entry_weights(prob)

    def fwd_bwd():
        c = torch.as_tensor(prob.c, device="cuda").requires_grad_(True)
        b = torch.as_tensor(prob.b, device="cuda").requires_grad_(True)
        x = ag.unrolled_x(sol, prob, c, b, K=Kun, rho=1.0, use_checkpoint=True)
        L = (w * c * x).sum()
        L.backward()
        return c.grad, b.grad

    for _ in range(max(args.warmup // 50, 1)):
        fwd_bwd()
    torch.cuda.synchronize()
    reps = max(args.steps // 100, 1)
    t0 = time.perf_counter()
    for _ in range(reps):
        fwd_bwd()
    torch.cuda.synchronize()
    elapsed = (time.perf_counter() - t0) / reps
    _log(f"forward+backward through {Kun} iterations: {elapsed * 1e3:.1f} ms")
    result = base_result(Kun / elapsed, "unrolled ADMM iterations/s (forward + backward)", reps, 1,
                         1e3 * elapsed / Kun,
                         "gradient of <C, X_K> w.r.t. C and b, block-arrow l=100 d=16 h=8 m=800, K=100 unrolled "
                         "Alg. 1 iterations with per-iteration checkpointing",
                         {"K": Kun, "p": sol.p, "m": sol.m})
    result["gradient_s"] = elapsed
    if not args.no_cpu:
        from threadpoolctl import threadpool_limits

        from oracle import oracle as orc
        n_pass = 2  # about 10 s of oracle work
        with threadpool_limits(limits=1):
            o = orc.Oracle(prob)
            t0 = time.perf_counter()
            for _ in range(n_pass):
                U = orc.Unrolled(o, K=Kun)
                x = U.forward(prob.c, prob.b)
                _, g = orc.loss_linear(prob, o.dec, x)
                U.backward(g)
            cpu_s = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": n_pass * Kun / cpu_s,
                                  "unit": "unrolled ADMM iterations/s (forward + backward)", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"{n_pass} forward + reverse passes over K={Kun}, FP64, one thread "
                                            f"({cpu_s:.1f}s)"}
    sol.close()
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--form", default="primal", choices=["primal", "dual"])
    ap.add_argument("--cpu-iters", type=int, default=None, help="oracle iterations timed for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB elementwise kernel (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--print-hash", action="store_true", help="print the kernel source hash and exit")
    ap.add_argument("--profile", action="store_true",
                    help="profiler runs: skip the accuracy solve, the plain-form comparison and the oracle")
    args = ap.parse_args()
    if args.print_hash:
        print(kernel_source_hash())
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        xp = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        yp = torch.empty_like(xp)
        for _ in range(3):
            torch.mul(xp, 2.0, out=yp)
        torch.cuda.synchronize()
        del xp, yp
    if args.workload in SINGLE:
        result = run_single(args, torch, args.workload)
    elif args.workload == "c4":
        result = run_many(args, torch)
    else:
        result = run_grad(args, torch)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
