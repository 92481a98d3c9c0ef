#!/usr/bin/env python
"""Benchmark of the hot path: ADMM iterations/s and clique projections/s at
1e-4 relative accuracy, batched vs plain, on one MI355X.

Default workload (--workload c2): random block-arrow SDP with l = 200 blocks
of size d = 20 and an arrow head of h = 10 (n = 4010), 200 cliques of size
30, m = 2000 dense symmetrised N(0,1) constraints (seeded synthetic data
standing in for the paper's block-arrow benchmark), rho = 1, Algorithm 1.

A step is one ADMM iteration (scatter -> affine projection -> batched PSD
projection with multiplier epilogue -> residuals), replayed from captured
HIP graphs of 50 iterations (the last graph holds the remaining steps mod 50).
The --warmup iterations run first through graphs of the same size on the same
state; the graphs of the timed solve are captured before the timer starts
(cdcs_admm_prepare), so the timed region holds exactly --steps launched
iterations, with the early exit disabled, on inputs already resident in HBM.
A separate cold-start solve reports the iterations needed for
max(eps_p, eps_d) <= 1e-4.  Per-kernel durations (and the roofline figure)
are averages over the timed iterations themselves: they are run again from a
copy of their starting state with eager launches and HIP events around every
kernel; the JSON line reports whether the replay ended on the timed run's iterate
bit for bit (kernels_replay_bitwise).

cpu_baseline is the oracle (FP64, test infrastructure) on the host cores:
one thread and all threads of the process's CPU share (OpenMP over cliques,
threaded BLAS), with the CPU model and os.cpu_count() recorded; its parity
record compares the GPU iterates with the oracle's after 50 and after the
sampled number of iterations.

The default line (C2 headline) also carries two sub-objects measured in the
same run, with the same --steps/--warmup:
  c3  uneven cliques: clique tree of 3000 cliques of 4..96 vertices with
      separators of 1..8, m = 8000 sparse constraints (20 coefficients each):
      iterations/s, scatter GB/s against the method's bytes, batched vs plain
      projection, and 50-iteration parity against the oracle-written golden
      (tests/golden/c3_iter50.json);
  c4  512 independent block-arrow SDPs in one handle: iterations/s,
      per-instance p50/p99 time to tolerance, batched vs plain, and
      50-iteration parity against the oracle on sampled instances.
--only-headline skips them.  --workload c3|c4|c5 prints a full line for one
workload (c5: gradient of <C, X_K> through K = 100 unrolled iterations,
l = 100, d = 16, h = 8, m = 800, with per-iteration checkpointing).

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
        # sparse: L^-1 and L^-T as CSR (4 B column + 8 B value + 8 B gathered element) and four vectors;
        # dense: M^-1 as stored and read (m x m; its symmetry is not exploited), t in, y out
        "trmv": (2 * sol.nnz_factor * (4 + 8 + 8) + 4 * m * 8 if sol.sparse_factor else m * m * 8 + 2 * m * 8),
        # x, lam in/out, x_k in/out, the per-slot x_k difference out, partials
        "project": nU * 8 + ns * (4 + 4 + 4 + 4 + 4) + p * 24,
        # per slot: its index, x_k, lam and x_k difference; per entry: the inverse-map
        # pointer, c, u out and a bit of w
        "scatter": ns * (4 + 4 + 4 + 4) + nU * (4 + 8 + 8) + nU // 8,
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
    """Clique projections/s of the batched form against the clique-per-launch
    form, both on the same clique matrices W_k = x_k - lam_k / rho and both
    from a cold start (Jacobi from the identity).  Batched: the handle's tuned
    plan (one persistent work-queue launch, or one launch per size bucket),
    cdcs_psd_project_cliques.  Plain: the same projection kernel launched
    once per clique with a one-workgroup grid of that clique's own size
    bucket, no graph."""
    import numpy as np
    from paper_1609_06068_amd import cdcs
    sizes_h = np.asarray(sol.sizes, dtype=np.int64)
    sizes_d = torch.as_tensor(sizes_h.astype(np.int32), device="cuda")
    off_d = torch.as_tensor(sol.offsets, device="cuda")
    Wp = (state["blk"] - state["lam"] / rho).contiguous()
    P1 = sol.project_cliques(Wp)
    t_batched = time_events(torch, lambda: sol.project_cliques(Wp, P=P1), reps_outer=10)
    P2 = cdcs.psd_project_plain(Wp, sizes_d, off_d, sizes_h)
    t_plain = time_events(torch, lambda: cdcs.psd_project_plain(Wp, sizes_d, off_d, sizes_h, P=P2), reps_outer=3)
    diff = float(torch.linalg.norm((P1 - P2).double()) / torch.linalg.norm(Wp.double()))
    _log(f"projection batched {t_batched:.3f}ms vs plain {t_plain:.3f}ms ({t_plain / t_batched:.1f}x), "
         f"|P_batched - P_plain| / |W| = {diff:.2e}")
    return {"batched_clique_proj_per_s": sol.p / (t_batched * 1e-3),
            "plain_clique_proj_per_s": sol.p / (t_plain * 1e-3),
            "batched_ms": t_batched, "plain_ms": t_plain, "speedup": t_plain / t_batched,
            "batched_form": "tuned plan (cdcs_psd_project_cliques), cold start",
            "plain_form": "one launch per clique at its own size bucket, cold start",
            "rel_diff_batched_plain": diff}


def roofline_for(kern_ms, abytes, sizes, traffic_file):
    """Roofline of the kernel that takes the most time per iteration; `traffic`
    is its counter-measured HBM bytes per launch while the counters were taken
    on the current kernel sources.  Without cliques the projection is the
    vector cones' elementwise pass, bound by HBM."""
    dom = max(kern_ms, key=lambda n: kern_ms[n])
    traffic = counter_bytes(traffic_file, dom)
    if dom == "project" and len(sizes) > 0:
        fl = projection_model_flops(sizes)
        ach = fl / (kern_ms[dom] * 1e-3) / 1e12
        return {"bound": "alu", "kernel": dom, "achieved": ach, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP32_VALU_PEAK_TFLOPS, "traffic": traffic, "algorithmic_flops": fl,
                "avg_us": kern_ms[dom] * 1e3}
    gbs = abytes[dom] / (kern_ms[dom] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes": abytes[dom],
            "avg_us": kern_ms[dom] * 1e3}


def counter_bytes(traffic_file, kernel):
    """HBM bytes per launch of `kernel` from the counter summary, or None when
    the summary was taken on other kernel sources."""
    if not traffic_file or not os.path.exists(traffic_file):
        return None
    with open(traffic_file) as fh:
        tj = json.load(fh)
    if tj.get("source_hash") == kernel_source_hash() and kernel in tj.get("kernels", {}):
        return tj["kernels"][kernel]["bytes_per_launch"]
    return None


def base_result(value, unit, K, W, ms_per_step, workload, extra_config=None):
    cfg = {"workload": workload}
    cfg.update(extra_config or {})
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": K, "warmup": W,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 eig + f64 affine", "data": "synthetic", "config": cfg}


# --------------------------------------------------------------------------
# The oracle on the host cores (cpu_baseline)
# --------------------------------------------------------------------------

def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def all_threads():
    """Threads of this process's CPU share: OMP_NUM_THREADS when it is set
    (the GPU hosts set it to their share), else os.cpu_count()."""
    n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return n


def oracle_timed(fn, threads):
    """Run fn() with `threads` BLAS and OpenMP threads; return (result, seconds)."""
    from threadpoolctl import threadpool_limits

    from oracle import oracle as orc
    orc.lib()  # loaded first, so that its OpenMP runtime is under the limit
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        out = fn()
        return out, time.perf_counter() - t0


def cpu_legs(fn, units, unit, sample, fn_all=None, how="OpenMP over cliques, threaded BLAS"):
    """cpu_baseline from one run of fn() on one thread and one on all threads
    of the share (fn_all(threads) when given, else fn under a thread limit);
    the all-threads run's result is returned for parity checks."""
    _, s1 = oracle_timed(fn, 1)
    nall = all_threads()
    if fn_all is None:
        res, sn = oracle_timed(fn, nall)
    else:
        t0 = time.perf_counter()
        res = fn_all(nall)
        sn = time.perf_counter() - t0
    _log(f"oracle: {units / s1:.3f} {unit} on 1 thread, {units / sn:.3f} on {nall} threads")
    rec = {"value": units / sn, "unit": unit, "cores": nall, "kind": "oracle",
           "sample": f"{sample}, FP64, {nall} threads ({how}; {sn:.1f}s; one thread: {s1:.1f}s)",
           "single_thread": {"value": units / s1, "cores": 1, "seconds": s1},
           "cpu_model": host_cpu(), "os_cpu_count": os.cpu_count()}
    return rec, res


_POOL = {}


def _pool_solve(i):
    """Worker of the many-SDP oracle leg: one instance on one thread."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        _POOL["oracles"][i].solve(_POOL["form"], rho=_POOL["rho"], max_iter=_POOL["iters"])
    return i


def oracle_pool_child(spec):
    """The all-threads leg of the many-SDP oracle baseline, in a child process
    that never touches the GPU (started by bench.py itself): the sampled
    instances on `workers` forked processes, one thread each, the oracles
    built before the fork so that the timed region holds the solves only.
    Prints {"seconds": ...}."""
    from multiprocessing import get_context

    from oracle import oracle as orc
    from paper_1609_06068_amd import synth
    qs = [int(v) for v in spec["instances"].split(",")]
    _POOL["oracles"] = [orc.Oracle(synth.c4(count=1, first=q)[0]) for q in qs]
    _POOL["rho"], _POOL["iters"], _POOL["form"] = spec["rho"], spec["iters"], spec.get("form", "primal")
    orc.lib()
    with get_context("fork").Pool(spec["workers"]) as pool:
        t0 = time.perf_counter()
        pool.map(_pool_solve, range(len(qs)), chunksize=1)
        sec = time.perf_counter() - t0
    print(json.dumps({"seconds": sec, "workers": spec["workers"]}), flush=True)


def pool_leg(sample, rho, n_it, workers, form="primal"):
    """Seconds of the all-threads many-SDP oracle leg (a child process)."""
    import subprocess
    spec = json.dumps({"instances": ",".join(str(q) for q in sample), "rho": rho, "iters": n_it,
                       "workers": workers, "form": form})
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--oracle-pool", spec],
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError(f"oracle pool leg failed: {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])["seconds"]


def rel(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# --------------------------------------------------------------------------
# One SDP: the block-arrow headline workload (c2) and the uneven one (c3)
# --------------------------------------------------------------------------

SINGLE = {
    "c2": dict(desc="block-arrow SDP l=200 d=20 h=10 (n=4010), 200 cliques of 30, m=2000 dense A",
               acc_cap=500, cpu_iters=100, traffic="traffic_c2.json"),
    "c3": dict(desc="clique-tree SDP, 3000 cliques of 4..96 (separators 1..8), m=8000 sparse A "
                    "(20 coefficients per constraint)",
               acc_cap=6000, cpu_iters=2, traffic="traffic_c3.json"),
    "lp": dict(desc="conic program with vector cones only: 4,000,000 orthant variables, a second-order cone of "
                    "100,000, 10,000 free variables, m=8,000 sparse constraints (20 coefficients each)",
               acc_cap=20000, cpu_iters=0, traffic=None),
    "big": dict(desc="clique-tree SDP, 40 cliques of 127..330 (separators 1..8), m=2000 sparse A "
                     "(20 coefficients per constraint), cliques projected by the matrix sign function",
                acc_cap=3000, cpu_iters=1, traffic=None),
}


def make_single(workload):
    from paper_1609_06068_amd import synth
    return {"c2": synth.c2, "c3": synth.c3, "big": synth.c3_big, "lp": synth.lp_big}[workload]()


def sign_function_flops(sizes, steps_per_clique):
    """FP32 flops of the large-clique projection: per Newton-Schulz step two
    products of symmetric k x k matrices, each needing only its lower triangle
    (k^2 (k + 1) flops), and the final product W (I + S); the steps are the
    measured average per clique (the iteration stops per clique)."""
    import numpy as np
    k = np.asarray(sizes, dtype=np.float64)
    return float(np.sum((2.0 * steps_per_clique + 1.0) * k * k * (k + 1.0)))


def timed_solve(torch, sol, form, rho, K, W):
    """W warm-up iterations, then exactly K timed iterations (graphs of
    GRAPH_CHUNK iterations plus one of K mod GRAPH_CHUNK, captured before the
    timer starts).  Returns (info, seconds, start state, end state)."""
    stt = sol.new_state(form)
    if W > 0:
        sol.solve(stt, form=form, rho=rho, tol=0.0, max_iter=W, check_every=GRAPH_CHUNK)
    sol.prepare(stt, form=form, rho=rho, tol=0.0, max_iter=K, check_every=GRAPH_CHUNK)
    start = snapshot(stt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = sol.solve(stt, form=form, rho=rho, tol=0.0, max_iter=K, check_every=GRAPH_CHUNK)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert info.iters == K, info
    return info, elapsed, start, stt


STEADY_K, STEADY_W = 300, 100


def steady_state(torch, sol, form, rho, K, W):
    """The same timed solve over a fixed window past the first iterations
    (W = 100 untimed, K = 300 timed), reported beside the requested window
    when that one differs: short windows right after a cold start time
    eigensolves that still need several sweeps.  None when the windows agree."""
    if (K, W) == (STEADY_K, STEADY_W):
        return None
    info, elapsed, _, _ = timed_solve(torch, sol, form, rho, STEADY_K, STEADY_W)
    out = {"steps": STEADY_K, "warmup": STEADY_W, "value": STEADY_K / elapsed,
           "ms_per_step": 1e3 * elapsed / STEADY_K}
    if sol.p > 0:
        out["jacobi_sweeps_per_eigensolve"] = info.jacobi_sweeps / (STEADY_K * sol.p)
    _log(f"steady state: {STEADY_K} iterations after {STEADY_W}: {out['value']:.1f} it/s")
    return out


def packed_at(sol, packed, ks, a, b):
    """Values of packed clique blocks at (clique, row a >= column b)."""
    import numpy as np
    ks, a, b = (np.asarray(v, dtype=np.int64) for v in (ks, a, b))
    return packed[sol.offsets[ks] + a * (a + 1) // 2 + b]


def golden_parity(torch, sol, rho):
    """50 iterations of Algorithms 1 and 2 from a cold state against the
    oracle-written golden (sampled x entries and clique-block slots),
    element by element: |gpu - oracle| <= 1e-4 RMS(oracle vector)."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "c3_iter50.json")
    with open(path) as fh:
        g = json.load(fh)
    out = {"iterations": g["iterations"], "tol": 1e-4, "samples": len(g["entries"])}
    ok = True
    for form in ("primal", "dual"):
        st = sol.new_state(form)
        sol.solve(st, form=form, rho=rho, tol=0.0, max_iter=g["iterations"], check_every=GRAPH_CHUNK)
        ref = g[form]
        got = {"x": st["x"].cpu().numpy()[np.asarray(g["entries"])]}
        for name in ("blk", "lam") + (("v",) if form == "dual" else ()):
            got[name] = packed_at(sol, st[name].cpu().numpy().astype(np.float64), g["slots"]["clique"],
                                  g["slots"]["a"], g["slots"]["b"])
        rec = {}
        for name, val in got.items():
            r = np.asarray(ref[name])
            worst = float(np.max(np.abs(val - r)) / (1e-4 * ref[name + "_rms"]))
            rec[name] = {"max_err_over_tol": worst, "sampled_rel": rel(val, r)}
            ok = ok and worst <= 1.0
        out[form] = rec
    out["pass"] = ok
    _log(f"c3 golden parity at 50 iterations: {out}")
    return out


def run_single(args, torch, workload, nested=False):
    import numpy as np
    from paper_1609_06068_amd import cdcs, synth
    spec = SINGLE[workload]
    form, rho = args.form, 1.0
    _log(f"generating workload {workload}")
    prob = make_single(workload)
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
    info, elapsed, start, stt = timed_solve(torch, sol, form, rho, K, W)
    # 0 when every clique takes the sign function or there are no cliques
    sweeps_per_solve = info.jacobi_sweeps / (K * sol.p) if sol.p > 0 else 0.0
    ips = K / elapsed
    _log(f"timed: {K} iterations in {elapsed:.4f}s -> {ips:.1f} it/s, {sweeps_per_solve:.2f} sweeps/eigensolve")

    kern_ms, replay_same = replay_kernel_ms(torch, sol, start, stt, form, rho, K)
    abytes = algorithmic_bytes(sol, prob)
    kern = {n: {"us": kern_ms[n] * 1e3, "GB_s": abytes[n] / (kern_ms[n] * 1e-3) / 1e9} for n in kern_ms}
    _log("kernels: " + ", ".join(f"{n} {v['us']:.1f}us {v['GB_s']:.0f}GB/s" for n, v in kern.items()))
    # (the clique-per-launch form exists for cliques of the LDS path only)
    batched = None if (args.profile or workload in ("big", "lp")) else batched_vs_plain(torch, sol, st, rho)
    tfile = os.path.join(ROOT, "profiles", spec["traffic"]) if spec["traffic"] else None
    roofline = roofline_for(kern_ms, abytes, sol.sizes, tfile)
    if workload == "big":
        # every clique above the LDS limit: the projection is FP32 products on the matrix cores
        fl = sign_function_flops(sol.sizes, sweeps_per_solve)
        ach = fl / (kern_ms["project"] * 1e-3) / 1e12
        roofline = {"bound": "mfma", "kernel": "project (sign function)", "achieved": ach,
                    "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP32_VALU_PEAK_TFLOPS,
                    "traffic": None, "algorithmic_flops": fl, "avg_us": kern_ms["project"] * 1e3,
                    "newton_schulz_steps_per_clique": sweeps_per_solve}
    result = base_result(ips, "ADMM iterations/s", K, W, 1e3 * elapsed / K,
                         spec["desc"] + (", Alg. 1 (primal)" if form == "primal" else ", Alg. 2 (dual)") + ", rho=1",
                         {"graph_chunk": GRAPH_CHUNK, "setup_s": setup_s, "n": sol.n, "nnz": sol.nnz,
                          "p": sol.p, "m": sol.m})
    ss = None if args.profile else steady_state(torch, sol, form, rho, K, W)
    if ss is not None:
        result["steady_state"] = ss
    # gather/scatter against the method's bytes: the scatter reads one 4-byte
    # contribution per clique slot and writes one 8-byte right-hand side entry
    # per pattern entry; the gather is fused into the projection kernel
    if "scatter" in kern_ms:
        sb = 4 * sol.nslots + 8 * sol.nnz
        sgbs = sb / (kern_ms["scatter"] * 1e-3) / 1e9
        gs = {"scatter_us": kern_ms["scatter"] * 1e3, "scatter_method_bytes": sb, "scatter_GB_s": sgbs,
              "scatter_frac": sgbs / HBM_PEAK_GBS, "scatter_impl_bytes": abytes["scatter"],
              "scatter_counter_bytes": counter_bytes(tfile, "scatter"),
              "gather": "fused into the projection kernel (not timed apart)"}
    else:
        gs = None
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
        "gather_scatter": gs,
        "roofline": roofline,
    })
    if workload == "c3":
        result["projection_model_tflops"] = projection_model_flops(sol.sizes) / (kern_ms["project"] * 1e-3) / 1e12
        if not args.profile:
            result["parity"] = golden_parity(torch, sol, rho)
            # the decomposition from the pattern alone (host): chordality test,
            # maximal cliques; the generator's cliques are the exact answer
            t0 = time.perf_counter()
            fi, _, cptr, cvert = cdcs.chordal_extension(prob.n, prob.ei, prob.ej)
            ext_s = time.perf_counter() - t0
            same = (sorted(tuple(cvert[cptr[k]:cptr[k + 1]]) for k in range(len(cptr) - 1)) ==
                    sorted(tuple(prob.clique(k)) for k in range(prob.p)))
            result["chordal_extension"] = {"seconds": ext_s, "calls": 2, "fill": int(fi.shape[0]),
                                           "cliques": int(len(cptr) - 1), "same_cliques_as_generator": bool(same)}
            _log(f"chordal extension of the pattern: {result['chordal_extension']}")

    if workload in ("c2", "big") and not (args.no_cpu or args.profile):
        from oracle import oracle as orc
        n_cpu = args.cpu_iters if args.cpu_iters is not None else spec["cpu_iters"]
        o = orc.Oracle(prob)
        snap = {}

        def keep50(it, x, y, blocks, lam):
            if it == 50:
                snap.update(x=x.copy(), blocks=[B.copy() for B in blocks], lam=[B.copy() for B in lam])

        _log(f"oracle legs ({n_cpu} iterations)")
        cpu, ref = cpu_legs(lambda: o.solve(form, rho=rho, max_iter=n_cpu, callback=keep50), n_cpu,
                            "ADMM iterations/s", f"first {n_cpu} iterations of the same solve (setup excluded)")
        result["cpu_baseline"] = cpu
        # parity: a cold solve of 50 iterations, continued to n_cpu (the state
        # carries the eigenvector warm start, so this equals one solve)
        par = {"tol": 1e-4}
        sp = sol.new_state(form)
        done = 0
        for n_it, r in ((50, snap), (n_cpu, {"x": ref.x, "blocks": ref.blocks, "lam": ref.lam})):
            if not r or n_it <= done:
                continue
            sol.solve(sp, form=form, rho=rho, tol=0.0, max_iter=n_it - done, check_every=GRAPH_CHUNK)
            done = n_it
            xg = sp["x"].cpu().numpy()
            blk = sp["blk"].cpu().numpy().astype(np.float64)
            lam = sp["lam"].cpu().numpy().astype(np.float64)
            par[f"iter{n_it}"] = {"x_rel": rel(xg, r["x"]), "blk_rel": rel(blk, cdcs.pack_blocks(r["blocks"])),
                                  "lam_rel": rel(lam, cdcs.pack_blocks(r["lam"]))}
        result["parity"] = par
        _log(f"parity {par}")
    sol.close()
    if nested:
        keep = ("value", "unit", "ms_per_step", "clique_projections_per_s", "jacobi_sweeps_per_eigensolve",
                "accuracy", "batched_vs_plain", "projection_plan", "kernels", "kernels_replay_bitwise",
                "gather_scatter", "roofline", "projection_model_tflops", "parity", "chordal_extension",
                "steady_state")
        out = {k: result[k] for k in keep if k in result}
        out["config"] = result["config"]
        return out
    return result


def run_hsde(args, torch, workload):
    """The homogeneous self-dual embedding solver on a single-SDP workload:
    HSDE iterations/s over exactly K timed iterations (graphs captured before
    the timer), a cold solve to 1e-4 (outcome, iterations, objectives beside
    Algorithm 1's), per-kernel averages from an instrumented replay of the
    timed iterations, the oracle's HSDE on the host and parity after 50
    iterations."""
    import numpy as np
    from paper_1609_06068_amd import cdcs, synth
    spec = SINGLE[workload]
    _log(f"generating workload {workload}")
    prob = make_single(workload)
    t0 = time.perf_counter()
    sol = cdcs.Solver(prob)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    cap = 1 if args.profile else 4 * spec["acc_cap"]
    st = sol.new_hsde_state()
    acc = sol.hsde_solve(st, tol=1e-4, max_iter=cap, check_every=GRAPH_CHUNK)
    torch.cuda.synchronize()
    _log(f"HSDE to 1e-4: status {acc.status}, {acc.iters} iterations, {acc.loop_s:.4f}s, "
         f"objectives {acc.obj_primal:.6f} / {acc.obj_dual:.6f}")
    ref1 = None
    if not args.profile:
        s1 = sol.new_state("primal")
        ref1 = sol.solve(s1, form="primal", tol=1e-4, max_iter=spec["acc_cap"], check_every=GRAPH_CHUNK)
    # timed region: W warm-up iterations, graphs for K captured on the state
    # (then the state is restored), exactly K iterations timed
    K, W = args.steps, args.warmup
    stt = sol.new_hsde_state()
    if W > 0:
        sol.hsde_solve(stt, tol=0.0, max_iter=W, check_every=GRAPH_CHUNK)
    start = snapshot(stt)
    sol.hsde_solve(stt, tol=0.0, max_iter=K, check_every=GRAPH_CHUNK)
    for k in stt:
        stt[k].copy_(start[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = sol.hsde_solve(stt, tol=0.0, max_iter=K, check_every=GRAPH_CHUNK)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    assert info.iters == K, info
    ips = K / elapsed
    _log(f"timed: {K} HSDE iterations in {elapsed:.4f}s -> {ips:.1f} it/s")
    rep = snapshot(start)
    _, times = sol.hsde_solve_timed(rep, tol=0.0, max_iter=K)
    same = all(torch.equal(rep[k], stt[k]) for k in ("x", "y", "s", "z", "tk"))
    kern_ms = {n: ms / cnt for n, (ms, cnt) in times.items() if cnt > 0}
    abytes = algorithmic_bytes(sol, prob)
    kern = {n: {"us": kern_ms[n] * 1e3, "GB_s": abytes[n] / (kern_ms[n] * 1e-3) / 1e9} for n in kern_ms}
    _log("kernels: " + ", ".join(f"{n} {v['us']:.1f}us {v['GB_s']:.0f}GB/s" for n, v in kern.items()))
    roofline = roofline_for(kern_ms, abytes, sol.sizes, None)
    result = base_result(ips, "HSDE iterations/s", K, W, 1e3 * elapsed / K,
                         spec["desc"] + ", homogeneous self-dual embedding (no over-relaxation)",
                         {"graph_chunk": GRAPH_CHUNK, "setup_s": setup_s, "n": sol.n, "nnz": sol.nnz,
                          "p": sol.p, "m": sol.m})
    result.update({
        "accuracy": {"tol": 1e-4, "cap": cap, "status": cdcs.STATUS_NAMES.get(acc.status, acc.status),
                     "iters_to_tol": acc.iters, "time_to_tol_s": acc.loop_s, "res_pri": acc.res_pri,
                     "res_dual": acc.res_dual, "gap": acc.gap, "obj_primal": acc.obj_primal,
                     "obj_dual": acc.obj_dual,
                     "algorithm_1": None if ref1 is None else {"iters_to_tol": ref1.iters,
                                                               "obj_primal": ref1.obj_primal,
                                                               "obj_dual": ref1.obj_dual}},
        "kernels": kern,
        "kernels_replay_bitwise": same,
        "roofline": roofline,
    })
    n_cpu = args.cpu_iters if args.cpu_iters is not None else spec["cpu_iters"]
    if not (args.no_cpu or args.profile) and n_cpu > 0:
        from oracle import oracle as orc
        h = orc.Hsde(prob)
        keep = {}

        def at50(it, x, y, z, s_, tau, kappa):
            if it == 50:
                keep.update(x=x.copy(), y=y.copy(), z=[B.copy() for B in z], s=[B.copy() for B in s_], tau=tau,
                            kappa=kappa)

        _log(f"oracle HSDE ({n_cpu} iterations)")
        cpu, _ = cpu_legs(lambda: h.solve(max_iter=n_cpu, tol=0.0, callback=at50), n_cpu, "HSDE iterations/s",
                          f"first {n_cpu} HSDE iterations of the same solve (setup excluded)")
        result["cpu_baseline"] = cpu
        if keep:
            sp = sol.new_hsde_state()
            sol.hsde_solve(sp, tol=0.0, max_iter=50, check_every=GRAPH_CHUNK)

            def packed(blocks):
                return np.concatenate([B[np.tril_indices(B.shape[0])] if B.ndim == 2 else B for B in blocks])

            sw = np.sqrt(h.dec.w)
            par = {"iterations": 50, "tol": 1e-4,
                   "x_rel": rel(sp["x"].cpu().numpy() * sw, keep["x"] * sw),
                   "y_rel": rel(sp["y"].cpu().numpy(), keep["y"]),
                   "s_rel": rel(sp["s"].cpu().numpy(), packed(keep["s"])),
                   "z_rel": rel(sp["z"].cpu().numpy(), packed(keep["z"])),
                   "tau_rel": rel([sp["tk"][0].item()], [keep["tau"]])}
            par["pass"] = max(v for k, v in par.items() if k.endswith("_rel")) <= 1e-4
            result["parity"] = par
            _log(f"HSDE parity at 50 iterations: {par}")
    sol.close()
    return result


# --------------------------------------------------------------------------
# Many SDPs in one handle (c4)
# --------------------------------------------------------------------------

def run_many(args, torch, nested=False):
    import numpy as np
    from paper_1609_06068_amd import cdcs, synth
    rho = 1.0
    form = args.form
    alg = "Alg. 1" if form == "primal" else "Alg. 2"
    _log("generating 512 block-arrow instances")
    probs = synth.c4()
    t0 = time.perf_counter()
    sol = cdcs.BatchSolver(probs)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    _log(f"setup {setup_s:.2f}s  nnz={sol.nnz} m={sol.m} p={sol.p}")
    # cold solves to 1e-4, every instance stopping on its own
    cap = 1 if args.profile else 3000
    st = sol.new_state(form)
    sol.prepare(st, form=form, rho=rho, tol=1e-4, max_iter=cap, check_every=GRAPH_CHUNK)
    acc = sol.solve(st, form=form, rho=rho, tol=1e-4, max_iter=cap, check_every=GRAPH_CHUNK)
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
    info, elapsed, start, stt = timed_solve(torch, sol, form, rho, K, W)
    ips = K / elapsed
    _log(f"timed: {K} batch iterations in {elapsed:.4f}s -> {ips:.1f} it/s")
    result = base_result(ips, "ADMM iterations/s (all 512 instances)", K, W, 1e3 * elapsed / K,
                         "512 independent block-arrow SDPs, l in 5..40, d in 8..32, h in 2..12, m = 5 l, "
                         f"one handle, {alg}, rho=1",
                         {"graph_chunk": GRAPH_CHUNK, "setup_s": setup_s, "p": sol.p, "m": sol.m, "nnz": sol.nnz})
    ss = None if args.profile else steady_state(torch, sol, form, rho, K, W)
    if ss is not None:
        result["steady_state"] = ss
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
    kms, replay_same = replay_kernel_ms(torch, sol, start, stt, form, rho, K)
    kern = {"project": {"us": kms["project"] * 1e3}, "scatter": {"us": kms["scatter"] * 1e3},
            "affine": {"us": kms["gemv_Au"] * 1e3}}
    # algorithmic bytes of the affine step: A_q read twice (FP32, rows of ld_q),
    # the triangular factors (FP64 triangles) and the vectors u, x, t, y
    a_bytes = 0
    f_bytes = 0
    for pr in probs:
        ld = (pr.nU + 31) // 32 * 32
        a_bytes += 2 * pr.m * ld * 4
        f_bytes += 2 * (pr.m * (pr.m + 1) // 2) * 8
    aff_bytes = a_bytes + f_bytes + sol.nnz * 8 * 4 + sol.m * 8 * 4
    kern["affine"]["GB_s"] = aff_bytes / (kern["affine"]["us"] * 1e-6) / 1e9
    sb = 4 * sol.nslots + 8 * sol.nnz
    kern["scatter"]["GB_s"] = sb / (kern["scatter"]["us"] * 1e-6) / 1e9
    result["kernels"] = kern
    result["kernels_replay_bitwise"] = replay_same
    result["gather_scatter"] = {"scatter_us": kern["scatter"]["us"], "scatter_method_bytes": sb,
                                "scatter_GB_s": kern["scatter"]["GB_s"],
                                "scatter_frac": kern["scatter"]["GB_s"] / HBM_PEAK_GBS,
                                "gather": "fused into the projection kernel (not timed apart)"}
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
        from oracle import oracle as orc
        sample = list(range(0, len(probs), len(probs) // 40))[:40]  # about 10 s of oracle work on one thread
        n_cpu = 50
        _log(f"oracle legs ({len(sample)} instances x {n_cpu} iterations)")
        oracles = [orc.Oracle(probs[q]) for q in sample]
        # n_cpu iterations of the sampled instances stand for n_cpu |sample| / 512
        # iterations of the whole batch
        units = n_cpu * len(sample) / len(probs)
        refs, s1 = oracle_timed(lambda: [o.solve(form, rho=rho, max_iter=n_cpu) for o in oracles], 1)
        nall = all_threads()
        try:
            sn = pool_leg(sample, rho, n_cpu, nall, form)
        except Exception as exc:  # the single-thread figure still stands
            _log(f"oracle all-threads leg failed: {exc}")
            sn = None
        smp = f"{n_cpu} iterations of instances {sample}, scaled to all 512 instances (setup excluded), FP64"
        if sn is not None:
            _log(f"oracle: {units / s1:.3f} batch it/s on 1 thread, {units / sn:.3f} on {nall} processes")
            result["cpu_baseline"] = {
                "value": units / sn, "unit": "ADMM iterations/s (all 512 instances)", "cores": nall,
                "kind": "oracle",
                "sample": f"{smp}, {nall} processes of one thread each ({sn:.1f}s; one thread: {s1:.1f}s)",
                "single_thread": {"value": units / s1, "cores": 1, "seconds": s1},
                "cpu_model": host_cpu(), "os_cpu_count": os.cpu_count()}
        else:
            result["cpu_baseline"] = {
                "value": units / s1, "unit": "ADMM iterations/s (all 512 instances)", "cores": 1,
                "kind": "oracle", "sample": f"{smp}, one thread ({s1:.1f}s)",
                "cpu_model": host_cpu(), "os_cpu_count": os.cpu_count()}
        # parity: the batch after 50 iterations from a cold state, per sampled instance
        sp = sol.new_state(form)
        sol.solve(sp, form=form, rho=rho, tol=0.0, max_iter=n_cpu, check_every=GRAPH_CHUNK)
        xg = sp["x"].cpu().numpy()
        blk = sp["blk"].cpu().numpy().astype(np.float64)
        lam = sp["lam"].cpu().numpy().astype(np.float64)
        worst = {"x_rel": 0.0, "blk_rel": 0.0, "lam_rel": 0.0}
        for q, r in zip(sample, refs):
            e0, e1 = sol.entry_off[q], sol.entry_off[q + 1]
            k0, k1 = sol.clique_off[q], sol.clique_off[q + 1]
            o0, o1 = sol.offsets[k0], sol.offsets[k1]
            worst["x_rel"] = max(worst["x_rel"], rel(xg[e0:e1], r.x))
            worst["blk_rel"] = max(worst["blk_rel"], rel(blk[o0:o1], cdcs.pack_blocks(r.blocks)))
            worst["lam_rel"] = max(worst["lam_rel"], rel(lam[o0:o1], cdcs.pack_blocks(r.lam)))
        result["parity"] = {"iterations": n_cpu, "instances": sample, "worst": worst, "tol": 1e-4,
                            "pass": max(worst.values()) <= 1e-4}
        _log(f"c4 parity at {n_cpu} iterations: {result['parity']['worst']}")
    sol.close()
    if nested:
        keep = ("value", "unit", "ms_per_step", "clique_projections_per_s", "instance_iterations_per_s",
                "accuracy", "batched_vs_plain", "projection_plan", "kernels", "kernels_replay_bitwise",
                "gather_scatter", "roofline", "cpu_baseline", "parity", "steady_state")
        out = {k: result[k] for k in keep if k in result}
        out["config"] = result["config"]
        return out
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
        x = ag.unrolled_x(sol, c, b, K=Kun, rho=1.0)
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
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5", "big", "lp"])
    ap.add_argument("--form", default="primal", choices=["primal", "dual", "hsde"],
                    help="Algorithm 1, Algorithm 2, or the homogeneous self-dual embedding (c2, c3)")
    ap.add_argument("--cpu-iters", type=int, default=None, help="oracle iterations timed for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB elementwise kernel (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--print-hash", action="store_true", help="print the kernel source hash and exit")
    ap.add_argument("--profile", action="store_true",
                    help="profiler runs: skip the accuracy solve, the plain-form comparison and the oracle")
    ap.add_argument("--only-headline", action="store_true",
                    help="default workload without the c3 and c4 sub-objects")
    ap.add_argument("--oracle-pool", default=None, help=argparse.SUPPRESS)  # internal: the c4 oracle child
    args = ap.parse_args()
    if args.oracle_pool is not None:
        oracle_pool_child(json.loads(args.oracle_pool))
        return
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
    if args.form == "hsde":
        if args.workload not in SINGLE:
            print(json.dumps({"error": "--form hsde runs on the single-SDP workloads c2 and c3"}), flush=True)
            sys.exit(2)
        result = run_hsde(args, torch, args.workload)
    elif args.workload in SINGLE:
        result = run_single(args, torch, args.workload)
        if args.workload == "c2" and not (args.only_headline or args.profile):
            result["c3"] = run_single(args, torch, "c3", nested=True)
            result["c4"] = run_many(args, torch, nested=True)
    elif args.workload == "c4":
        result = run_many(args, torch)
    else:
        result = run_grad(args, torch)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
