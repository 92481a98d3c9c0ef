"""Summarise rocprofv3 counter CSVs into HBM bytes per kernel launch.

Input: the counter_collection CSVs of two `rocprofv3 --pmc FETCH_SIZE` and
`rocprofv3 --pmc WRITE_SIZE` runs of `bench.py --copy-probe` (each counter in
KiB per dispatch).  The copy probe is an elementwise multiply over a 1 GiB
FP32 tensor (1 GiB read, 1 GiB written); its counter readings give the scale
factor from counter units to bytes.  Output: JSON with, per kernel, the mean
scaled FETCH and WRITE bytes per launch and the source hash of the kernels
(bench.py reports `traffic` only while the hash matches).

usage: python -m paper_1609_06068_amd.pmc_summary FETCH_CSV WRITE_CSV HASH OUT_JSON
       python -m paper_1609_06068_amd.pmc_summary trace KERNEL_TRACE_CSV [MIN_US]

The `trace` form prints, per kernel of a `rocprofv3 --kernel-trace` CSV, the
launch count and the median / mean duration of the launches longer than
MIN_US (default 5 us): launches of captured graphs after the device stop flag
is set return at once and would otherwise dominate the statistics.
"""
from __future__ import annotations

import csv
import json
import re
import sys
from collections import defaultdict

PROBE_BYTES = 1 << 30
PROBE_PATTERN = re.compile(r"MulFunctor")
KERNELS = {"gemv_Au": r"k_gemv_Au<", "gemv_ATy": r"k_gemv_ATy", "project": r"k_project(<|_queue<)",
           "scatter": r"k_scatter_primal", "trmv": r"k_trmv", "reduce_t": r"k_reduce_t",
           "spmv_Au": r"k_spmv_Au", "sp_xcorr": r"k_sp_xcorr", "csr_mv": r"k_csr_mv"}


def _read(path, counter):
    per = defaultdict(list)
    with open(path) as fh:
        for row in csv.DictReader(fh):
            name = row.get("Kernel_Name") or row.get("Kernel-Name") or ""
            cname = row.get("Counter_Name") or row.get("Counter-Name") or ""
            if counter not in cname:
                continue
            per[name].append(float(row.get("Counter_Value") or row.get("Counter-Value")))
    return per


def summarise(fetch_csv, write_csv, source_hash):
    f = _read(fetch_csv, "FETCH_SIZE")
    w = _read(write_csv, "WRITE_SIZE")

    def probe(per):
        vals = [v for n, vs in per.items() if PROBE_PATTERN.search(n) for v in vs]
        # the 1 GiB launches only; FETCH_SIZE reads about half of the KiB
        # count on MI355X, so the cut sits well below that
        vals = [v for v in vals if v > 0.25 * PROBE_BYTES / 1024]
        return sum(vals) / len(vals)

    sf = PROBE_BYTES / probe(f)
    sw = PROBE_BYTES / probe(w)
    out = {"source_hash": source_hash, "probe_bytes": PROBE_BYTES,
           "fetch_scale_bytes_per_unit": sf, "write_scale_bytes_per_unit": sw, "kernels": {}}
    def busiest(per, pat):
        # the launches of the matching kernel name that did the most launches
        # with work: the plan's kernel, which runs every iteration (the setup
        # autotuner's variants run a few times each); launches of captured
        # graphs after the stop flag return at once and read ~0
        best = []
        for n, vs in per.items():
            if not re.search(pat, n) or not vs:
                continue
            work = [v for v in vs if v > 0.01 * max(vs)]
            if len(work) > len(best):
                best = work
        return sorted(best)

    for key, pat in KERNELS.items():
        fv = busiest(f, pat)
        wv = busiest(w, pat)
        if not fv:
            continue
        wv = wv or [0.0]
        fb = fv[len(fv) // 2] * sf
        wb = wv[len(wv) // 2] * sw
        out["kernels"][key] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                               "launches": len(fv)}
    return out


def trace_summary(trace_csv, min_us=5.0):
    """Per-kernel launch statistics of a kernel-trace CSV (text table)."""
    dur = defaultdict(list)
    with open(trace_csv) as fh:
        for row in csv.DictReader(fh):
            name = (row.get("Kernel_Name") or "").replace("cdcs::(anonymous namespace)::", "")
            name = name.replace("void ", "").split("(")[0]
            dur[name].append((int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3)
    rows = []
    for name, v in dur.items():
        real = sorted(x for x in v if x > min_us)
        if not real:
            continue
        rows.append((sum(real), name, len(v), len(real), real[len(real) // 2], sum(real) / len(real)))
    rows.sort(reverse=True)
    out = [f"{'kernel':44s} {'launches':>8s} {'>' + str(min_us) + 'us':>8s} {'median_us':>10s} {'mean_us':>10s} "
           f"{'total_ms':>9s}"]
    for tot, name, n, nr, med, mean in rows:
        out.append(f"{name[:44]:44s} {n:8d} {nr:8d} {med:10.1f} {mean:10.1f} {tot / 1e3:9.2f}")
    return "\n".join(out)


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        print(trace_summary(sys.argv[2], float(sys.argv[3]) if len(sys.argv) > 3 else 5.0))
        sys.exit(0)
    fetch_csv, write_csv, h, out_json = sys.argv[1:5]
    res = summarise(fetch_csv, write_csv, h)
    with open(out_json, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))
