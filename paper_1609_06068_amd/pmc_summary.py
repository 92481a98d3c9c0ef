"""Summarise rocprofv3 counter CSVs into HBM bytes per kernel launch.

Input: the counter_collection CSVs of two `rocprofv3 --pmc FETCH_SIZE` and
`rocprofv3 --pmc WRITE_SIZE` runs of `bench.py --copy-probe` (each counter in
KiB per dispatch).  The copy probe is an elementwise multiply over a 1 GiB
FP32 tensor (1 GiB read, 1 GiB written); its counter readings give the scale
factor from counter units to bytes.  Output: JSON with, per kernel, the mean
scaled FETCH and WRITE bytes per launch and the source hash of the kernels
(bench.py reports `traffic` only while the hash matches).

usage: python -m paper_1609_06068_amd.pmc_summary FETCH_CSV WRITE_CSV HASH OUT_JSON
"""
from __future__ import annotations

import csv
import json
import re
import sys
from collections import defaultdict

PROBE_BYTES = 1 << 30
PROBE_PATTERN = re.compile(r"MulFunctor")
KERNELS = {"gemv_Au": r"k_gemv_Au<", "gemv_ATy": r"k_gemv_ATy", "project": r"k_project<",
           "scatter": r"k_scatter_primal", "trmv": r"k_trmv", "reduce_t": r"k_reduce_t"}


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
        vals = [v for v in vals if v > 0.5 * PROBE_BYTES / 1024]  # the 1 GiB launches only
        return sum(vals) / len(vals)

    sf = PROBE_BYTES / probe(f)
    sw = PROBE_BYTES / probe(w)
    out = {"source_hash": source_hash, "probe_bytes": PROBE_BYTES,
           "fetch_scale_bytes_per_unit": sf, "write_scale_bytes_per_unit": sw, "kernels": {}}
    for key, pat in KERNELS.items():
        fv = [v for n, vs in f.items() if re.search(pat, n) for v in vs]
        wv = [v for n, vs in w.items() if re.search(pat, n) for v in vs]
        if not fv or not wv:
            continue
        # median over launches (early-exit launches of captured graphs read ~0)
        fv.sort()
        wv.sort()
        fb = fv[len(fv) // 2] * sf
        wb = wv[len(wv) // 2] * sw
        out["kernels"][key] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                               "launches": len(fv)}
    return out


if __name__ == "__main__":
    fetch_csv, write_csv, h, out_json = sys.argv[1:5]
    res = summarise(fetch_csv, write_csv, h)
    with open(out_json, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))
