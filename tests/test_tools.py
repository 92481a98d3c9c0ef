"""Host-side measurement tools (no GPU): the rocprofv3 counter and trace
summaries behind profiles/ and bench.py's `traffic`, and bench.py's refusal
of more than one GPU."""
import csv
import json
import os
import subprocess
import sys

from paper_1609_06068_amd import pmc_summary

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_counter_summary_scales_by_the_probe_and_takes_the_plan_kernel(tmp_path):
    probe = "void at::native::vectorized_elementwise_kernel<4, at::native::MulFunctor<float> >(int)"
    plan = "void cdcs::(anonymous namespace)::k_project_queue<96, 512>(cdcs::ProjArgs, unsigned long long*)"
    tuner = "void cdcs::(anonymous namespace)::k_project<96, 256>(cdcs::ProjArgs)"
    gemv = "void cdcs::(anonymous namespace)::k_gemv_Au<8>(float const*, long)"
    # 1 GiB read and 1 GiB written by the probe: 512 Ki units of FETCH, 1 Mi units of WRITE
    fetch = [(probe, 524288.0), (probe, 10.0)] + [(plan, v) for v in (100.0, 101.0, 0.2, 99.0, 100.0)] + \
            [(tuner, 300.0), (tuner, 310.0)] + [(gemv, 7.0)]
    write = [(probe, 1048576.0)] + [(plan, v) for v in (40.0, 40.0, 0.0, 40.0, 40.0)] + [(tuner, 90.0), (gemv, 0.0)]
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", write)
    out = pmc_summary.summarise(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "abc")
    assert out["source_hash"] == "abc"
    assert out["fetch_scale_bytes_per_unit"] == 2048.0 and out["write_scale_bytes_per_unit"] == 1024.0
    proj = out["kernels"]["project"]
    # median over the four launches of the plan's kernel that did work; the tuner's variant is not mixed in
    assert proj["launches"] == 4
    assert proj["fetch_bytes"] == 100.0 * 2048 and proj["write_bytes"] == 40.0 * 1024
    assert out["kernels"]["gemv_Au"]["fetch_bytes"] == 7.0 * 2048
    assert out["kernels"]["gemv_Au"]["write_bytes"] == 0.0


def test_trace_summary_filters_the_no_op_launches(tmp_path):
    path = tmp_path / "kt.csv"
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 0
        for dur_ns in (100000, 102000, 500, 98000):  # three launches that did work, one that returned at once
            w.writerow({"Kernel_Name": "void cdcs::(anonymous namespace)::k_gemv_ATy(float const*)",
                        "Start_Timestamp": t, "End_Timestamp": t + dur_ns})
            t += dur_ns + 1000
    text = pmc_summary.trace_summary(str(path), 5.0)
    row = [ln for ln in text.splitlines() if ln.startswith("k_gemv_ATy")][0].split()
    assert row[1:] == ["4", "3", "100.0", "100.0", "0.30"]


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
