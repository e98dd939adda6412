"""Host-side pieces of bench.py: the counter summary that turns rocprofv3 FETCH_SIZE / WRITE_SIZE
readings into HBM bytes per launch (scaled by a plain copy of known size), and the one-GPU rule."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FIELDS = ["Kernel_Name", "Counter_Name", "Counter_Value"]


def write_counters(d, sub, rows):
    os.makedirs(os.path.join(d, sub))
    with open(os.path.join(d, sub, "pmc_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_counter_summary_scales_by_the_copy(tmp_path):
    d = str(tmp_path)
    bp = "void recon::(anonymous namespace)::bp_update_kernel<1>(recon::Geo, ...)"
    fp = "void recon::(anonymous namespace)::fp_kernel<16, true>(recon::(anonymous namespace)::FpArgs)"
    # two dispatches each; the summary takes the mean per dispatch
    write_counters(d, "pmc_FETCH_SIZE", [(bp, "FETCH_SIZE", 100.0), (bp, "FETCH_SIZE", 300.0),
                                         (fp, "FETCH_SIZE", 50.0), (fp, "FETCH_SIZE", 50.0)])
    write_counters(d, "pmc_WRITE_SIZE", [(bp, "WRITE_SIZE", 10.0), (bp, "WRITE_SIZE", 30.0),
                                         (fp, "WRITE_SIZE", 1.0), (fp, "WRITE_SIZE", 3.0)])
    # a 4 MiB copy reads as 2048 KiB fetched (factor 2) and 4096 KiB written (factor 1)
    write_counters(d, "cal_FETCH_SIZE", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 2048.0)])
    write_counters(d, "cal_WRITE_SIZE", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 4096.0)])
    out = os.path.join(d, "traffic.json")
    rec = bench.summarize_counters(d, copy_mib=4, out_path=out)
    assert json.load(open(out)) == rec
    k = rec["kernels"]["bp_update_kernel"]
    assert k["fetch_kib"] == 200.0 and k["write_kib"] == 20.0
    assert k["fetch_bytes"] == 200.0 * 1024 * 2.0 and k["write_bytes"] == 20.0 * 1024
    assert rec["kernels"]["fp_kernel<OS>"]["fetch_bytes"] == 50.0 * 1024 * 2.0
    assert rec["calibration"]["fetch_factor"] == 2.0 and rec["calibration"]["write_factor"] == 1.0
    # the recorded hash is the one bench.py checks before reporting the traffic
    assert len(k["source_sha"]) == 16


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
