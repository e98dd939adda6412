"""Host-side pieces of bench.py: the counter summary that turns rocprofv3 readings into per-launch
HBM bytes (scaled by a plain copy of known size) and VALU issue time, the source stamps that tie
counters to the sources they were taken from, and the one-GPU rule."""
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


def fake_runs(d, stamp):
    """Counter files of every run bench.py summarizes, two dispatches per kernel, each run stamped
    with the given source hashes."""
    bp = "void recon::(anonymous namespace)::bp_update_kernel<5>(recon::Geo, ...)"
    fp = "void recon::(anonymous namespace)::fp_kernel<16, true>(recon::(anonymous namespace)::FpArgs)"
    other = "void recon::(anonymous namespace)::bp_update_kernel<1>(recon::Geo, ...)"
    for run, names in bench.COUNTER_RUNS.items():
        rows = []
        for c in names:
            base = 1000.0 + len(c)
            rows += [(bp, c, base), (bp, c, base + 200.0), (fp, c, 50.0), (fp, c, 50.0), (other, c, 9e9)]
        write_counters(d, run, rows)
    # a 256 MiB copy reads as 131072 KiB fetched (factor 2) and 262144 KiB written (factor 1)
    write_counters(d, "cal_fetch", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 131072.0)])
    write_counters(d, "cal_write", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 262144.0)])
    for run in list(bench.COUNTER_RUNS) + list(bench.CAL_RUNS):
        with open(os.path.join(d, run, "source_stamp.json"), "w") as f:
            json.dump({"sources": stamp}, f)


def test_counter_summary(tmp_path):
    """Per-dispatch means per kernel and counter (the kernel picked by its exact template), HBM bytes
    scaled by the plain copy, VALU issue time at one wave64 instruction per SIMD every 2 cycles, and
    the hash of the sources recorded at collection time."""
    d = str(tmp_path)
    fake_runs(d, bench.source_hashes())
    out = os.path.join(d, "counters.json")
    rec = bench.summarize_counters(d, out_path=out)
    assert json.load(open(out)) == rec
    k = rec["kernels"]["bp_update_kernel"]
    assert k["dispatches"] == 2
    assert k["counters"]["FETCH_SIZE"] == 1000.0 + len("FETCH_SIZE") + 100.0
    assert k["fetch_bytes"] == k["counters"]["FETCH_SIZE"] * 1024 * 2.0
    assert k["write_bytes"] == k["counters"]["WRITE_SIZE"] * 1024 * 1.0
    valu = k["counters"]["SQ_INSTS_VALU"]
    assert abs(k["valu_issue_s"] - valu * 2 / (1024 * 2.4e9)) <= 1e-18
    assert rec["kernels"]["fp_kernel<OS>"]["counters"]["SQ_WAVES"] == 50.0
    assert len(k["source_sha"]) == 16
    assert rec["calibration"]["fetch_factor"] == 2.0 and rec["calibration"]["write_factor"] == 1.0


def test_counter_summary_refuses_other_sources(tmp_path):
    """Counters stamped with sources other than the current ones (a kernel changed after the runs),
    or runs stamped differently from each other, are refused."""
    import pytest

    d = str(tmp_path / "a")
    stamp = dict(bench.source_hashes())
    stamp["paper_1903_10088_amd/csrc/bp.hip"] = "0" * 16
    fake_runs(d, stamp)
    with pytest.raises(SystemExit):
        bench.summarize_counters(d, out_path=os.path.join(d, "x.json"))
    d2 = str(tmp_path / "b")
    fake_runs(d2, bench.source_hashes())
    with open(os.path.join(d2, "sq_wait", "source_stamp.json"), "w") as f:
        json.dump({"sources": stamp}, f)
    with pytest.raises(SystemExit):
        bench.summarize_counters(d2, out_path=os.path.join(d2, "x.json"))


def test_stamp_records_the_library_sources(tmp_path):
    bench.write_stamp(str(tmp_path))
    rec = json.load(open(os.path.join(str(tmp_path), "source_stamp.json")))
    assert "paper_1903_10088_amd/csrc/bp.hip" in rec["sources"] and "include/recon.h" in rec["sources"]
    assert rec["sources"] == bench.source_hashes()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_batch_counter_summary(tmp_path):
    """The batched kernels' VALU record: SQ_INSTS_VALU per dispatch averaged over each kernel's last 20
    dispatches (the last run of one epoch), other counters and non-batched kernels ignored; a run
    stamped with other sources of the batched kernels is refused."""
    import pytest

    d = str(tmp_path / "a")
    os.makedirs(d)
    bp = "void recon::(anonymous namespace)::bp_update_batch_kernel<5>(recon::SliceDesc const*, ...)"
    fp = "void recon::(anonymous namespace)::fp_batch_kernel<4>(recon::SliceDesc const*, ...)"
    single = "void recon::(anonymous namespace)::bp_update_kernel<5>(recon::Geo, ...)"
    rows, disp = [], 0
    for k in range(30):  # ten tuner dispatches (9e9), then the last run's 20 (k = 10..29)
        disp += 1
        rows.append((disp, bp, "SQ_INSTS_VALU", 9e9 if k < 10 else 1000.0 + k))
        rows.append((disp, bp, "SQ_WAVES", 5.0))
        disp += 1
        rows.append((disp, fp, "SQ_INSTS_VALU", 40.0))
        disp += 1
        rows.append((disp, single, "SQ_INSTS_VALU", 7.0))
    with open(os.path.join(d, "pmc_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], r)))
    bench.write_stamp(d)
    out = os.path.join(d, "rec.json")
    rec = bench.summarize_batch_counters(d, out_path=out)
    assert json.load(open(out)) == rec
    k = rec["kernels"]
    assert set(k) == {"bp_update_batch_kernel<5>", "fp_batch_kernel<4>"}
    assert k["bp_update_batch_kernel<5>"]["valu_instructions"] == sum(1000.0 + i for i in range(10, 30)) / 20
    assert k["fp_batch_kernel<4>"]["valu_instructions"] == 40.0
    st = json.load(open(os.path.join(d, "source_stamp.json")))
    st["sources"]["paper_1903_10088_amd/csrc/batch.hip"] = "0" * 16
    with open(os.path.join(d, "source_stamp.json"), "w") as f:
        json.dump(st, f)
    with pytest.raises(SystemExit):
        bench.summarize_batch_counters(d, out_path=out)
