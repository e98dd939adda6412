#!/usr/bin/env python3
"""Throughput of the ordered-subset TV reconstruction on one MI355X.

Workload: one clinical-scale slice, 512 x 512 at 0.78125 mm (400 mm FOV), fan
beam with 800 views over 360 degrees and 738 arc channels (SAD 850 mm, SDD
1450 mm), seeded low-contrast ellipse phantom, Poisson counts at I0 = 2e3,
20 equal-interval subsets, 500 sub-iterations, TV weight beta = 1e-3.  A step
is one complete reconstruction of the slice from the homogeneous start (inputs
already resident in HBM).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
PAPER_S_PER_SLICE = 3.71  # GTX 1080 Ti, thinning 1/20, 512^2, 800 views (Table I)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


SOURCES_DIRS = ["paper_1903_10088_amd/csrc", "include"]
COUNTER_RECORD = os.path.join(ROOT, "profiles", "counters_512x800.json")
# kernel record name: (name pattern in the counter files, the sources it is built from)
COUNTER_KERNELS = {
    "bp_update_kernel": ("bp_update_kernel<5>", ["paper_1903_10088_amd/csrc/bp.hip",
                                                 "paper_1903_10088_amd/csrc/gather.h",
                                                 "paper_1903_10088_amd/csrc/internal.h"]),
    "fp_kernel<OS>": ("fp_kernel<16, true>", ["paper_1903_10088_amd/csrc/kernels.hip",
                                              "paper_1903_10088_amd/csrc/gather.h",
                                              "paper_1903_10088_amd/csrc/internal.h"]),
}
# counter runs of COUNTER_ARGS (one rocprofv3 --pmc run each, within the per-block limits) and of
# the plain-copy calibration
COUNTER_RUNS = {
    "hbm_fetch": ["FETCH_SIZE"],
    "hbm_write": ["WRITE_SIZE"],
    "sq_issue": ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES",
                 "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT"],
    "sq_wait": ["SQ_WAIT_INST_ANY", "SQ_WAIT_ANY", "SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU",
                "SQ_WAIT_INST_LDS", "SQ_INST_LEVEL_LDS"],
    "l2": ["TCC_HIT_sum", "TCC_MISS_sum"],
}
CAL_RUNS = {"cal_fetch": ["FETCH_SIZE"], "cal_write": ["WRITE_SIZE"]}
COUNTER_ARGS = ("--steps 1 --warmup 0 --iters 40 --cpu-iters 0 --time-iters 0 --cnn-batch 0 --warm-slices 0 "
                "--batch-slices 0 --rebin-slices 0")
CAL_MIB = 256
# the batched leg's VALU instructions per sub-iteration: one rocprofv3 --pmc SQ_INSTS_VALU run of
# BATCH_COUNTER_ARGS (64 mixed slices, tuned, 3 runs of 20 sub-iterations), averaged over each
# kernel's last 20 dispatches (the last run: one dispatch per subset)
BATCH_COUNTER_RECORD = os.path.join(ROOT, "profiles", "counters_batched_64mixed.json")
BATCH_COUNTER_SOURCES = ["paper_1903_10088_amd/csrc/batch.hip", "paper_1903_10088_amd/csrc/bp.hip",
                         "paper_1903_10088_amd/csrc/kernels.hip", "paper_1903_10088_amd/csrc/gather.h",
                         "paper_1903_10088_amd/csrc/internal.h"]
BATCH_COUNTER_ARGS = ("--steps 1 --warmup 0 --iters 20 --cpu-iters 0 --time-iters 0 --cnn-batch 0 --warm-slices 0 "
                      "--rebin-slices 0 --batch-slices 64")
SIMDS = 1024              # 256 compute units x 4 SIMDs
CLOCK_HZ = 2.4e9          # peak engine clock
# the published FP32 vector rate, 157.3 TFLOP/s, counts an FMA as two operations: 32 lanes per SIMD per
# cycle, i.e. one wave64 VALU instruction every 2 cycles (what plain FP32 and integer adds reach;
# conversions, 32-bit integer multiplies and the bf16 dot product issue every 4, recon_valu_rate)
VALU_CYCLES = 2
VALU_PEAK_TOPS = SIMDS * 64 / VALU_CYCLES * CLOCK_HZ / 1e12


def source_hashes(paths=None) -> dict:
    """sha256 (first 16 hex digits) of the given repo files, or of every library source."""
    import hashlib

    if paths is None:
        paths = sorted(os.path.join(d, f) for d in SOURCES_DIRS for f in os.listdir(os.path.join(ROOT, d)))
    return {p: hashlib.sha256(open(os.path.join(ROOT, p), "rb").read()).hexdigest()[:16] for p in paths}


def combined_sha(hashes: dict, paths) -> str:
    import hashlib

    return hashlib.sha256("".join(hashes[p] for p in paths).encode()).hexdigest()[:16]


def write_stamp(d: str):
    """Records, at collection time, the hashes of the library sources a counter run is taken from."""
    import hashlib

    os.makedirs(d, exist_ok=True)
    so = os.path.join(ROOT, "paper_1903_10088_amd", "librecon.so")
    rec = {"sources": source_hashes(),
           "librecon_so": hashlib.sha256(open(so, "rb").read()).hexdigest()[:16] if os.path.exists(so) else None,
           "time": time.time()}
    with open(os.path.join(d, "source_stamp.json"), "w") as fh:
        json.dump(rec, fh, indent=1)


def measured_counters(kernel: str):
    """The committed counter record of one kernel (HBM bytes per launch from calibrated FETCH_SIZE +
    WRITE_SIZE, SQ instruction counts per launch), or None when the kernel's sources differ from
    those the counters were taken from."""
    try:
        rec = json.load(open(COUNTER_RECORD))["kernels"][kernel]
        if combined_sha(source_hashes(rec["sources"]), rec["sources"]) != rec["source_sha"]:
            return None
        return rec
    except (OSError, KeyError, ValueError):
        return None


def summarize_counters(d: str, out_path: str | None = None) -> dict:
    """profiles/counters_512x800.json from the rocprofv3 --pmc runs under d (d/<run>/pmc_counter_collection.csv
    for every run of COUNTER_RUNS and CAL_RUNS, each with the source_stamp.json its bench.py wrote).
    Counters are averaged per dispatch; FETCH_SIZE and WRITE_SIZE are scaled by bytes moved / counter
    reading of the plain copy.  Refuses runs whose stamps differ from each other or from the current
    sources of a recorded kernel."""
    import collections
    import csv

    def agg(run):
        a = collections.defaultdict(list)
        for r in csv.DictReader(open(os.path.join(d, run, "pmc_counter_collection.csv"))):
            a[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in a.items()}, {k: len(v) for k, v in a.items()}

    def pick(a, pat, counter):
        ks = [k for k in a if pat in k[0] and k[1] == counter]
        if len(ks) != 1:
            raise SystemExit(f"bench: {len(ks)} kernels match {pat!r} / {counter} in the counter files")
        return a[ks[0]]

    stamps = {}
    for run in list(COUNTER_RUNS) + list(CAL_RUNS):
        stamps[run] = json.load(open(os.path.join(d, run, "source_stamp.json")))["sources"]
    first = stamps["hbm_fetch"]
    now = source_hashes()
    for run, st in stamps.items():
        if st != first:
            raise SystemExit(f"bench: counter run {run} was taken from different sources than hbm_fetch")
    data = {run: agg(run) for run in COUNTER_RUNS}
    cf = pick(agg("cal_fetch")[0], "copyBuffer", "FETCH_SIZE")
    cw = pick(agg("cal_write")[0], "copyBuffer", "WRITE_SIZE")
    copy_kib = CAL_MIB * 1024
    ff, wf = copy_kib / cf, copy_kib / cw
    kernels = {}
    for name, (pat, src) in COUNTER_KERNELS.items():
        sha = combined_sha(first, src)
        if sha != combined_sha(now, src):
            raise SystemExit(f"bench: the sources of {name} changed since the counters were taken")
        counters = {}
        n_disp = None
        for run, names in COUNTER_RUNS.items():
            vals, counts = data[run]
            for c in names:
                counters[c] = pick(vals, pat, c)
                n_disp = pick(counts, pat, c)
        rec = {"pattern": pat, "dispatches": n_disp, "counters": counters,
               "fetch_bytes": counters["FETCH_SIZE"] * 1024 * ff, "write_bytes": counters["WRITE_SIZE"] * 1024 * wf,
               "valu_issue_s": counters["SQ_INSTS_VALU"] * VALU_CYCLES / (SIMDS * CLOCK_HZ),
               "l2_hit_rate": counters["TCC_HIT_sum"] / max(1.0, counters["TCC_HIT_sum"] + counters["TCC_MISS_sum"]),
               "source_sha": sha, "sources": src}
        kernels[name] = rec
    cmd = f"python3 <repo>/bench.py {COUNTER_ARGS}"
    commands = [f"cd /tmp && rocprofv3 --pmc {' '.join(c)} --output-format csv -d <dir>/{run} -o pmc -- "
                f"{cmd} --stamp <dir>/{run}" for run, c in COUNTER_RUNS.items()]
    commands += [f"cd /tmp && rocprofv3 --pmc {' '.join(c)} --output-format csv -d <dir>/{run} -o pmc -- "
                 f"python3 <repo>/bench.py --calibrate-copy {CAL_MIB} --stamp <dir>/{run}" for run, c in CAL_RUNS.items()]
    commands.append("python3 <repo>/bench.py --summarize-counters <dir>")
    out = {"workload": "512x512, 800 views x 738 channels, 20 subsets, 40 sub-iterations (two dispatches of "
                       "each subset per kernel); averages per dispatch",
           "calibration": {"copy_mib": CAL_MIB, "fetch_kib_read": cf, "write_kib_read": cw,
                           "fetch_factor": ff, "write_factor": wf},
           "clock_hz": CLOCK_HZ, "simds": SIMDS, "kernels": kernels, "commands": commands}
    with open(out_path or COUNTER_RECORD, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def summarize_batch_counters(d: str, out_path: str | None = None) -> dict:
    """profiles/counters_batched_64mixed.json from one rocprofv3 --pmc SQ_INSTS_VALU run of
    BATCH_COUNTER_ARGS under d (d/pmc_counter_collection.csv and the source_stamp.json its bench.py
    wrote): SQ_INSTS_VALU per dispatch of every batched kernel, averaged over its last 20 dispatches.
    Refuses a run taken from sources other than the current ones."""
    import collections
    import csv
    import re

    stamp = json.load(open(os.path.join(d, "source_stamp.json")))["sources"]
    now = source_hashes()
    sha = combined_sha(stamp, BATCH_COUNTER_SOURCES)
    if sha != combined_sha(now, BATCH_COUNTER_SOURCES):
        raise SystemExit("bench: the batched kernels' sources changed since the counters were taken")
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(os.path.join(d, "pmc_counter_collection.csv"))):
        if r["Counter_Name"] != "SQ_INSTS_VALU":
            continue
        m = re.search(r"([A-Za-z_0-9]+(<[^>]*>)?)\(", r["Kernel_Name"])
        name = m.group(1) if m else r["Kernel_Name"]
        if "batch_kernel" in name:
            per[name].append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    kernels = {}
    for name, v in per.items():
        last = [x for _, x in sorted(v)[-20:]]
        kernels[name] = {"valu_instructions": sum(last) / len(last), "dispatches_averaged": len(last)}
    out = {"workload": "64 mixed slices (38 at 512x512, 26 at 256x256; 600-900 views, 520-738 channels), seeds "
                       "1000+, 20 subsets; SQ_INSTS_VALU (wave64 instructions) per dispatch, mean over each "
                       "kernel's last 20 dispatches",
           "source_sha": sha, "sources": BATCH_COUNTER_SOURCES, "kernels": kernels,
           "commands": [f"cd /tmp && rocprofv3 --pmc SQ_INSTS_VALU --output-format csv -d <dir> -o pmc -- "
                        f"python3 <repo>/bench.py {BATCH_COUNTER_ARGS} --stamp <dir>",
                        "python3 <repo>/bench.py --summarize-batch-counters <dir>"]}
    with open(out_path or BATCH_COUNTER_RECORD, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def batch_counters():
    """The committed VALU record of the batched kernels, or None when missing or when their sources
    differ from those it was taken from."""
    try:
        rec = json.load(open(BATCH_COUNTER_RECORD))
        if combined_sha(source_hashes(rec["sources"]), rec["sources"]) != rec["source_sha"]:
            return None
        return rec["kernels"]
    except (OSError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=500, help="sub-iterations per reconstruction")
    ap.add_argument("--beta", type=float, default=1e-3)
    ap.add_argument("--cpu-iters", type=int, default=500,
                    help="sub-iterations of the oracle timed for the CPU baseline (0 = skip)")
    ap.add_argument("--time-iters", type=int, default=100, help="sub-iterations of the per-kernel timing pass")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the oracle baseline (0 = all; 1 = the paper's single-CPU setting)")
    ap.add_argument("--fp-segments", type=int, default=0)
    ap.add_argument("--bp-variant", type=int, default=0,
                    help="update variant as recon_set_launch numbers them (1-6; 0 = the library's default, 6)")
    ap.add_argument("--cnn-batch", type=int, default=8,
                    help="slices per timed CNN kernel launch (512 x 512; 0 = skip the CNN leg)")
    ap.add_argument("--batch-slices", type=int, default=64,
                    help="mixed 256/512 slices for the batched-plain leg (0 = skip)")
    ap.add_argument("--warm-slices", type=int, default=32,
                    help="full-study slices for the warm-start leg (0 = skip; needs trained weights)")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1903_10088_amd", "weights", "warm_cnn.bin"))
    ap.add_argument("--rebin-slices", type=int, default=16,
                    help="slices of the helical-rebinning leg (0 = skip)")
    ap.add_argument("--summarize-counters", default=None, metavar="DIR",
                    help="write profiles/counters_512x800.json from the counter runs under DIR (no GPU)")
    ap.add_argument("--summarize-batch-counters", default=None, metavar="DIR",
                    help="write profiles/counters_batched_64mixed.json from the batched counter run under DIR "
                         "(no GPU)")
    ap.add_argument("--stamp", default=None, metavar="DIR",
                    help="write DIR/source_stamp.json (hashes of the library sources) before running")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 10 plain device copies of MIB MiB (reference for HBM byte counters) and exit")
    args = ap.parse_args()

    if args.summarize_counters:
        rec = summarize_counters(args.summarize_counters)
        print(json.dumps(rec["kernels"]))
        return
    if args.summarize_batch_counters:
        rec = summarize_batch_counters(args.summarize_batch_counters)
        print(json.dumps(rec["kernels"]))
        return
    if args.stamp:
        write_stamp(args.stamp)
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (slices shard across GPUs with no "
              "exchange, so N GPUs would run N independent copies). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copied {args.calibrate_copy} MiB 10 times")
        return

    from paper_1903_10088_amd import phantom as ph
    from paper_1903_10088_amd import recon

    dev = torch.device("cuda:0")
    g = ph.config1_geometry()
    M, i0, seed = 20, 2e3, 100
    log(f"bench: generating slice (seed {seed}) ...")
    sl = ph.make_slice(g, seed, i0, low_contrast=True)
    R = recon.Recon(g, M, args.beta)
    if args.fp_segments or args.bp_variant:
        R.set_launch(fp_segments=args.fp_segments, bp_variant=args.bp_variant)
    counts = torch.from_numpy(sl.counts).to(dev)
    img = torch.empty((g.n, g.n), dtype=torch.float32, device=dev)

    def step():
        R.initial_image_(img)
        R.os_iterate(counts, i0, img, args.iters)

    log(f"bench: warmup {args.warmup} step(s)")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} step(s) of {args.iters} sub-iterations")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ev_ms_per_step = ev0.elapsed_time(ev1) / args.steps
    ms_per_step = 1e3 * elapsed / args.steps
    slices_per_s = args.steps / elapsed
    log(f"bench: {ms_per_step:.2f} ms per slice, {slices_per_s:.2f} slices/s")

    # Per-kernel durations: each kernel launched time_iters times back to back on
    # the library's stream (torch's current stream) between two HIP events.
    # Kernel durations in the timed run: a graph-replayed sub-iteration is the projector and the
    # update back to back, each meeting the cache state the other leaves, so each kernel's duration
    # in the run is its share of the sub-iteration time measured over the timed region (HIP events
    # on the library's stream), split in the ratio of the two kernels' back-to-back durations.  The
    # back-to-back means (caches warm for the same kernel) and means with an event pair around every
    # launch in sub-iteration order (which adds the events' own gaps) bracket it.
    sub_ms = ev_ms_per_step / args.iters
    if args.time_iters > 0:
        kimg = R.initial_image(dev)
        fp_b2b, _, bp_b2b, bp_pair, fp_pair = R.time_kernels(counts, i0, kimg, args.time_iters)
        torch.cuda.synchronize()
        fp_ms = sub_ms * fp_b2b / (fp_b2b + bp_b2b)
        bp_ms = sub_ms * bp_b2b / (fp_b2b + bp_b2b)
    else:
        fp_ms = bp_ms = fp_b2b = bp_b2b = fp_pair = bp_pair = float("nan")
    # Algorithmic bytes per launch (per unit: 4 B per ray-pixel interpolation
    # pair read, over every in-image pixel of the projector's matrix; projector
    # 12 B per ray for y/I0 and p read and w written; update 8 B per pixel for
    # mu read and mu' written), averaged over subsets.
    n_rays = [R.subset_size(s) * g.n_channels for s in range(M)]
    pairs = [R.count_pairs(s) for s in range(M)]
    npix = g.n * g.n
    fp_bytes = np.mean([4 * p + 12 * r for p, r in zip(pairs, n_rays)])
    bp_bytes = np.mean([4 * p + 8 * npix for p in pairs])
    fp_gbps = fp_bytes / (fp_ms * 1e-3) / 1e9
    bp_gbps = bp_bytes / (bp_ms * 1e-3) / 1e9
    slice_bytes = args.iters * (fp_bytes + bp_bytes)
    log(f"bench: graph sub-iteration {sub_ms * 1e3:.2f} us: fp {fp_ms * 1e3:.2f} us ({fp_gbps:.0f} GB/s alg), "
        f"step rule + bp + tv + update {bp_ms * 1e3:.2f} us ({bp_gbps:.0f} GB/s alg); back to back "
        f"{fp_b2b * 1e3:.1f} and {bp_b2b * 1e3:.1f} us, with event pairs {fp_pair * 1e3:.1f} and "
        f"{bp_pair * 1e3:.1f} us")
    # ceiling of the gather kernels' algorithmic rates: what 2048 blocks reading an L2-resident
    # buffer draw from the caches, measured now on this GPU
    l2_gbps = recon.read_bandwidth(2 << 20, 10) if args.time_iters > 0 else None
    if l2_gbps:
        log(f"bench: L2-resident read bandwidth {l2_gbps:.0f} GB/s")
    # the vector ALU's issue rate for a few instruction kinds, measured now (T lane-ops/s)
    valu_rates = {name: recon.valu_rate(k, 5) / 1e12 for k, name in enumerate(recon.VALU_OPS)} \
        if args.time_iters > 0 else None
    if valu_rates:
        log("bench: VALU issue (T lane-ops/s): " + ", ".join(f"{k} {v:.1f}" for k, v in valu_rates.items()))
    kern = {"bp_update_kernel": kernel_roofline("bp_update_kernel", bp_ms, bp_bytes, l2_gbps),
            "fp_kernel<OS>": kernel_roofline("fp_kernel<OS>", fp_ms, fp_bytes, l2_gbps)}
    dom = kern["bp_update_kernel"] if bp_ms >= fp_ms else kern["fp_kernel<OS>"]

    cpu = None
    parity = None
    if args.cpu_iters > 0:
        import oracle

        n_cpu = min(args.cpu_iters, args.iters)
        if args.cpu_threads > 0:
            oracle.set_threads(args.cpu_threads)
        log(f"bench: oracle on {oracle.num_threads()} host threads, {n_cpu} sub-iterations ...")
        t0 = time.perf_counter()
        ref, _ = oracle.os_iterate(g, M, args.beta, sl.counts, i0, None, n_cpu, want_trace=False)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": 1.0 / (t_cpu * args.iters / n_cpu), "unit": "slices/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{n_cpu} of {args.iters} sub-iterations of the same slice, FP64 C oracle, "
                         f"{t_cpu:.1f} s, scaled to a full reconstruction"}
        gimg, _ = R.os_iterate(counts, i0, None, n_cpu)
        disc = oracle.initial_image(g, 1.0) > 0
        rmse = float(np.sqrt(np.mean((gimg.cpu().numpy().astype(np.float64) - ref)[disc] ** 2)))
        parity = {"sub_iterations": n_cpu, "rmse_vs_oracle_per_mm": rmse,
                  "tolerance_per_mm": 1e-4 * ph.MU_WATER_PER_MM, "ok": rmse <= 1e-4 * ph.MU_WATER_PER_MM}
        log(f"bench: cpu {cpu['value']:.4f} slices/s; GPU vs oracle rmse after {n_cpu} sub-iterations {rmse:.2e}")

    fbp = fbp_leg(R, counts, sl.i0)
    rebin = rebin_leg(args.rebin_slices, dev) if args.rebin_slices > 0 else None
    batch = batch_leg(args.batch_slices, args.iters, dev, l2_gbps) if args.batch_slices > 0 else None
    cnn = cnn_leg(args.cnn_batch, dev) if args.cnn_batch > 0 else None
    warm = warm_leg(args.warm_slices, args.weights, dev) if args.warm_slices > 0 else None

    out = {
        "metric": "512² slices/s to oracle RMSE: plain OS-TV vs CNN warm start; projector GB/s",
        "value": slices_per_s,
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": slices_per_s * PAPER_S_PER_SLICE,
        "dtype": "f32",
        "data": "synthetic: seeded low-contrast ellipse phantom, analytic line integrals, Poisson counts",
        "config": {"workload": "one 512x512 slice (0.78125 mm), fan beam 800 views x 738 arc channels, "
                               "SAD 850 / SDD 1450 mm, I0 2e3, 20 subsets, 500 sub-iterations, beta 1e-3",
                   "image": g.n, "views": g.n_views, "channels": g.n_channels, "subsets": M,
                   "sub_iterations": args.iters, "beta": args.beta, "i0": i0},
        "roofline": dom["roofline"],
        "cpu_baseline": cpu,
        "projector_gbps": fp_gbps,
        "projector": kern["fp_kernel<OS>"]["roofline"],
        "l2_read_gbps": l2_gbps,
        "valu_rates_tops": valu_rates,
        "slice_alg_gbps": slice_bytes / (ms_per_step * 1e-3) / 1e9,
        "slice_alg_frac_of_l2_read": (slice_bytes / (ms_per_step * 1e-3) / 1e9 / l2_gbps) if l2_gbps else None,
        "kernel_us": {"fp": fp_ms * 1e3, "bp_update": bp_ms * 1e3, "graph_sub_iteration": sub_ms * 1e3,
                      "fp_back_to_back": fp_b2b * 1e3, "bp_update_back_to_back": bp_b2b * 1e3,
                      "fp_event_pairs": fp_pair * 1e3, "bp_update_event_pairs": bp_pair * 1e3},
        "parity": parity,
        "fbp_baseline": fbp,
        "helical_rebin": rebin,
        "batched_plain": batch,
        "cnn_kernels": cnn,
        "warm_start": warm,
        "paper_context": {"s_per_slice": PAPER_S_PER_SLICE, "hardware": "GeForce GTX 1080 Ti",
                          "thinning": "1/20", "note": "context only; channel count and precision not stated"},
    }
    print(json.dumps(out), flush=True)


def kernel_roofline(name: str, ms: float, alg_bytes: float, l2_gbps):
    """Roofline of one kernel from its live mean launch time: the fraction of each ceiling it
    reaches -- VALU issue (SQ_INSTS_VALU per launch from the committed counter record, one wave64
    instruction per SIMD every 2 cycles), HBM (calibrated FETCH_SIZE + WRITE_SIZE bytes per launch
    against 8 TB/s) and the L2-resident read bandwidth (algorithmic bytes) -- and the largest of
    them as the bound.  Without a counter record for the current sources only the L2 fraction is
    known."""
    sec = ms * 1e-3
    alg_gbps = alg_bytes / sec / 1e9
    ctr = measured_counters(name)
    fr = {}
    if l2_gbps:
        fr["l2"] = alg_gbps / l2_gbps
    traffic = None
    if ctr:
        fr["alu"] = ctr["valu_issue_s"] / sec
        traffic = ctr["fetch_bytes"] + ctr["write_bytes"]
        fr["hbm"] = traffic / sec / 1e9 / PEAK_HBM_GBPS
    roof = {"kernel": name, "avg_launch_us": ms * 1e3, "alg_bytes_per_launch": alg_bytes, "alg_gbps": alg_gbps,
            "fractions": fr, "traffic": traffic,
            "hbm_gbps_measured": traffic / sec / 1e9 if traffic else None,
            "counters": "profiles/counters_512x800.json" if ctr else None}
    if not fr:
        roof.update(bound=None, achieved=None, peak=None, unit=None, frac=None)
    else:
        bound = max(fr, key=fr.get)
        if bound == "alu":
            lane_ops = ctr["counters"]["SQ_INSTS_VALU"] * 64 / sec / 1e12
            roof.update(bound="alu", achieved=lane_ops, peak=VALU_PEAK_TOPS, unit="T VALU lane-ops/s")
        elif bound == "hbm":
            roof.update(bound="hbm", achieved=traffic / sec / 1e9, peak=PEAK_HBM_GBPS, unit="GB/s")
        else:
            roof.update(bound="l2", achieved=alg_gbps, peak=l2_gbps, unit="GB/s")
        roof["frac"] = roof["achieved"] / roof["peak"]
    return {"name": name, "ms": ms, "bytes": alg_bytes, "gbps": alg_gbps, "roofline": roof}


def fbp_leg(R, counts, i0: float, reps: int = 20):
    """The filtered-backprojection baseline (recon_fbp) on the same slice: time per slice over
    `reps` back-to-back calls (HIP events on the library's stream)."""
    import torch

    R.fbp(counts, i0)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        R.fbp(counts, i0)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    log(f"bench: fbp baseline {ms:.3f} ms per slice")
    return {"ms_per_slice": ms, "slices_per_s": 1e3 / ms}


def batch_leg(n_slices: int, iters: int, dev, l2_gbps=None):
    """Batched plain method on helical-rebinned-like slices (256^2 or 512^2 over 400 mm, 600-900
    views, 520-738 channels, I0 log-uniform 1e3..1e4; 20 subsets, beta 1e-3): launch shapes
    autotuned on the batch, then `iters` sub-iterations of every slice from the homogeneous
    start, timed over 3 runs (best).  Algorithmic bytes as for the single slice (per sub-iteration,
    averaged over the subsets: 8 B per ray-pixel pair, 12 B per ray, 8 B per pixel), the pairs
    counted from each slice's own ray tables."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    from paper_1903_10088_amd import phantom as ph
    from paper_1903_10088_amd import recon
    from paper_1903_10088_amd import warmstart as ws

    geoms, i0s, items = [], [], []
    for i in range(n_slices):
        g, i0 = ph.random_batch_geometry(1000 + i)
        geoms.append(g)
        i0s.append(i0)
        items.append((g, 1000 + i, i0))
    log(f"bench: batched leg: {n_slices} slices ...")
    counts = ws.make_counts(items, workers=8)
    B = recon.Batch(geoms, 20, 1e-3)
    cts = [torch.from_numpy(c).to(dev) for c in counts]
    seg, var = B.tune(cts, i0s, B.initial_images(dev), reps=20)
    best = None
    for _ in range(3):
        imgs = B.initial_images(dev)
        _, dt = ws.timed(lambda: B.run(cts, i0s, imgs, iters))
        best = dt if best is None else min(best, dt)
    n512 = sum(1 for g in geoms if g.n == 512)

    def sub_iteration_bytes(g):
        R = recon.Recon(g, 20, 1e-3)
        pairs = R.count_pairs(-1)
        R.close()
        return (8 * pairs + 12 * g.n_views * g.n_channels) / 20 + 8 * g.n * g.n

    with ThreadPoolExecutor(8) as ex:
        alg = iters * sum(ex.map(sub_iteration_bytes, geoms))
    gbps = alg / best / 1e9
    out = {"slices": n_slices, "slices_512": n512, "slices_256": n_slices - n512, "sub_iterations": iters,
           "tuned_fp_segments": seg, "tuned_bp_variant": var, "seconds": best, "slices_per_s": n_slices / best,
           "alg_bytes": alg, "alg_gbps": gbps, "alg_frac_of_l2_read": gbps / l2_gbps if l2_gbps else None,
           "roofline": None}
    # VALU issue of a whole batched sub-iteration (projector + step rule + update) from the committed
    # instruction counts, against the sub-iteration's time in this run (the 64-slice workload only)
    ctr = batch_counters() if n_slices == 64 else None
    names = [f"fp_batch_kernel<{seg}>", "step_batch_kernel", f"bp_update_batch_kernel<{var - 1}>"]
    if ctr and all(k in ctr for k in names):
        instr = sum(ctr[k]["valu_instructions"] for k in names)
        t_sub = best / iters
        out["roofline"] = {"bound": "alu", "scope": "whole batched sub-iteration: " + " + ".join(names),
                           "valu_instructions": instr, "sub_iteration_us": t_sub * 1e6,
                           "achieved": instr * 64 / t_sub / 1e12, "peak": VALU_PEAK_TOPS,
                           "unit": "T VALU lane-ops/s", "frac": instr * VALU_CYCLES / (SIMDS * CLOCK_HZ) / t_sub,
                           "counters": "profiles/counters_batched_64mixed.json"}
    alu = f", VALU issue {out['roofline']['frac']:.2f} of peak" if out["roofline"] else ""
    log(f"bench: batched plain {out['slices_per_s']:.1f} slices/s ({n512} of {n_slices} at 512^2; "
        f"fp_segments {seg}, bp variant {var}); {gbps:.0f} GB/s algorithmic{alu}")
    B.close()
    return out


PEAK_BF16_TFLOPS = 2500.0  # dense bf16 matrix-core peak


def rebin_leg(n_slices: int, dev):
    """Helical rebinning (recon_rebin_helical) of a 3-turn single-row scan of 800 views x 738
    channels per turn (pitch 10 mm) to n_slices slices: HBM rate of the kernel from 8 bytes read
    and 4 written per output element, mean over 20 calls (CUDA events on the library's stream)."""
    import numpy as np
    import torch

    from paper_1903_10088_amd import phantom as ph
    from paper_1903_10088_amd import recon

    g = ph.config1_geometry()
    nh, pitch, z0 = 3 * g.n_views, 10.0, -15.0
    rng = np.random.default_rng(9)
    counts = torch.from_numpy(rng.poisson(2000.0 * np.exp(-rng.uniform(0, 3, (nh, g.n_channels))))
                              .astype(np.float32)).to(dev)
    lo = z0 + pitch * (g.n_views - 1) / g.n_views + 1e-6
    hi = z0 + pitch * (nh - g.n_views) / g.n_views - 1e-6
    zs = list(np.linspace(lo, hi, n_slices))
    out = recon.rebin_helical(g, counts, 2e3, pitch, z0, zs)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        recon.rebin_helical(g, counts, 2e3, pitch, z0, zs, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    nbytes = 12.0 * n_slices * g.n_views * g.n_channels
    gbps = nbytes / (ms * 1e-3) / 1e9
    log(f"bench: helical rebinning {ms * 1e3:.1f} us for {n_slices} slices ({gbps:.0f} GB/s, "
        f"{gbps / PEAK_HBM_GBPS:.2f} of HBM peak)")
    return {"slices": n_slices, "views": g.n_views, "channels": g.n_channels, "helical_views": nh,
            "us": ms * 1e3, "gbps": gbps, "frac_of_hbm_peak": gbps / PEAK_HBM_GBPS,
            "bytes_per_output": 12}


def cnn_leg(batch: int, dev):
    """Warm-start network kernels on `batch` 512 x 512 slices: mean launch time (HIP events over
    back-to-back launches on the library's stream) of the 32-channel convolution forward, its
    input-gradient form and the weight-gradient kernel, against the bf16 matrix-core peak and the
    HBM peak; plus a whole forward pass and a whole loss-and-gradient pass."""
    import numpy as np
    import torch

    from paper_1903_10088_amd import phantom as ph
    from paper_1903_10088_amd import recon

    n = 512
    rng = np.random.default_rng(5)
    mu = torch.from_numpy((ph.MU_WATER_PER_MM * (1 + 0.05 * rng.standard_normal((batch, n, n)))).astype(np.float32))
    mu = mu.to(dev)
    tgt = (mu * 1.01).contiguous()
    net = recon.Cnn(ph.cnn_initial_params(0, zero_last=False, last_std=0.05), max_batch=batch, max_n=n,
                    mu_scale=ph.MU_WATER_PER_MM)
    ms = net.time_kernels(mu, tgt, reps=20)
    torch.cuda.synchronize()
    flops = 2.0 * 9 * 32 * 32 * batch * n * n           # one 32 -> 32 layer
    act = float(batch * n * n * 32 * 2)                    # one bf16 activation tensor
    # compulsory tensors: forward reads a_{l-1}, writes a_l; dgrad reads the incoming gradient and
    # the activation its ReLU mask comes from, writes the outgoing gradient; wgrad reads a_{l-1}
    # and the gradient (its 18 KB of weights written are negligible)
    out = {"batch": batch, "n": n}
    for name, t, hbm in zip(("conv32_forward", "conv32_dgrad", "wgrad32"), ms[:3], (2 * act, 3 * act, 2 * act)):
        out[name] = {"us": t * 1e3, "tflops": flops / (t * 1e-3) / 1e12,
                     "frac_of_bf16_peak": flops / (t * 1e-3) / 1e12 / PEAK_BF16_TFLOPS,
                     "gbps_compulsory": hbm / (t * 1e-3) / 1e9,
                     "frac_of_hbm_peak": hbm / (t * 1e-3) / 1e9 / PEAK_HBM_GBPS}
    out["forward_ms"] = ms[3]
    out["loss_grad_ms"] = ms[4]
    out["forward_slices_per_s"] = batch / (ms[3] * 1e-3)
    log(f"bench: cnn conv32 fwd {ms[0] * 1e3:.1f} us ({out['conv32_forward']['tflops']:.0f} TFLOP/s), dgrad "
        f"{ms[1] * 1e3:.1f} us, wgrad {ms[2] * 1e3:.1f} us; forward {ms[3]:.2f} ms, loss+grad {ms[4]:.2f} ms "
        f"for {batch} slices")
    return out


def warm_leg(n_slices: int, weights: str, dev):
    """Warm-start pipeline (10 sub-iterations, network, the record's refining count, a cold start of
    the record's length above the record's limit) on full-study slices (512^2, views U{600..900}, 738 channels, I0
    log-uniform 1e3..1e4), against the plain batched method run to the smallest sub-iteration count
    (grid of 5) that reaches the same mean RMSE to each slice's converged (500-sub-iteration) image."""
    import json as _json

    import numpy as np
    import torch

    from paper_1903_10088_amd import phantom as ph
    from paper_1903_10088_amd import recon
    from paper_1903_10088_amd import warmstart as ws

    if not os.path.exists(weights):
        log(f"bench: no trained weights at {weights}; warm-start leg skipped")
        return None
    meta = os.path.join(os.path.dirname(weights), "train.json")
    rec = _json.load(open(meta)) if os.path.exists(meta) else {}
    ratio = rec.get("residual_ratio_limit", 1.05)
    n_pre, n_refine, n_cold = rec.get("n_pre", 10), rec.get("n_refine", 5), rec.get("n_cold", 500)
    stride = rec.get("check_stride", 1)
    items = ws.config4_items(range(30000, 30000 + n_slices))
    log(f"bench: warm-start leg: {n_slices} slices ...")
    counts = ws.make_counts(items, workers=8)
    iters = ws.EQUAL_RMSE_GRID
    runs = ws.plain_runs(items, counts, iters, chunk=n_slices, device=dev)
    conv = runs[500]
    curve = {k: float(np.mean(ws.disc_rmse(runs[k], conv, 512)) / ph.MU_WATER_PER_MM) for k in iters}
    del runs
    net = recon.Cnn(None, max_batch=n_slices, max_n=512, mu_scale=ph.MU_WATER_PER_MM)  # one pass per batch
    net.load(weights)
    B = recon.Batch([g for g, _, _ in items], 20, 1e-3)
    cts = [torch.from_numpy(c).to(dev) for c in counts]
    i0s = [i0 for _, _, i0 in items]
    imgs = [torch.empty((512, 512), dtype=torch.float32, device=dev) for _ in items]
    # both sides timed under sustained load (back-to-back calls after an untimed stretch of the same calls)
    (_, res, flo, fb), t_warm = ws.timed_steady(
        lambda: B.warm_start(net, cts, i0s, imgs, n_pre, n_refine, n_cold, ratio, check_stride=stride))
    rmse_w = float(np.mean(ws.disc_rmse(torch.stack(imgs), conv, 512)) / ph.MU_WATER_PER_MM)
    n_eq = ws.equal_rmse_count(curve, rmse_w)
    pimgs = B.initial_images(dev)

    def plain():
        B.initial_images_into(pimgs)
        B.run(cts, i0s, pimgs, n_eq)

    _, t_plain = ws.timed_steady(plain)
    out = {"slices": n_slices, "n_pre": n_pre, "n_refine": n_refine, "n_cold": n_cold, "check_stride": stride,
           "warm_slices_per_s": n_slices / t_warm,
           "warm_rmse_to_converged_over_muw": rmse_w, "fallbacks": int(fb.sum()), "residual_ratio_limit": ratio,
           "plain_sub_iterations_at_equal_rmse": n_eq, "plain_rmse_to_converged_over_muw": curve[n_eq],
           "plain_slices_per_s_at_equal_rmse": n_slices / t_plain, "speedup": t_plain / t_warm}
    log(f"bench: warm start {out['warm_slices_per_s']:.1f} slices/s at RMSE {rmse_w:.4f} mu_w "
        f"({out['fallbacks']} fallbacks); plain needs {n_eq} sub-iterations: "
        f"{out['plain_slices_per_s_at_equal_rmse']:.1f} slices/s; speedup {out['speedup']:.2f}")
    return out


if __name__ == "__main__":
    main()
