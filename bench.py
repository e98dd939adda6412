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


def measured_traffic(kernel: str):
    """HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE) recorded in profiles/, or None when
    the kernel's sources have changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic_512x800.json")
    try:
        rec = json.load(open(path))["kernels"][kernel]
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest()[:16] != rec["source_sha"]:
            return None
        return rec["fetch_bytes"] + rec["write_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=500, help="sub-iterations per reconstruction")
    ap.add_argument("--beta", type=float, default=1e-3)
    ap.add_argument("--cpu-iters", type=int, default=100,
                    help="sub-iterations of the oracle timed for the CPU baseline (0 = skip)")
    ap.add_argument("--time-iters", type=int, default=100, help="sub-iterations of the per-kernel timing pass")
    ap.add_argument("--fp-segments", type=int, default=0)
    ap.add_argument("--bp-variant", type=int, default=0, help="1 = global reads, 2 = LDS-staged (0 = default)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 10 plain device copies of MIB MiB (reference for HBM byte counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (slices shard across GPUs with no "
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
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    slices_per_s = args.steps / elapsed
    log(f"bench: {ms_per_step:.2f} ms per slice, {slices_per_s:.2f} slices/s")

    # Per-kernel durations: each kernel launched time_iters times back to back on
    # the library's stream (torch's current stream) between two HIP events.
    if args.time_iters > 0:
        kimg = R.initial_image(dev)
        fp_ms, _, bp_ms = R.time_kernels(counts, i0, kimg, args.time_iters)
        torch.cuda.synchronize()
    else:
        fp_ms = bp_ms = float("nan")
    # Algorithmic bytes per launch (per unit: 4 B per ray-pixel interpolation
    # pair read; projector 12 B per ray for y/I0 and p read and w written;
    # update 8 B per pixel for mu read and mu' written), averaged over subsets.
    n_rays = [R.subset_size(s) * g.n_channels for s in range(M)]
    pairs = [R.count_pairs(s) for s in range(M)]
    npix = g.n * g.n
    fp_bytes = np.mean([4 * p + 12 * r for p, r in zip(pairs, n_rays)])
    bp_bytes = np.mean([4 * p + 8 * npix for p in pairs])
    fp_gbps = fp_bytes / (fp_ms * 1e-3) / 1e9
    bp_gbps = bp_bytes / (bp_ms * 1e-3) / 1e9
    sub_ms = ms_per_step / args.iters
    slice_bytes = args.iters * (fp_bytes + bp_bytes)
    log(f"bench: kernels fp {fp_ms * 1e3:.1f} us ({fp_gbps:.0f} GB/s alg), step rule + bp + tv + update "
        f"{bp_ms * 1e3:.1f} us ({bp_gbps:.0f} GB/s alg); graph sub-iteration {sub_ms * 1e3:.1f} us")
    if bp_ms >= fp_ms:
        dom = dict(name="bp_update_kernel", ms=bp_ms, bytes=bp_bytes, gbps=bp_gbps)
    else:
        dom = dict(name="fp_kernel<OS>", ms=fp_ms, bytes=fp_bytes, gbps=fp_gbps)
    traffic = measured_traffic(dom["name"])

    cpu = None
    parity = None
    if args.cpu_iters > 0:
        import oracle

        n_cpu = min(args.cpu_iters, args.iters)
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
        "roofline": {"bound": "hbm", "kernel": dom["name"], "achieved": dom["gbps"], "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": dom["gbps"] / PEAK_HBM_GBPS, "traffic": traffic,
                     "alg_bytes_per_launch": dom["bytes"], "avg_launch_us": dom["ms"] * 1e3},
        "cpu_baseline": cpu,
        "projector_gbps": fp_gbps,
        "projector_frac_of_hbm_peak": fp_gbps / PEAK_HBM_GBPS,
        "slice_alg_gbps": slice_bytes / (ms_per_step * 1e-3) / 1e9,
        "kernel_us": {"fp": fp_ms * 1e3, "bp_update": bp_ms * 1e3,
                      "graph_sub_iteration": sub_ms * 1e3},
        "parity": parity,
        "paper_context": {"s_per_slice": PAPER_S_PER_SLICE, "hardware": "GeForce GTX 1080 Ti",
                          "thinning": "1/20", "note": "context only; channel count and precision not stated"},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
