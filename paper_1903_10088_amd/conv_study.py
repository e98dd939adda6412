"""Convergence study of the plain method on 512 x 512 slices (sections 3.C.2, 3.D and 4.B-4.D):
the squared difference between projection and reprojection over the whole sinogram against the
sub-iteration count, for the step-rule readings, a constant step, the three homogeneous initial
images, the thinning factors and fewer projection data -- every other view, half a turn and a
fan-beam short scan (section 4's reconstructions from half of the projection data) -- (Fig. 3's
quantities), the kept best-epoch iterate, and the time to reconstruct one slice at each thinning
factor (Table I's quantity).

Orchestration only: every reconstruction step runs in the library (recon_os_iterate_ex,
recon_data_residual); this module draws the seeded slices, schedules the calls and reduces the
results.  The squared difference is reported as r / v, the full-data mean of (l - p)^2 over its
Poisson noise level (recon_data_residual), so that 1 means "explains the data to the noise".

    python -m paper_1903_10088_amd.conv_study --out profiles/convergence_study_512x800.json
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import sys
import time

import numpy as np

from . import phantom as ph
from . import recon

MU_PER_CM_TO_MM = 0.1
PAPER_TABLE1_GPU_S = {1: 11.00, 2: 7.76, 5: 5.37, 10: 4.30, 20: 3.71, 40: 3.39}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _torch():
    import torch
    return torch


def checkpoints(n_total: int):
    pts = list(range(5, 50, 5)) + list(range(50, 200, 10)) + list(range(200, 500, 25)) + \
        list(range(500, 3001, 50))
    return [p for p in pts if p <= n_total]


class Case:
    """One seeded slice on the device: counts, truth and the reconstruction disc."""

    def __init__(self, g, seed: int, i0: float, dev, view_stride: int = 1, first_views: int = 0):
        torch = _torch()
        sl = ph.make_slice(g, seed, i0, low_contrast=True)
        if first_views:
            # the first views of the turn, at the full turn's spacing: limited-angle data over an
            # arc of 2 pi first_views / n_views (the same measured rows)
            counts = sl.counts[:first_views]
            self.g = dataclasses.replace(g, n_views=first_views,
                                         scan_arc_rad=2 * math.pi * first_views / g.n_views)
        else:
            counts = sl.counts[::view_stride]  # every view_stride-th view: still equally spaced over the turn
            self.g = dataclasses.replace(g, n_views=counts.shape[0])
        self.seed, self.i0 = seed, i0
        self.counts = torch.from_numpy(np.ascontiguousarray(counts)).to(dev)
        self.truth = torch.from_numpy(sl.truth).to(dev)
        c = torch.arange(g.n, device=dev, dtype=torch.float64) - 0.5 * (g.n - 1)
        self.disc = (c[None, :] ** 2 + c[:, None] ** 2) <= (0.5 * g.n) ** 2

    def rmse_to_truth(self, img) -> float:
        d = (img.double() - self.truth)[self.disc]
        return float((d * d).mean().sqrt()) / ph.MU_WATER_PER_MM


def track(case: Case, M: int, beta: float, n_total: int, params: dict | None = None):
    """Runs n_total sub-iterations from the homogeneous start in chunks ending at the checkpoints
    (resumed runs are bitwise equal to uninterrupted ones) and records, at each checkpoint, r / v,
    the RMSE to the phantom and lambda; also the per-epoch mean of the subset squared differences
    and of lambda, and with keep_best the kept epoch."""
    torch = _torch()
    p = dict(params or {})
    R = recon.Recon(case.g, M, beta, p)
    dev = case.counts.device
    img = R.initial_image(dev)
    st = recon.State()
    hist = torch.zeros(M, dtype=torch.float64, device=dev) if p.get("lambda_compare") else None
    best = torch.zeros_like(img) if p.get("keep_best") else None
    rows, traces, done, numeric = [], [], 0, None
    for n in checkpoints(n_total):
        try:
            _, tr = R.os_iterate(case.counts, case.i0, img, n - done, state=st, trace=True, f_hist=hist,
                                 best=best)
        except recon.ReconError as e:
            if e.status != recon.RECON_NUMERIC:
                raise
            numeric = n  # a non-finite squared difference: the run diverged; stop tracking it
            break
        traces.append(tr)
        done = n
        res = R.data_residual(case.counts, case.i0, img).cpu().numpy()
        rows.append((n, float(res[0] / res[1]), case.rmse_to_truth(img), st.lam))
    tr = torch.cat(traces).cpu().numpy() if traces else np.zeros((0, 2))
    ne = tr.shape[0] // M
    out = {"n": [r[0] for r in rows], "r_over_v": [r[1] for r in rows], "rmse_truth": [r[2] for r in rows],
           "lambda": [r[3] for r in rows],
           "epoch_mean_f": tr[:ne * M, 0].reshape(ne, M).mean(axis=1).tolist(),
           "epoch_mean_lambda": tr[:ne * M, 1].reshape(ne, M).mean(axis=1).tolist(), "diverged_at": numeric}
    if best is not None:
        res = R.data_residual(case.counts, case.i0, best).cpu().numpy()
        out["kept"] = {"best_n": st.best_n, "r_over_v": float(res[0] / res[1]),
                       "rmse_truth": case.rmse_to_truth(best)}
    R.close()
    return out


def time_slice(case: Case, M: int, beta: float, n_iter: int, reps: int = 5) -> float:
    """Seconds for one uninterrupted reconstruction of n_iter sub-iterations (best of reps)."""
    torch = _torch()
    R = recon.Recon(case.g, M, beta)
    img0 = R.initial_image(case.counts.device)
    best = None
    for k in range(reps + 1):
        img = img0.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        R.os_iterate(case.counts, case.i0, img, n_iter)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        if k > 0:  # the first run captures the graphs
            best = dt if best is None else min(best, dt)
    R.close()
    return best


def first_reaching(track_out: dict, target: float):
    """First checkpoint at which r / v is at or below target (None if never)."""
    for n, r in zip(track_out["n"], track_out["r_over_v"]):
        if r <= target:
            return n
    return None


def mean_tracks(tracks):
    """Average over slices of the checkpoint series (all tracks share the checkpoints; a diverged
    track shortens the series to its last finite checkpoint)."""
    L = min(len(t["n"]) for t in tracks)
    out = {"n": tracks[0]["n"][:L], "diverged_at": [t["diverged_at"] for t in tracks]}
    for k in ("r_over_v", "rmse_truth", "lambda"):
        out[k] = np.mean([t[k][:L] for t in tracks], axis=0).tolist()
    m = min(len(t["epoch_mean_f"]) for t in tracks)
    out["epoch_mean_f"] = np.mean([t["epoch_mean_f"][:m] for t in tracks], axis=0).tolist()
    if "kept" in tracks[0]:
        out["kept"] = {"best_n": [t["kept"]["best_n"] for t in tracks],
                       "r_over_v": float(np.mean([t["kept"]["r_over_v"] for t in tracks])),
                       "rmse_truth": float(np.mean([t["kept"]["rmse_truth"] for t in tracks]))}
    return out


def run(seeds, beta: float = 1e-3, i0: float = 2e3, M: int = 20, n_long: int = 1500, n_std: int = 500):
    torch = _torch()
    dev = torch.device("cuda:0")
    g = ph.config1_geometry()
    log(f"study: {len(seeds)} slices ...")
    cases = [Case(g, s, i0, dev) for s in seeds]
    half = [Case(g, s, i0, dev, view_stride=2) for s in seeds]
    # limited angle: half a turn (400 views) and a short scan, half a turn plus the fan
    n_short = math.ceil(g.n_views * (math.pi + 2 * g.gamma_max) / (2 * math.pi))
    half_turn = [Case(g, s, i0, dev, first_views=g.n_views // 2) for s in seeds]
    short = [Case(g, s, i0, dev, first_views=n_short) for s in seeds]
    mu0 = lambda cm: dict(mu0_per_mm=cm * MU_PER_CM_TO_MM)  # noqa: E731
    const = dict(lambda_inc=0.0, lambda_dec=0.0)

    variants = {
        # step rule (all from 0.05 / cm, M = 20)
        "adaptive": (cases, M, n_long, dict(keep_best=1)),
        "adaptive_same_subset": (cases, M, n_long, dict(lambda_compare=1, keep_best=1)),
        "constant_0.01": (cases, M, n_long, dict(const, keep_best=1)),
        # initial image (adaptive, M = 20)
        "adaptive_mu0_0": (cases, M, n_std, mu0(0.0)),
        "adaptive_mu0_0.1": (cases, M, n_std, mu0(0.1)),
        "constant_0.01_mu0_0": (cases, M, n_long, dict(const, **mu0(0.0))),
        # half of the views (every other one), subsets of the same 40 views
        "half_views_M10": (half, M // 2, n_std, {}),
        # limited angle, subsets of about 40 views
        "half_turn_M10": (half_turn, M // 2, n_std, {}),
        f"short_scan_M{round(n_short / 40)}": (short, round(n_short / 40), n_std, {}),
    }
    for m in (1, 2, 5, 10, 40):  # thinning factors (M = 20 is "adaptive")
        variants[f"thinning_M{m}"] = (cases, m, 1000 if m == 40 else n_std, {})

    out = {"workload": f"512x512 at 0.78125 mm, 800 views x 738 channels, I0 {i0:g}, beta {beta:g}, "
                       f"low-contrast phantoms, seeds {list(seeds)}",
           "variants": {}}
    for name, (cs, m, n, p) in variants.items():
        t = time.perf_counter()
        tracks = [track(c, m, beta, n, p) for c in cs]
        out["variants"][name] = dict(M=m, params=p, **mean_tracks(tracks))
        log(f"study: {name} ({m} subsets, {n} sub-iterations) in {time.perf_counter() - t:.1f} s; "
            f"r/v at end {out['variants'][name]['r_over_v'][-1]:.4f}")

    # Table I's quantity: seconds per slice at 500 sub-iterations for each thinning factor
    table = {}
    for m in (1, 2, 5, 10, 20, 40):
        s = time_slice(cases[0], m, beta, n_std)
        table[m] = {"s_per_slice": s, "paper_gtx1080ti_s": PAPER_TABLE1_GPU_S[m],
                    "ratio_to_paper": PAPER_TABLE1_GPU_S[m] / s}
        log(f"study: M={m}: {s * 1e3:.1f} ms per slice ({table[m]['ratio_to_paper']:.0f}x the paper's GPU row)")
    out["table1_s_per_slice_500"] = table

    # summary: the adaptive rule against a constant step, and the thinning factors at equal data fit
    V = out["variants"]
    idx500 = V["adaptive"]["n"].index(n_std)
    target = V["adaptive"]["r_over_v"][idx500]
    summ = {"target_r_over_v": target, "sub_iterations_to_target": {}, "least_rmse_truth": {}}
    for name, v in V.items():
        summ["sub_iterations_to_target"][name] = first_reaching(v, target * 1.001)
        k = int(np.argmin(v["rmse_truth"]))
        summ["least_rmse_truth"][name] = {"rmse": v["rmse_truth"][k], "at": v["n"][k]}
    a = summ["sub_iterations_to_target"]
    if a.get("constant_0.01_mu0_0"):
        summ["adaptive_vs_constant_from_zero"] = a["constant_0.01_mu0_0"] / n_std
    if a.get("constant_0.01"):
        summ["adaptive_vs_constant"] = a["constant_0.01"] / n_std
    out["summary"] = summ
    return out


def compact(x, digits: int = 5):
    """The record with floats rounded to `digits` significant digits."""
    if isinstance(x, float):
        return float(f"{x:.{digits}g}")
    if isinstance(x, (list, tuple)):
        return [compact(y, digits) for y in x]
    if isinstance(x, dict):
        return {k: compact(v, digits) for k, v in x.items()}
    return x


LABELS = {
    "adaptive": "adaptive, literal comparison (default)",
    "adaptive_same_subset": "adaptive, same-subset comparison",
    "constant_0.01": "constant lambda 0.01",
    "adaptive_mu0_0": "adaptive, mu0 = 0",
    "adaptive_mu0_0.1": "adaptive, mu0 = 0.1 / cm",
    "constant_0.01_mu0_0": "constant 0.01, mu0 = 0",
    "half_views_M10": "every other view (400 views over the turn)",
    "half_turn_M10": "half a turn (the first 400 views, arc pi)",
}


def markdown(res: dict, out_name: str) -> str:
    """The record's tables as markdown: every variant at 100 and 500 sub-iterations, its least RMSE
    to the phantom and its sub-iterations to the literal rule's data fit, then Table I's quantity."""
    V = res["variants"]
    S = res["summary"]

    def at(v, key, n):
        return v[key][v["n"].index(n)] if n in v["n"] else float("nan")

    lines = [f"# Convergence study: {res['workload']}", "",
             "Command (GPU, about half a minute):", "", "```",
             f"python -m paper_1903_10088_amd.conv_study --out {out_name}", "```", "",
             "`r/v`: full-data mean of (l - p)^2 over its Poisson noise level (`recon_data_residual`), on each "
             "variant's own views; 1 = the image explains the data to the noise, below 1 it fits the noise. `RMSE`: "
             "to the rasterised phantom over the disc, in units of mu_water. All runs from the homogeneous start; "
             "means over the slices. \"to target\" = first checkpoint at which r/v is at or below the literal "
             f"adaptive rule's value after 500 sub-iterations ({S['target_r_over_v']:.4f}; comparable only between "
             "variants with the same views).", "",
             "| variant | M | r/v @100 | r/v @500 | RMSE @100 | RMSE @500 | least RMSE (at) | lambda @500 | to target |",
             "|---|---|---|---|---|---|---|---|---|"]
    for name, v in V.items():
        label = LABELS.get(name, name)
        if name.startswith("short_scan"):
            label = "short scan (half a turn plus the fan: the first views over pi + 2 gamma_max)"
        elif name.startswith("thinning_M"):
            m = int(name[len("thinning_M"):])
            label = f"thinning 1/{m}" if m > 1 else "thinning 1"
        least = S["least_rmse_truth"][name]
        tgt = S["sub_iterations_to_target"][name]
        lines.append(f"| {label} | {v['M']} | {at(v, 'r_over_v', 100):.4g} | {at(v, 'r_over_v', 500):.4g} | "
                     f"{at(v, 'rmse_truth', 100):.4g} | {at(v, 'rmse_truth', 500):.4g} | "
                     f"{least['rmse']:.4g} ({least['at']}) | {at(v, 'lambda', 500):.2g} | "
                     f"{tgt if tgt is not None else 'never'} |")
    kept = {name: v["kept"]["best_n"] for name, v in V.items() if "kept" in v}
    if kept:
        lines += ["", "Best-epoch iterate (keep_best): sub-iterations of the kept image per slice -- " +
                  "; ".join(f"{LABELS.get(k, k)}: {b}" for k, b in kept.items()) +
                  " (the last epoch whenever the epoch sums of f keep falling)."]
    T = res["table1_s_per_slice_500"]
    ms = sorted(T, key=lambda k: int(k))
    lines += ["", "Time per slice, 500 sub-iterations, one slice per launch (Table I's quantity; the paper's "
              "GTX 1080 Ti row for context only):", "",
              "| thinning | " + " | ".join("1" if int(m) == 1 else f"1/{m}" for m in ms) + " |",
              "|---|" + "---|" * len(ms),
              "| MI355X, this library (s) | " + " | ".join(f"{T[m]['s_per_slice']:.3g}" for m in ms) + " |",
              "| paper, GTX 1080 Ti (s) | " + " | ".join(f"{T[m]['paper_gtx1080ti_s']:.2f}" for m in ms) + " |", ""]
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--seeds", type=int, nargs="*", default=[100, 101, 102, 103])
    ap.add_argument("--beta", type=float, default=1e-3)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = run(a.seeds, beta=a.beta)
    res = compact(res)
    res["table1_s_per_slice_500"] = {str(k): v for k, v in res["table1_s_per_slice_500"].items()}
    if a.out:
        with open(a.out.rsplit(".", 1)[0] + ".md", "w") as f:
            f.write(markdown(res, a.out))
        with open(a.out, "w") as f:  # one line per variant
            f.write("{\n")
            items = [(k, v) for k, v in res.items() if k != "variants"]
            for k, v in items:
                f.write(f" {json.dumps(k)}: {json.dumps(v)},\n")
            f.write(' "variants": {\n')
            vs = list(res["variants"].items())
            for i, (k, v) in enumerate(vs):
                f.write(f"  {json.dumps(k)}: {json.dumps(v)}{',' if i + 1 < len(vs) else ''}\n")
            f.write(" }\n}\n")
    print(json.dumps(res["summary"]))


if __name__ == "__main__":
    main()
