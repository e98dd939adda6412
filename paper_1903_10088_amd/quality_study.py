"""Image quality of the iterative method against the filtered-backprojection baseline on synthetic
low-contrast slices (the quantities of sections 4.A and 4.E: signal-to-noise and contrast-to-noise
ratios on insert regions, here on seeded ellipse phantoms with known inserts instead of the
phantoms and patients of the paper).

Orchestration only: every reconstruction runs in the library (recon_fbp, recon_os_iterate); this
module draws the slices, defines the regions from the phantom's own ellipses and reduces the
images.  Regions: each insert's ellipse shrunk to 60 % of its semi-axes (pixels of no other insert),
and the background, the body shrunk to 80 % minus every insert grown to 130 %.  SNR = background
mean / background standard deviation; CNR = |insert mean - background mean| / background standard
deviation, averaged over the inserts; RMSE to the rasterised phantom over the reconstruction disc.

    python -m paper_1903_10088_amd.quality_study --out profiles/quality_study_512x800.json
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

import numpy as np

from . import phantom as ph
from . import recon


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _torch():
    import torch
    return torch


def _mask(e: ph.Ellipse, g, scale: float) -> np.ndarray:
    grown = dataclasses.replace(e, a=e.a * scale, b=e.b * scale, value=1.0)
    return ph.rasterize([grown], g.n, g.pixel_mm, supersample=1) > 0


def regions(sl):
    """(background mask, [insert masks]) of a slice from its phantom's ellipses (body first)."""
    g = sl.geometry
    body, inserts = sl.ellipses[0], sl.ellipses[1:]
    bg = _mask(body, g, 0.8)
    masks = []
    for k, e in enumerate(inserts):
        m = _mask(e, g, 0.6)
        for q, o in enumerate(inserts):
            if q != k:
                m &= ~_mask(o, g, 1.0)
        bg &= ~_mask(e, g, 1.3)
        if m.sum() >= 20:
            masks.append(m)
    return bg, masks


def metrics(img: np.ndarray, sl, bg, masks, disc) -> dict:
    b = img[bg]
    sd = float(b.std())
    cnr = [abs(float(img[m].mean()) - float(b.mean())) / sd for m in masks]
    return dict(snr=float(b.mean()) / sd, cnr=float(np.mean(cnr)),
                rmse_truth=float(np.sqrt(np.mean((img - sl.truth)[disc] ** 2))) / ph.MU_WATER_PER_MM)


def run(seeds, i0: float = 2e3, M: int = 20):
    torch = _torch()
    dev = torch.device("cuda:0")
    g = ph.config1_geometry()
    c = 0.5 * (g.n - 1)
    x = np.arange(g.n) - c
    disc = (x[None, :] ** 2 + x[:, None] ** 2) <= (0.5 * g.n) ** 2
    methods = {"fbp": None, "ostv_100_beta1e-3": (100, 1e-3), "ostv_500_beta1e-3": (500, 1e-3)}
    for beta in (0.0, 3e-4, 3e-3):
        methods[f"ostv_500_beta{beta:g}"] = (500, beta)
    per = {k: [] for k in methods}
    times = {}
    for s in seeds:
        sl = ph.make_slice(g, s, i0, low_contrast=True)
        bg, masks = regions(sl)
        counts = torch.from_numpy(sl.counts).to(dev)
        for name, spec in methods.items():
            if spec is None:
                R = recon.Recon(g, M, 1e-3)
                R.fbp(counts, i0)
                torch.cuda.synchronize()
                t = time.perf_counter()
                img = R.fbp(counts, i0)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
            else:
                n_iter, beta = spec
                R = recon.Recon(g, M, beta)
                R.os_iterate(counts, i0, None, n_iter)
                torch.cuda.synchronize()
                t = time.perf_counter()
                img, _ = R.os_iterate(counts, i0, None, n_iter)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
            R.close()
            times.setdefault(name, []).append(dt)
            per[name].append(metrics(img.cpu().numpy().astype(np.float64), sl, bg, masks, disc))
        log(f"quality: slice {s}: " + ", ".join(f"{k} CNR {per[k][-1]['cnr']:.2f}" for k in methods))
    out = {"workload": f"512x512 at 0.78125 mm, 800 views x 738 channels, I0 {i0:g}, {M} subsets, "
                       f"low-contrast phantoms, seeds {list(seeds)}",
           "methods": {}}
    for name in methods:
        rows = per[name]
        out["methods"][name] = {k: float(np.mean([r[k] for r in rows])) for k in rows[0]}
        out["methods"][name]["ms_per_slice"] = 1e3 * float(np.min(times[name]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--seeds", type=int, nargs="*", default=[100, 101, 102, 103])
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = run(a.seeds)
    text = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(json.dumps(res["methods"]))


if __name__ == "__main__":
    main()
