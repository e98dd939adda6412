"""Learned warm start: training-set generation, training and evaluation driver.

Orchestration only.  Every reconstruction step runs in the library's kernels
(recon_batch_run, recon_cnn_train_step, recon_cnn_forward, recon_warm_start,
recon_data_residual); this module draws the seeded inputs, schedules the
calls, and measures the results.

Workflow (the network is trained only on images the plain iteration produced):
  1. `plain_runs`: for each seeded slice, the iterate after n_pre
     sub-iterations (network input) and after n_final (target), both from the
     homogeneous start, by the batched plain method;
  2. `train`: Adam on random minibatches of (input, target) pairs, with the
     eight symmetries of the square (rotations by 90 degrees and flips, which
     map the reconstruction disc onto itself) as augmentation;
  3. `calibrate_equal_rmse`: on training slices, the warm start's mean RMSE to
     the converged image, the smallest sub-iteration count at which the plain
     method reaches it, and the largest ratio of full-data residual to noise
     level (recon_data_residual) of the plain method's images at that count,
     widened by a margin: the limit above which the warm start falls back to a
     cold start (its output must explain the data as well as the plain image it
     stands in for); a slice that falls back is reconstructed by a cold start
     of the full n_final sub-iterations;
  4. `disc_rmse` / `timed`: RMSE to each slice's converged image and
     throughput of the warm-start pipeline (recon_warm_start) and of the plain
     batched method (warm_study.py runs the comparison).
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import os
import sys
import time

import numpy as np

from . import phantom as ph
from . import recon


def _torch():
    import torch
    return torch


def log(*a):
    """Progress lines go to stderr (stdout stays free for results)."""
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Seeded slices (CPU, process pool)
# ---------------------------------------------------------------------------

def _counts_job(args):
    g, seed, i0 = args
    sl = ph.make_slice(g, seed, i0, low_contrast=True, supersample=1)
    return sl.counts


def make_counts(items, workers: int = 12):
    """items: list of (Geometry, seed, I0) -> list of float32 count sinograms (numpy).  Workers are
    spawned (not forked), so they never inherit the parent's GPU state; they use no GPU."""
    import multiprocessing as mp

    workers = max(1, min(workers, len(items), os.cpu_count() or 1))
    if workers == 1:
        return [_counts_job(it) for it in items]
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_counts_job, items, chunksize=4))


def config3_items(seeds):
    """The clinical-scale slice (512^2, 800 views, 738 channels, I0 2e3) for each seed."""
    g = ph.config1_geometry()
    return [(g, int(s), 2e3) for s in seeds]


def calibration_items(n: int = 128):
    """Slices drawn like the full-study workload (config4_items) with seeds of their own (40000+),
    disjoint from the evaluation (20000+) and the benchmark (30000+)."""
    return config4_items(range(40000, 40000 + n))


def config4_items(seeds):
    """Full-study slices: 512^2 at 0.78125 mm, views U{600..900}, 738 channels, I0 log-uniform in [1e3, 1e4]."""
    out = []
    for s in seeds:
        rng = np.random.default_rng([int(s), 7])
        nv = int(rng.integers(600, 901))
        i0 = float(10 ** rng.uniform(3, 4))
        out.append((ph.Geometry(n=512, pixel_mm=400.0 / 512, n_views=nv, n_channels=738), int(s), i0))
    return out


# ---------------------------------------------------------------------------
# Plain-method pairs
# ---------------------------------------------------------------------------

def plain_runs(items, counts, iters, subsets: int = 20, beta: float = 1e-3, chunk: int = 64, device="cuda"):
    """Batched plain reconstructions of every slice from the homogeneous start for each count in
    `iters` (each a fresh run).  Returns {n_iter: float32 CUDA tensor [S][n][n]} (all slices must
    share n)."""
    torch = _torch()
    n = items[0][0].n
    out = {k: torch.empty((len(items), n, n), dtype=torch.float32, device=device) for k in iters}
    for c0 in range(0, len(items), chunk):
        sub = items[c0:c0 + chunk]
        B = recon.Batch([g for g, _, _ in sub], subsets, beta)
        cts = [torch.from_numpy(c).to(device) for c in counts[c0:c0 + chunk]]
        i0s = [i0 for _, _, i0 in sub]
        for k in iters:
            imgs = [out[k][c0 + i] for i in range(len(sub))]
            B.initial_images_into(imgs)
            B.run(cts, i0s, imgs, k)
        torch.cuda.synchronize()
        B.close()
        log(f"plain: {min(c0 + chunk, len(items))}/{len(items)} slices")
    return out


# ---------------------------------------------------------------------------
# Training
# ---------------------------------------------------------------------------

def _symmetry(x, k: int):
    """One of the eight symmetries of the square on [B][n][n] (index ops only)."""
    torch = _torch()
    if k >= 4:
        x = torch.flip(x, dims=(2,))
    return torch.rot90(x, k % 4, dims=(1, 2))


def train(net, inputs, targets, *, epochs: int, batch: int, lr: float, lr_final: float, seed: int = 0,
          augment: bool = True, val=None, log_every: int = 1):
    """Adam on random minibatches; cosine learning-rate decay from lr to lr_final.  val: optional
    (inputs, targets) evaluated (loss only) after every epoch.  Returns a list of per-epoch
    (train_loss, val_loss)."""
    torch = _torch()
    S = inputs.shape[0]
    rng = np.random.default_rng([seed, 3])
    steps_per_epoch = S // batch
    total = epochs * steps_per_epoch
    loss = torch.empty(1, dtype=torch.float64, device=inputs.device)
    hist = []
    step = 0
    for ep in range(epochs):
        perm = rng.permutation(S)
        tl = 0.0
        for b in range(steps_per_epoch):
            idx = torch.from_numpy(perm[b * batch:(b + 1) * batch]).to(inputs.device)
            x, t = inputs[idx], targets[idx]
            if augment:
                k = int(rng.integers(8))
                x, t = _symmetry(x, k).contiguous(), _symmetry(t, k).contiguous()
            cur = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * step / max(1, total)))
            net.train_step(x, t, cur, loss)
            tl += loss.item() if b == steps_per_epoch - 1 or b % 16 == 0 else 0.0
            step += 1
        vl = evaluate_loss(net, *val, batch=batch) if val is not None else float("nan")
        hist.append((loss.item(), vl))
        if (ep + 1) % log_every == 0:
            log(f"train: epoch {ep + 1}/{epochs} last-batch loss {loss.item():.4e} val loss {vl:.4e}")
    return hist


def evaluate_loss(net, inputs, targets, batch: int = 8):
    """Loss (recon_cnn_loss_grad, no update) over a whole set: the minibatch losses weighted by
    their sizes (every image has the same disc, so this is the loss of the set)."""
    torch = _torch()
    loss = torch.empty(1, dtype=torch.float64, device=inputs.device)
    tot = 0.0
    S = inputs.shape[0]
    for b in range(0, S, batch):
        e = min(S, b + batch)
        net.loss_grad(inputs[b:e].contiguous(), targets[b:e].contiguous(), None, loss)
        tot += loss.item() * (e - b)
    return tot / max(S, 1)


EQUAL_RMSE_GRID = list(range(10, 200, 5)) + [200, 250, 300, 400, 500]


def residual_ratios(items, counts, imgs, subsets: int = 20, beta: float = 1e-3, check_stride: int = 1):
    """Residual over its noise level (recon_data_residual) of each slice's image, over the rays of
    every check_stride-th subset."""
    out = []
    for (g, _, i0), c, img in zip(items, counts, imgs):
        R = recon.Recon(g, subsets, beta)
        r = R.data_residual(c, i0, img.contiguous(), check_stride).cpu().numpy()
        out.append(r[0] / r[1])
        R.close()
    return np.asarray(out)


def equal_rmse_count(curve: dict, rmse: float, n_final: int = 500) -> int:
    """Smallest sub-iteration count of the curve {count: mean RMSE} at or below rmse."""
    return next((k for k in sorted(curve) if curve[k] <= rmse), n_final)


def calibrate_equal_rmse(items, counts, net, n_pre: int, n_refine: int, n_final: int = 500, subsets: int = 20,
                         beta: float = 1e-3, margin: float = 0.02, grid=None, device="cuda", check_stride: int = 1):
    """Fallback limit for the pipeline (n_pre, network, n_refine): the plain method's largest
    residual ratio (over the rays of every check_stride-th subset, as the pipeline's check takes
    it) at the sub-iteration count where its mean RMSE to the converged image first reaches the
    pipeline's (no fallback while measuring), times (1 + margin).  Returns a record."""
    torch = _torch()
    grid = sorted(set((grid or EQUAL_RMSE_GRID) + [n_final]))
    cts = [torch.from_numpy(c).to(device) for c in counts]
    i0s = [i0 for _, _, i0 in items]
    runs = plain_runs(items, counts, grid, subsets=subsets, beta=beta, chunk=len(items), device=device)
    conv = runs[n_final]
    n = items[0][0].n
    curve = {k: float(np.mean(disc_rmse(runs[k], conv, n))) / ph.MU_WATER_PER_MM for k in grid}
    B = recon.Batch([g for g, _, _ in items], subsets, beta)
    imgs = [torch.empty((n, n), dtype=torch.float32, device=device) for _ in items]
    _, rr, fl, _ = B.warm_start(net, cts, i0s, imgs, n_pre, n_refine, n_final, 1e30, check_stride=check_stride)
    B.close()
    warm_rmse = float(np.mean(disc_rmse(torch.stack(imgs), conv, n))) / ph.MU_WATER_PER_MM
    n_eq = equal_rmse_count(curve, warm_rmse, n_final)
    plain_r = residual_ratios(items, cts, [runs[n_eq][i] for i in range(len(items))], subsets, beta, check_stride)
    warm_r = rr / fl
    return dict(limit=float(plain_r.max() * (1 + margin)), n_pre=n_pre, n_refine=n_refine, n_cold=n_final,
                check_stride=check_stride,
                warm_rmse_over_muw=warm_rmse, plain_sub_iterations_at_equal_rmse=n_eq,
                plain_ratio=dict(min=float(plain_r.min()), median=float(np.median(plain_r)),
                                 max=float(plain_r.max())),
                warm_ratio=dict(min=float(warm_r.min()), median=float(np.median(warm_r)),
                                max=float(warm_r.max())),
                slices=len(items))


# ---------------------------------------------------------------------------
# Evaluation
# ---------------------------------------------------------------------------

def disc_rmse(a, b, n):
    """Root-mean-square difference over the reconstruction disc, per slice (CUDA tensors [S][n][n])."""
    torch = _torch()
    c = torch.arange(n, device=a.device, dtype=torch.float64) - 0.5 * (n - 1)
    D = (c[None, :] ** 2 + c[:, None] ** 2) <= (0.5 * n) ** 2
    d = (a.double() - b.double())[:, D]
    return torch.sqrt((d * d).mean(dim=1)).cpu().numpy()


def timed(fn):
    torch = _torch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t


# The GPU runs a batch's first sub-iterations after an idle gap up to a quarter slower than under
# sustained load (its clocks settle after some 40 ms of continuous work), so a short pipeline timed
# after a gap pays a cost that a longer plain run mostly hides.  Throughput is timed as a stream: the
# calls run back to back, after an untimed pass of at least STEADY_S seconds of the same calls.
STEADY_S = 0.1


def stream_times(fns, min_s: float = STEADY_S):
    """Run the callables `fns` (one per batch) back to back as a stream and time each call.  An
    untimed warm-up repeats the whole stream until it has lasted `min_s` seconds; the timed pass
    follows without a gap.  Returns (results, seconds per call)."""
    torch = _torch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    while True:
        for f in fns:
            f()
        torch.cuda.synchronize()
        if time.perf_counter() - t >= min_s:
            break
    res, dts = [], []
    for f in fns:
        t = time.perf_counter()
        res.append(f())
        torch.cuda.synchronize()
        dts.append(time.perf_counter() - t)
    return res, dts


def stream_total(fns, finish, min_s: float = STEADY_S):
    """Wall time of one pass of the callables `fns` run back to back followed by `finish()` (which waits
    for work they left running, e.g. asynchronous cold starts), after untimed passes of the same that
    last at least `min_s` seconds.  No synchronisation between the calls.  Returns (results, seconds)."""
    torch = _torch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    while True:
        for f in fns:
            f()
        finish()
        torch.cuda.synchronize()
        if time.perf_counter() - t >= min_s:
            break
    t = time.perf_counter()
    res = [f() for f in fns]
    finish()
    torch.cuda.synchronize()
    return res, time.perf_counter() - t


def timed_steady(fn, min_s: float = STEADY_S):
    """Seconds per call of `fn` under sustained load: `fn` is repeated until `min_s` seconds have
    passed, then the same number of back-to-back calls is timed.  Returns (last result, seconds per
    call)."""
    torch = _torch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    n = 0
    while True:
        fn()
        n += 1
        torch.cuda.synchronize()
        if time.perf_counter() - t >= min_s:
            break
    t = time.perf_counter()
    for _ in range(n):
        r = fn()
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t) / n
