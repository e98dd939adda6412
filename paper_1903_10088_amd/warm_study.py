"""Trains the warm-start network and evaluates the warm-start pipeline against the plain method.

  python -m paper_1903_10088_amd.warm_study train --out DIR     (training set + training + calibration)
  python -m paper_1903_10088_amd.warm_study eval --weights FILE --out DIR   (full-study evaluation)

train: 2000 seeded clinical-scale slices (512^2 at 0.78125 mm, 800 views, 738
channels, I0 2e3; seeds 10000-11999, 11800-11999 held out); network input =
the plain iterate after 10 sub-iterations, target = after 500 (20 subsets,
beta 1e-3), both from the homogeneous start.  Writes DIR/warm_cnn.bin (the
network file of recon_cnn_save) and DIR/train.json (losses, the calibrated
residual limit, timings).

eval: 256 full-study slices (512^2, views U{600..900}, 738 channels, I0
log-uniform in [1e3, 1e4]; seeds 20000+): each slice's converged image (500
sub-iterations), the plain method's RMSE to it after n sub-iterations, and the
warm-start pipeline (10 + network + the record's refining sub-iterations, cold
fallback) timed as a stream of batches of 32 run back to back, the fallback
cold starts of each batch left running on the batch's own stream while the next
batches' pipelines run (recon_warm_start_async), all awaited at the end.
Per-slice latency comes from the same stream with every call waiting for its
own cold starts: a slice that passes the data-consistency check is done when
its batch's check is (the same pipeline with no fallback, timed), a fallback
slice when its batch's cold starts are.  The plain method at the equal-RMSE
count is timed as the same stream.  The network's own evaluation setting, 40 refining
sub-iterations, is timed the same way against the plain method at its
equal-RMSE count.  Writes DIR/eval.json.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import phantom as ph
from . import recon
from . import warmstart as ws

MU_W = ph.MU_WATER_PER_MM


def cmd_train(args):
    import torch

    dev = torch.device("cuda:0")
    t0 = time.time()
    seeds = list(range(10000, 10000 + args.slices))
    n_hold = args.slices // 10
    items = ws.config3_items(seeds)
    ws.log(f"train: generating {len(items)} count sinograms ...")
    counts = ws.make_counts(items, workers=args.workers)
    ws.log(f"train: counts in {time.time() - t0:.1f} s")
    t1 = time.time()
    runs = ws.plain_runs(items, counts, [args.n_pre, args.n_final], chunk=args.chunk, device=dev)
    t_plain = time.time() - t1
    ws.log(f"train: plain pairs in {t_plain:.1f} s")
    x, y = runs[args.n_pre], runs[args.n_final]
    ntr = len(items) - n_hold
    xtr, ytr, xva, yva = x[:ntr], y[:ntr], x[ntr:], y[ntr:]
    net = recon.Cnn(ph.cnn_initial_params(args.seed), max_batch=args.batch, max_n=512, mu_scale=MU_W)
    base_val = ws.evaluate_loss(net, xva, yva, batch=args.batch)
    ws.log(f"train: held-out loss of the identity map {base_val:.4e}")
    # time one epoch-sized probe to fit the epoch count into the budget
    probe = ws.train(net, xtr[:args.batch * 8], ytr[:args.batch * 8], epochs=1, batch=args.batch, lr=0.0,
                     lr_final=0.0, seed=args.seed, augment=False)
    torch.cuda.synchronize()
    tp = time.time()
    ws.train(net, xtr[:args.batch * 8], ytr[:args.batch * 8], epochs=1, batch=args.batch, lr=0.0, lr_final=0.0,
             seed=args.seed, augment=True)
    torch.cuda.synchronize()
    step_s = (time.time() - tp) / 8
    epochs = max(1, min(args.max_epochs, int(args.train_seconds / (step_s * (ntr // args.batch)))))
    ws.log(f"train: {step_s * 1e3:.1f} ms per step of {args.batch} slices; {epochs} epochs")
    net.set_state(ph.cnn_initial_params(args.seed), np.zeros(recon.Cnn.param_count(), np.float32),
                  np.zeros(recon.Cnn.param_count(), np.float32), 0)
    t2 = time.time()
    hist = ws.train(net, xtr, ytr, epochs=epochs, batch=args.batch, lr=args.lr, lr_final=args.lr * 0.02,
                    seed=args.seed, augment=True, val=(xva, yva))
    t_train = time.time() - t2
    os.makedirs(args.out, exist_ok=True)
    wpath = os.path.join(args.out, "warm_cnn.bin")
    net.save(wpath)
    # fallback limit and cold-start length: the plain method at the warm start's RMSE, on
    # calibration slices drawn like the workload
    citems = ws.calibration_items(args.calibrate)
    calib = ws.calibrate_equal_rmse(citems, ws.make_counts(citems, workers=args.workers), net, args.n_pre,
                                    args.n_refine, n_final=args.n_final, device=dev, check_stride=args.check_stride)
    # held-out RMSE to the converged image: network alone, and after refinement
    out = torch.empty_like(xva)
    net.forward(xva, out, project=True)
    r_in = ws.disc_rmse(xva, yva, 512) / MU_W
    r_net = ws.disc_rmse(out, yva, 512) / MU_W
    rec = dict(slices=len(items), held_out=n_hold, n_pre=args.n_pre, n_final=args.n_final, epochs=epochs,
               batch=args.batch, lr=args.lr, step_ms=step_s * 1e3, train_s=t_train, plain_pairs_s=t_plain,
               loss_identity_val=base_val, history=hist, n_refine=args.n_refine, n_cold=calib["n_cold"],
               residual_ratio_limit=calib["limit"], check_stride=args.check_stride, calibration=calib,
               val_rmse_over_muw=dict(input=float(np.mean(r_in)), network=float(np.mean(r_net))),
               weights=os.path.basename(wpath))
    json.dump(rec, open(os.path.join(args.out, "train.json"), "w"), indent=1)
    ws.log(json.dumps({k: v for k, v in rec.items() if k != "history"}))


def cmd_calibrate(args):
    """Recomputes the fallback limit and the cold-start length of a trained network's record for the
    pipeline (n_pre, network, n_refine) on calibration slices drawn like the workload."""
    import torch

    dev = torch.device("cuda:0")
    rec = json.load(open(args.train_json))
    items = ws.calibration_items(args.calibrate)
    counts = ws.make_counts(items, workers=args.workers)
    net = recon.Cnn(None, max_batch=8, max_n=512, mu_scale=MU_W)
    net.load(args.weights or os.path.join(os.path.dirname(os.path.abspath(args.train_json)), rec["weights"]))
    calib = ws.calibrate_equal_rmse(items, counts, net, rec["n_pre"], args.n_refine, n_final=rec["n_final"],
                                    device=dev, check_stride=args.check_stride)
    for k in ("residual_ratios", "residual_statistic"):
        rec.pop(k, None)
    rec["n_refine"] = args.n_refine
    rec["n_cold"] = calib["n_cold"]
    rec["residual_ratio_limit"] = calib["limit"]
    rec["check_stride"] = args.check_stride
    rec["calibration"] = calib
    os.makedirs(args.out, exist_ok=True)
    json.dump(rec, open(os.path.join(args.out, "train.json"), "w"), indent=1)
    ws.log(json.dumps(calib))


def cmd_eval(args):
    import torch

    dev = torch.device("cuda:0")
    items = ws.config4_items(range(20000, 20000 + args.slices))
    ws.log(f"eval: generating {len(items)} count sinograms ...")
    counts = ws.make_counts(items, workers=args.workers)
    rec = json.load(open(args.train_json)) if args.train_json else {}
    lim = rec.get("residual_ratio_limit", args.ratio)
    if args.n_refine is None:
        args.n_refine = rec.get("n_refine", 5)
    n_cold = rec.get("n_cold", args.n_final)
    stride = rec.get("check_stride", 1)
    # converged images and the plain method's RMSE curve
    iters = sorted(set(args.curve + [args.n_final]))
    runs = ws.plain_runs(items, counts, iters, chunk=args.chunk, device=dev)
    conv = runs[args.n_final]
    curve = {k: float(np.mean(ws.disc_rmse(runs[k], conv, 512)) / MU_W) for k in iters}
    ws.log(f"eval: plain RMSE-to-converged curve {curve}")
    del runs
    # inference only: one network pass covers a whole batch of the study
    net = recon.Cnn(None, max_batch=args.chunk, max_n=512, mu_scale=MU_W)
    net.load(args.weights)
    res = dict(slices=len(items), n_pre=args.n_pre, n_refine=args.n_refine, n_cold=n_cold, residual_ratio_limit=lim,
               check_stride=stride, plain_curve=curve, batches=[])
    warm_imgs = torch.empty_like(conv)
    # every batch is set up before any timing, so that the timed passes run the batches back to back
    # as a stream (ws.stream_times): both methods are timed under the same sustained load
    batches = []
    for c0 in range(0, len(items), args.chunk):
        sub = items[c0:c0 + args.chunk]
        B = recon.Batch([g for g, _, _ in sub], 20, 1e-3)
        cts = [torch.from_numpy(c).to(dev) for c in counts[c0:c0 + args.chunk]]
        i0s = [i0 for _, _, i0 in sub]
        imgs = [warm_imgs[c0 + i] for i in range(len(sub))]
        batches.append((c0, B, cts, i0s, imgs))

    def pipelines(n_refine, limit, n_cold_run, check_stride, async_fallback=False):
        return [lambda b=b: b[1].warm_start(net, b[2], b[3], b[4], args.n_pre, n_refine, n_cold_run, limit,
                                            check_stride=check_stride, async_fallback=async_fallback)
                for b in batches]

    # per-batch latency: the batches up to their data-consistency check (no slice falls back), then
    # the pipeline, each call waiting for its own cold starts
    _, dts_check = ws.stream_times(pipelines(args.n_refine, 1e30, n_cold, stride))
    outs, dts = ws.stream_times(pipelines(args.n_refine, lim, n_cold, stride))
    # throughput: the same stream with each batch's cold starts left running on the batch's own stream
    # (recon_warm_start_async) while the next batches' pipelines run, all awaited at the end
    outs_async, t_total = ws.stream_total(pipelines(args.n_refine, lim, n_cold, stride, async_fallback=True),
                                          lambda: [b[1].wait() for b in batches])
    for (_, rr, _, fb), (_, rra, _, fba) in zip(outs, outs_async):
        assert np.array_equal(fb, fba) and np.array_equal(rr, rra)
    t_sync = float(sum(dts))
    lat, fb_all, r_all = [], [], []
    for (c0, _, cts, _, _), (_, rr, fl, fb), dt, dt_check in zip(batches, outs, dts, dts_check):
        lat += [dt if f else min(dt, dt_check) for f in fb]
        fb_all += list(map(int, fb))
        r_all += list((rr / fl).tolist())
        res["batches"].append(dict(first=c0, slices=len(cts), seconds=dt, seconds_to_check=dt_check,
                                   fallbacks=int(fb.sum())))
        ws.log(f"eval: warm batch {c0}: {dt:.4f} s ({dt_check:.4f} s to the check), {int(fb.sum())} fallbacks")
    r_warm = ws.disc_rmse(warm_imgs, conv, 512) / MU_W
    rmse_w = float(np.mean(r_warm))
    # the network's evaluation setting (40 refining sub-iterations, no fallback): RMSE to converged
    # and data residual (over every view) against the plain method, every slice
    outs40, dts40 = ws.stream_times(pipelines(40, 1e30, args.n_final, 1))
    t40 = float(sum(dts40))
    r40 = [x for (_, rr, fl, _) in outs40 for x in (rr / fl).tolist()]
    rmse40 = float(np.mean(ws.disc_rmse(warm_imgs, conv, 512) / MU_W))
    n_eq40 = ws.equal_rmse_count(curve, rmse40, args.n_final)
    res_refine40 = dict(n_refine=40, rmse_to_converged_over_muw=rmse40, plain_sub_iterations_at_equal_rmse=n_eq40,
                        slices_per_s=len(items) / t40,
                        residual_ratio=dict(median=float(np.median(r40)), max=float(np.max(r40))))
    n_eq = ws.equal_rmse_count(curve, rmse_w, args.n_final)
    # plain batched throughput at n_eq sub-iterations (same batches, same stream timing; each call
    # starts from the homogeneous image)
    plain_imgs = [b[1].initial_images(dev) for b in batches]

    def plain_time(n_iter):
        def run(b, imgs):
            b[1].initial_images_into(imgs)
            b[1].run(b[2], b[3], imgs, n_iter)
        _, dts_p = ws.stream_times([lambda b=b, im=im: run(b, im) for b, im in zip(batches, plain_imgs)])
        return float(sum(dts_p))

    t_plain = plain_time(n_eq)
    t_plain40 = plain_time(n_eq40)
    res_refine40.update(plain_slices_per_s_at_equal_rmse=len(items) / t_plain40, speedup=t_plain40 / t40)
    for b in batches:
        b[1].close()
    res.update(warm=dict(rmse_to_converged_over_muw=rmse_w, slices_per_s=len(items) / t_total,
                         slices_per_s_fallbacks_waited_per_batch=len(items) / t_sync,
                         latency_p50_s=float(np.percentile(lat, 50)), latency_p99_s=float(np.percentile(lat, 99)),
                         fallbacks=int(sum(fb_all)), residual_ratio=dict(median=float(np.median(r_all)),
                                                                         max=float(np.max(r_all)))),
               plain_equal_rmse=dict(sub_iterations=n_eq, rmse_to_converged_over_muw=curve[n_eq],
                                     slices_per_s=len(items) / t_plain),
               speedup=(len(items) / t_total) / (len(items) / t_plain), refine40=res_refine40)
    os.makedirs(args.out, exist_ok=True)
    json.dump(res, open(os.path.join(args.out, "eval.json"), "w"), indent=1)
    ws.log(json.dumps({k: v for k, v in res.items() if k != "batches"}))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sp = ap.add_subparsers(dest="cmd", required=True)
    t = sp.add_parser("train")
    t.add_argument("--out", required=True)
    t.add_argument("--slices", type=int, default=2000)
    t.add_argument("--n-pre", type=int, default=10)
    t.add_argument("--n-final", type=int, default=500)
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--train-seconds", type=float, default=300.0)
    t.add_argument("--max-epochs", type=int, default=60)
    t.add_argument("--calibrate", type=int, default=128)
    t.add_argument("--n-refine", type=int, default=5, help="refining sub-iterations the limit is calibrated for")
    t.add_argument("--check-stride", type=int, default=10, help="the check uses every k-th subset's rays")
    t.add_argument("--chunk", type=int, default=64)
    t.add_argument("--workers", type=int, default=12)
    t.add_argument("--seed", type=int, default=0)
    c = sp.add_parser("calibrate")
    c.add_argument("--out", required=True)
    c.add_argument("--train-json", required=True)
    c.add_argument("--calibrate", type=int, default=128)
    c.add_argument("--n-refine", type=int, default=5)
    c.add_argument("--check-stride", type=int, default=10, help="the check uses every k-th subset's rays")
    c.add_argument("--weights", default=None, help="default: the record's weights file beside it")
    c.add_argument("--workers", type=int, default=12)
    e = sp.add_parser("eval")
    e.add_argument("--out", required=True)
    e.add_argument("--weights", required=True)
    e.add_argument("--train-json", default=None)
    e.add_argument("--ratio", type=float, default=1.05)
    e.add_argument("--slices", type=int, default=256)
    e.add_argument("--n-pre", type=int, default=10)
    e.add_argument("--n-refine", type=int, default=None, help="default: the record's, else 5")
    e.add_argument("--n-final", type=int, default=500)
    e.add_argument("--curve", type=int, nargs="*", default=ws.EQUAL_RMSE_GRID)
    e.add_argument("--chunk", type=int, default=32)
    e.add_argument("--workers", type=int, default=12)
    args = ap.parse_args()
    {"train": cmd_train, "calibrate": cmd_calibrate, "eval": cmd_eval}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
