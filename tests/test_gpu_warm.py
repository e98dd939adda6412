"""The warm-start pipeline on the GPU: the full-data residual against the oracle's projector, and
the pipeline's composition (early iterate -> network -> refinement -> residual test -> cold
fallback) against the same steps run one by one, bit for bit, with the fallback forced both
ways from the host through the residual limit."""
import numpy as np
import pytest

import oracle
from paper_1903_10088_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_10088_amd import recon
    recon.lib()
    return torch.device("cuda:0")


def small_batch():
    geoms = [ph.config0_geometry(),
             ph.Geometry(n=96, pixel_mm=400 / 96, n_views=123, n_channels=150),
             ph.Geometry(n=64, pixel_mm=6.25, n_views=64, n_channels=97)]
    slices = [ph.make_slice(g, 500 + i, 10 ** (3.2 + 0.3 * i), low_contrast=True, supersample=1)
              for i, g in enumerate(geoms)]
    return geoms, slices


@pytest.mark.parametrize("k", [0, 1, 2])
def test_data_residual_matches_oracle(dev, k):
    from paper_1903_10088_amd import recon
    geoms, slices = small_batch()
    g, sl = geoms[k], slices[k]
    R = recon.Recon(g, 5, 1e-3)
    counts = torch.from_numpy(sl.counts).to(dev)
    img, _ = R.os_iterate(counts, sl.i0, None, 7)
    out = R.data_residual(counts, sl.i0, img).cpu().numpy()
    ell = oracle.project(g, img.cpu().numpy().astype(np.float64))
    p = np.log(sl.i0 / np.maximum(sl.counts.astype(np.float64), 1.0))
    ref = np.mean((ell - p) ** 2)
    floor = np.mean(1.0 / np.maximum(sl.counts.astype(np.float64), 1.0))
    print(f"slice {k}: residual {out[0]:.6e} (oracle {ref:.6e}), floor {out[1]:.6e}", flush=True)
    assert abs(out[0] - ref) <= 1e-5 * ref
    assert abs(out[1] - floor) <= 1e-12 * floor


@pytest.mark.parametrize("k,stride", [(0, 2), (1, 3), (2, 5), (0, 4)])
def test_strided_residual_matches_oracle(dev, k, stride):
    """Residual over the views of every stride-th subset (subset s holds the views v with
    v mod M = s), against the oracle's projection of those views alone."""
    from paper_1903_10088_amd import recon
    geoms, slices = small_batch()
    g, sl, M = geoms[k], slices[k], 5
    R = recon.Recon(g, M, 1e-3)
    counts = torch.from_numpy(sl.counts).to(dev)
    img, _ = R.os_iterate(counts, sl.i0, None, 7)
    out = R.data_residual(counts, sl.i0, img, stride).cpu().numpy()
    views = np.concatenate([oracle.subset_views(g.n_views, M, s) for s in range(0, M, stride)])
    ell = oracle.project(g, img.cpu().numpy().astype(np.float64), views)
    y = np.maximum(sl.counts[views].astype(np.float64), 1.0)
    ref = np.mean((ell - np.log(sl.i0 / y)) ** 2)
    floor = np.mean(1.0 / y)
    print(f"slice {k} stride {stride}: {len(views)} views, residual {out[0]:.6e} (oracle {ref:.6e}), "
          f"floor {out[1]:.6e}", flush=True)
    assert abs(out[0] - ref) <= 1e-5 * ref
    assert abs(out[1] - floor) <= 1e-12 * floor


def test_strided_residual_limits(dev):
    """Strides outside [1, M], or choosing more than 64 subsets, are refused; stride 1 has no
    subset limit."""
    from paper_1903_10088_amd import recon
    g = ph.Geometry(n=32, pixel_mm=12.5, n_views=130, n_channels=49)
    sl = ph.make_slice(g, 3, 1e4, supersample=1)
    counts = torch.from_numpy(sl.counts).to(dev)
    R = recon.Recon(g, 65, 1e-3)
    img = R.initial_image(dev)
    for bad in (0, 66):
        with pytest.raises(recon.ReconError) as ei:
            R.data_residual(counts, sl.i0, img, bad)
        assert ei.value.status == recon.RECON_INVALID_ARG
    R.data_residual(counts, sl.i0, img, 2)
    R.data_residual(counts, sl.i0, img, 1)
    R130 = recon.Recon(g, 130, 1e-3)
    with pytest.raises(recon.ReconError) as ei:
        R130.data_residual(counts, sl.i0, img, 2)
    assert ei.value.status == recon.RECON_INVALID_ARG
    R130.data_residual(counts, sl.i0, img, 3)


def test_pipeline_equals_its_steps(dev):
    """Identity network: pipeline = n_pre plain sub-iterations, then n_refine from that image with a
    fresh state; no fallback when the limit is generous."""
    from paper_1903_10088_amd import recon
    geoms, slices = small_batch()
    M, beta, n_pre, n_ref = 5, 1e-3, 7, 11
    B = recon.Batch(geoms, M, beta)
    net = recon.Cnn(None, max_batch=2, max_n=128, mu_scale=ph.MU_WATER_PER_MM)
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    i0s = [s.i0 for s in slices]
    imgs, res, flo, fb = B.warm_start(net, counts, i0s, None, n_pre, n_ref, 20, 1e6)
    assert not fb.any()
    ref, _ = B.run(counts, i0s, None, n_pre)
    ref = [r.clone() for r in ref]
    ref, _ = B.run(counts, i0s, ref, n_ref)
    for a, b in zip(imgs, ref):
        assert torch.equal(a, b)
    for k, (g, sl) in enumerate(zip(geoms, slices)):
        R = recon.Recon(g, M, beta)
        r = R.data_residual(counts[k], sl.i0, imgs[k]).cpu().numpy()
        assert r[0] == res[k] and r[1] == flo[k]
    # the check over every second subset: same images, residuals of the single-slice call, bit for bit
    imgs2, res2, flo2, fb2 = B.warm_start(net, counts, i0s, None, n_pre, n_ref, 20, 1e6, check_stride=2)
    assert not fb2.any()
    for k, (g, sl) in enumerate(zip(geoms, slices)):
        assert torch.equal(imgs2[k], imgs[k])
        R = recon.Recon(g, M, beta)
        r = R.data_residual(counts[k], sl.i0, imgs2[k], 2).cpu().numpy()
        assert r[0] == res2[k] and r[1] == flo2[k]
    with pytest.raises(recon.ReconError):
        B.warm_start(net, counts, i0s, None, n_pre, n_ref, 20, 1e6, check_stride=M + 1)


def test_pipeline_falls_back_to_a_cold_start(dev):
    """A limit below every residual sends every slice to the cold start: the result is the plain
    n_cold-sub-iteration reconstruction from the homogeneous start."""
    from paper_1903_10088_amd import recon
    geoms, slices = small_batch()
    M, beta = 5, 1e-3
    B = recon.Batch(geoms, M, beta)
    theta = ph.cnn_initial_params(3, zero_last=False, last_std=0.05)
    net = recon.Cnn(theta, max_batch=2, max_n=128, mu_scale=ph.MU_WATER_PER_MM)
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    imgs, res, flo, fb = B.warm_start(net, counts, [s.i0 for s in slices], None, 4, 6, 13, 1e-9)
    assert fb.all()
    for k, (g, sl) in enumerate(zip(geoms, slices)):
        R = recon.Recon(g, M, beta)
        cold, _ = R.os_iterate(counts[k], sl.i0, None, 13)
        assert torch.equal(imgs[k], cold)


@pytest.mark.parametrize("kind", ["noise", "nan"])
def test_bad_network_falls_back_through_the_check(dev, kind):
    """A broken network (a huge random last layer, or a NaN bias) with the calibrated limit, not a
    forced one: the data-consistency check alone sends every slice to the cold start (a NaN residual
    counts as failing)."""
    import json
    import os

    from paper_1903_10088_amd import recon
    rec = json.load(open(os.path.join(os.path.dirname(recon.__file__), "weights", "train.json")))
    geoms, slices = small_batch()
    M, beta = 5, 1e-3
    B = recon.Batch(geoms, M, beta)
    theta = ph.cnn_initial_params(4, zero_last=False, last_std=2.0)
    if kind == "nan":
        theta = ph.cnn_initial_params(4)
        theta[-1] = np.nan
    net = recon.Cnn(theta, max_batch=2, max_n=128, mu_scale=ph.MU_WATER_PER_MM)
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    imgs, res, flo, fb = B.warm_start(net, counts, [s.i0 for s in slices], None, rec["n_pre"], rec["n_refine"], 13,
                                      rec["residual_ratio_limit"])
    print(f"  {kind} network: residual ratios {res / flo}", flush=True)
    assert fb.all()
    for k, (g, sl) in enumerate(zip(geoms, slices)):
        R = recon.Recon(g, M, beta)
        cold, _ = R.os_iterate(counts[k], sl.i0, None, 13)
        assert torch.equal(imgs[k], cold)


def test_one_fallback_runs_on_its_own_handle(dev):
    """A batch of one slice sent to the cold start (a single fallback slice runs on its own handle,
    not as a batch of one): the result is its plain cold reconstruction."""
    from paper_1903_10088_amd import recon
    geoms, slices = small_batch()
    M, beta = 5, 1e-3
    B = recon.Batch(geoms[1:2], M, beta)
    net = recon.Cnn(None, max_batch=1, max_n=128, mu_scale=ph.MU_WATER_PER_MM)
    counts = [torch.from_numpy(slices[1].counts).to(dev)]
    imgs, _, _, fb = B.warm_start(net, counts, [slices[1].i0], None, 4, 6, 13, 1e-9)
    assert fb.all()
    cold, _ = recon.Recon(geoms[1], M, beta).os_iterate(counts[0], slices[1].i0, None, 13)
    assert torch.equal(imgs[0], cold)


def test_many_fallbacks_go_through_a_batch(dev):
    """Nine slices, all sent to the cold start (the batched cold-start path): each equals its own
    single-slice cold reconstruction."""
    from paper_1903_10088_amd import recon
    geoms = [ph.Geometry(n=48 + 8 * (i % 3), pixel_mm=6.0, n_views=40 + 3 * i, n_channels=70 + i)
             for i in range(9)]
    slices = [ph.make_slice(g, 700 + i, 5e3, low_contrast=True, supersample=1) for i, g in enumerate(geoms)]
    M, beta = 4, 1e-3
    B = recon.Batch(geoms, M, beta)
    net = recon.Cnn(None, max_batch=4, max_n=64, mu_scale=ph.MU_WATER_PER_MM)
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    imgs, _, _, fb = B.warm_start(net, counts, [s.i0 for s in slices], None, 3, 5, 9, 1e-9)
    assert fb.all()
    for k, (g, sl) in enumerate(zip(geoms, slices)):
        R = recon.Recon(g, M, beta)
        cold, _ = R.os_iterate(counts[k], sl.i0, None, 9)
        assert torch.equal(imgs[k], cold), k


def test_trained_network_gains_over_the_plain_method(dev):
    """What the trained network adds, on full-study slices it never saw (seeds 50000+): its output
    is far closer to each slice's converged (500-sub-iteration) image than its input, the
    10-sub-iteration iterate; the pipeline with the record's refinement is closer than the plain
    method at the same sub-iteration count, and passes its data-consistency check."""
    import json
    import os

    from paper_1903_10088_amd import recon
    from paper_1903_10088_amd import warmstart as ws
    wdir = os.path.join(os.path.dirname(recon.__file__), "weights")
    rec = json.load(open(os.path.join(wdir, "train.json")))
    n_pre, n_refine = rec["n_pre"], rec["n_refine"]
    items = ws.config4_items(range(50000, 50004))
    print(f"trained network: {len(items)} unseen 512^2 slices, {n_pre} + network + {n_refine}", flush=True)
    counts = [ph.make_slice(g, s, i0, low_contrast=True, supersample=1).counts for g, s, i0 in items]
    runs = ws.plain_runs(items, counts, [n_pre, n_pre + n_refine, 500], chunk=4, device=dev)
    conv = runs[500]
    net = recon.Cnn(None, max_batch=8, max_n=512, mu_scale=ph.MU_WATER_PER_MM)
    net.load(os.path.join(wdir, rec["weights"]))
    out = torch.empty_like(runs[n_pre])
    net.forward(runs[n_pre].contiguous(), out, project=True)
    B = recon.Batch([g for g, _, _ in items], 20, 1e-3)
    cts = [torch.from_numpy(c).to(dev) for c in counts]
    imgs = [torch.empty((512, 512), device=dev) for _ in items]
    _, rr, fl, fb = B.warm_start(net, cts, [i0 for _, _, i0 in items], imgs, n_pre, n_refine, rec["n_cold"],
                                 rec["residual_ratio_limit"])
    B.close()
    r_in = ws.disc_rmse(runs[n_pre], conv, 512) / ph.MU_WATER_PER_MM
    r_net = ws.disc_rmse(out, conv, 512) / ph.MU_WATER_PER_MM
    r_warm = ws.disc_rmse(torch.stack(imgs), conv, 512) / ph.MU_WATER_PER_MM
    r_plain = ws.disc_rmse(runs[n_pre + n_refine], conv, 512) / ph.MU_WATER_PER_MM
    print(f"  RMSE to converged / mu_w: input {r_in.mean():.4f}, network {r_net.mean():.4f}, "
          f"pipeline {r_warm.mean():.4f}, plain at {n_pre + n_refine} {r_plain.mean():.4f}; "
          f"residual ratios {np.round(rr / fl, 4)}, fallbacks {int(fb.sum())}")
    assert np.all(r_net < 0.5 * r_in)
    assert np.all(r_warm < 0.5 * r_plain)
    assert not fb.any()


def test_async_fallbacks_equal_sync(dev):
    """recon_warm_start_async: with every slice sent to the cold start (three slices: the batched cold
    start; one slice: its own handle) the results after wait() equal recon_warm_start's bit for bit,
    also while another batch's pipeline runs on the caller's stream in between; a later call on the
    batch (a plain run, an allocation-free warm start) first waits for the pending cold starts."""
    from paper_1903_10088_amd import recon
    geoms, slices = small_batch()
    M, beta = 5, 1e-3
    theta = ph.cnn_initial_params(3, zero_last=False, last_std=0.05)
    net = recon.Cnn(theta, max_batch=3, max_n=128, mu_scale=ph.MU_WATER_PER_MM)
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    i0s = [s.i0 for s in slices]
    ref3, res3, _, fb3 = recon.Batch(geoms, M, beta).warm_start(net, counts, i0s, None, 4, 6, 13, 1e-9)
    ref1, _, _, _ = recon.Batch(geoms[1:2], M, beta).warm_start(net, counts[1:2], i0s[1:2], None, 4, 6, 13, 1e-9)
    assert fb3.all()
    A = recon.Batch(geoms, M, beta)
    C = recon.Batch(geoms[1:2], M, beta)
    imgs3, r3, _, f3 = A.warm_start(net, counts, i0s, None, 4, 6, 13, 1e-9, async_fallback=True)
    imgs1, _, _, f1 = C.warm_start(net, counts[1:2], i0s[1:2], None, 4, 6, 13, 1e-9, async_fallback=True)
    assert f3.all() and f1.all() and np.array_equal(r3, res3)
    A.wait()
    C.wait()
    torch.cuda.synchronize()
    for k in range(3):
        assert torch.equal(imgs3[k], ref3[k]), k
    assert torch.equal(imgs1[0], ref1[0])
    # a later call on the batch waits for the pending cold starts first
    A.warm_start(net, counts, i0s, imgs3, 4, 6, 13, 1e-9, async_fallback=True)
    run, _ = A.run(counts, i0s, None, 7)
    fresh, _ = recon.Batch(geoms, M, beta).run(counts, i0s, None, 7)
    torch.cuda.synchronize()
    for k in range(3):
        assert torch.equal(imgs3[k], ref3[k]), k
        assert torch.equal(run[k], fresh[k]), k
    # an allocation-free call after an asynchronous one (it waits without freeing the sub-batch)
    A.warm_start(net, counts, i0s, imgs3, 4, 6, 13, 1e-9, async_fallback=True)
    out, _, _, _ = A.warm_start(net, counts, i0s, None, 4, 6, 13, 1e-9, noalloc=True)
    A.close()
    torch.cuda.synchronize()
    for k in range(3):
        assert torch.equal(out[k], ref3[k]), k
        assert torch.equal(imgs3[k], ref3[k]), k
