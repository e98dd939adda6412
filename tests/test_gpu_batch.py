"""Batched reconstruction of uneven slices: every slice of a batch equals the same slice
reconstructed alone, bit for bit, for every launch shape and after autotuning; and a batch slice
meets the oracle parity bar."""
import numpy as np
import pytest

import oracle
from paper_1903_10088_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RMSE_TOL = 1e-4 * ph.MU_WATER_PER_MM


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_10088_amd import recon
    recon.lib()
    return torch.device("cuda:0")


def small_mixed():
    geoms = [ph.config0_geometry(),
             ph.Geometry(n=96, pixel_mm=400 / 96, n_views=123, n_channels=150),
             ph.Geometry(n=37, pixel_mm=10.0, n_views=33, n_channels=51, start_angle_rad=0.3),
             ph.Geometry(n=200, pixel_mm=2.0, n_views=91, n_channels=301),
             ph.Geometry(n=64, pixel_mm=6.25, n_views=64, n_channels=97)]
    slices = [ph.make_slice(g, 300 + i, 10 ** (3 + 0.25 * i), low_contrast=(i % 2 == 1), supersample=1)
              for i, g in enumerate(geoms)]
    return geoms, slices


def realistic_batch(n):
    out = []
    for i in range(n):
        g, i0 = ph.random_batch_geometry(1000 + i)
        out.append((g, ph.make_slice(g, 1000 + i, i0, low_contrast=True, supersample=1)))
    return [g for g, _ in out], [s for _, s in out]


def run_single(dev, g, sl, M, beta, n_iter):
    from paper_1903_10088_amd import recon
    R = recon.Recon(g, M, beta)
    img, tr = R.os_iterate(torch.from_numpy(sl.counts).to(dev), sl.i0, None, n_iter, trace=True)
    return img, tr


def test_mixed_batch_equals_single_slices(dev):
    from paper_1903_10088_amd import recon
    geoms, slices = small_mixed()
    M, beta, n_iter = 5, 1e-3, 13  # two graph epochs and three direct sub-iterations
    B = recon.Batch(geoms, M, beta)
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    imgs, trs = B.run(counts, [s.i0 for s in slices], None, n_iter, trace=True)
    torch.cuda.synchronize()
    for g, sl, img, tr in zip(geoms, slices, imgs, trs):
        print(f"slice n={g.n} views={g.n_views} channels={g.n_channels}", flush=True)
        ref, rtr = run_single(dev, g, sl, M, beta, n_iter)
        assert torch.equal(img, ref)
        assert torch.equal(tr, rtr)


def test_batch_launch_shapes_and_tuning_keep_bits(dev):
    from paper_1903_10088_amd import recon
    geoms, slices = small_mixed()
    M, beta, n_iter = 5, 1e-3, 10
    B = recon.Batch(geoms, M, beta)
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    i0s = [s.i0 for s in slices]
    ref, _ = B.run(counts, i0s, None, n_iter)
    ref = [r.clone() for r in ref]
    for seg, var in [(4, 1), (16, 2), (8, 3), (8, 4), (2, 5), (4, 6)]:
        B.set_launch(seg, var)
        out, _ = B.run(counts, i0s, None, n_iter)
        for a, b in zip(out, ref):
            assert torch.equal(a, b), (seg, var)
    start = B.initial_images(dev)
    seg, var = B.tune(counts, i0s, start, reps=5)
    print("tuned:", seg, var, flush=True)
    assert seg in (4, 8, 16) and 1 <= var <= 6
    out, _ = B.run(counts, i0s, None, n_iter)
    for a, b in zip(out, ref):
        assert torch.equal(a, b)


def test_batch_slice_meets_oracle_bar(dev):
    from paper_1903_10088_amd import recon
    geoms, slices = small_mixed()
    M, beta, n_iter = 5, 1e-3, 15
    B = recon.Batch(geoms, M, beta)
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    imgs, trs = B.run(counts, [s.i0 for s in slices], None, n_iter, trace=True)
    torch.cuda.synchronize()
    for k in (0, 2):
        g, sl = geoms[k], slices[k]
        ref, rtr = oracle.os_iterate(g, M, beta, sl.counts, sl.i0, None, n_iter)
        disc = oracle.initial_image(g, 1.0) > 0
        rmse = float(np.sqrt(np.mean((imgs[k].cpu().numpy() - ref)[disc] ** 2)))
        print(f"slice {k}: rmse {rmse:.2e}", flush=True)
        assert rmse <= RMSE_TOL
        assert np.array_equal(trs[k].cpu().numpy()[:, 1], rtr[:, 1])


def test_realistic_batch_equals_single(dev):
    """Eight helical-rebinned-like slices (256^2 or 512^2, 600-900 views, 520-738 channels,
    I0 1e3-1e4), one epoch of 20 subsets: batch = single, bit for bit."""
    from paper_1903_10088_amd import recon
    geoms, slices = realistic_batch(8)
    M, beta, n_iter = 20, 1e-3, 20
    B = recon.Batch(geoms, M, beta)
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    imgs, _ = B.run(counts, [s.i0 for s in slices], None, n_iter)
    torch.cuda.synchronize()
    for k in (0, 3, 7):
        ref, _ = run_single(dev, geoms[k], slices[k], M, beta, n_iter)
        assert torch.equal(imgs[k], ref), k


@pytest.mark.parametrize("k", [1, 3])
def test_batch_cut_over_xcds_equals_single(dev, k):
    """Batches that whole slices cannot balance over the 8 XCDs (one clinical slice; three
    helical-rebinned-like ones) are cut into parts placed on several XCDs: every slice still equals
    its single-slice run bit for bit, one epoch of 20 subsets, at every projector shape."""
    from paper_1903_10088_amd import recon
    if k == 1:
        g = ph.config1_geometry()
        geoms, slices = [g], [ph.make_slice(g, 100, 2e3, low_contrast=True, supersample=1)]
    else:
        geoms, slices = realistic_batch(3)
    errors, blocks = recon.batch_check_work(geoms, 20, 4)
    assert errors == 0
    M, beta, n_iter = 20, 1e-3, 20
    B = recon.Batch(geoms, M, beta)
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    refs = [run_single(dev, g, sl, M, beta, n_iter)[0] for g, sl in zip(geoms, slices)]
    for seg in (16, 4, 1):
        B.set_launch(fp_segments=seg)
        imgs, _ = B.run(counts, [s.i0 for s in slices], None, n_iter)
        torch.cuda.synchronize()
        for j in range(len(geoms)):
            assert torch.equal(imgs[j], refs[j]), (seg, j)


def test_one_shot_batch_call(dev):
    import ctypes
    from paper_1903_10088_amd import recon
    geoms, slices = small_mixed()
    M, beta, n_iter = 5, 1e-3, 5
    B = recon.Batch(geoms, M, beta)
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    i0s = [s.i0 for s in slices]
    ref, _ = B.run(counts, i0s, None, n_iter)
    imgs = B.initial_images(dev)
    n = len(geoms)
    garr = (recon.Geometry_c * n)(*[recon.geometry_c(g) for g in geoms])
    rc = recon.lib().recon_batch(garr, n, M, beta, None,
                                 recon._ptr_array(counts, torch.float32, B._count_shapes(), "c"),
                                 (ctypes.c_float * n)(*i0s),
                                 recon._ptr_array(imgs, torch.float32, B._img_shapes(), "i"), n_iter,
                                 recon._stream())
    assert rc == recon.RECON_OK
    for a, b in zip(imgs, ref):
        assert torch.equal(a, b)


def test_batch_rejects_bad_subsets(dev):
    from paper_1903_10088_amd import recon
    geoms = [ph.config0_geometry(), ph.Geometry(n=37, pixel_mm=10.0, n_views=33, n_channels=51)]
    with pytest.raises(recon.ReconError) as ei:
        recon.Batch(geoms, 40, 1e-3)  # more subsets than the second slice has views
    assert ei.value.status == recon.RECON_INVALID_ARG


def test_batch_of_several_launch_groups(dev):
    """70 slices, more than one group of the batched start / end kernels (64 slices a launch) and
    more than 64 of one image size for the network's staging copies: start images, run results and
    traces equal the single-slice ones, and the identity-network pipeline equals its steps."""
    from paper_1903_10088_amd import recon
    ga = ph.Geometry(n=37, pixel_mm=10.0, n_views=33, n_channels=51, start_angle_rad=0.3)
    gb = ph.Geometry(n=32, pixel_mm=12.5, n_views=40, n_channels=48)
    geoms = [gb if k in (10, 40, 64, 69) else ga for k in range(70)]
    slices = [ph.make_slice(g, 700 + k, 10 ** (3 + 0.02 * k), low_contrast=True, supersample=1)
              for k, g in enumerate(geoms)]
    M, beta, n_iter = 3, 1e-3, 4
    print(f"batch of {len(geoms)} slices, M={M}", flush=True)
    B = recon.Batch(geoms, M, beta)
    starts = B.initial_images(dev)
    for k in (0, 10, 63, 64, 69):
        assert torch.equal(starts[k], recon.Recon(geoms[k], M, beta).initial_image(dev)), k
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    i0s = [s.i0 for s in slices]
    imgs, trs = B.run(counts, i0s, None, n_iter, trace=True)
    imgs = [x.clone() for x in imgs]
    torch.cuda.synchronize()
    for k in (0, 10, 63, 64, 65, 69):
        ref, rtr = run_single(dev, geoms[k], slices[k], M, beta, n_iter)
        assert torch.equal(imgs[k], ref), k
        assert torch.equal(trs[k], rtr), k
    net = recon.Cnn(None, max_batch=8, max_n=64, mu_scale=ph.MU_WATER_PER_MM)
    w, _, _, fb = B.warm_start(net, counts, i0s, None, n_iter, 2, 3, 1e6)
    assert not fb.any()
    ref, _ = B.run(counts, i0s, [x.clone() for x in imgs], 2)
    for k, (a, b) in enumerate(zip(w, ref)):
        assert torch.equal(a, b), k
