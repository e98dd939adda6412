"""The allocation-free warm start (recon_warm_start_noalloc) against recon_warm_start, through the
C ABI: the same images bit for bit, the same residuals, noise levels and fallback decisions, over
consecutive calls that share the GPU's scratch array, each smaller than the one before (the
first stages its images in several chunks, the later ones find the previous call's contents in
the scratch)."""
import numpy as np
import pytest

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


def case(kind):
    if kind == "chunked":  # five 1024^2 slices: the 16 MiB stage holds four
        geoms = [ph.Geometry(n=1024, pixel_mm=400 / 1024, n_views=48 + 4 * i, n_channels=257) for i in range(5)]
    elif kind == "mixed":
        geoms = [ph.config0_geometry(),
                 ph.Geometry(n=96, pixel_mm=400 / 96, n_views=123, n_channels=150),
                 ph.Geometry(n=64, pixel_mm=6.25, n_views=64, n_channels=97),
                 ph.Geometry(n=96, pixel_mm=400 / 96, n_views=90, n_channels=131, scan_arc_rad=4.0)]
    else:  # smaller than both
        geoms = [ph.Geometry(n=48, pixel_mm=400 / 48, n_views=40, n_channels=61),
                 ph.Geometry(n=64, pixel_mm=6.25, n_views=33, n_channels=71)]
    slices = [ph.make_slice(g, 700 + 10 * i + len(geoms), 10 ** (3.1 + 0.2 * i), low_contrast=True, supersample=1)
              for i, g in enumerate(geoms)]
    return geoms, slices


def compare(dev, kind, net, stride=1):
    from paper_1903_10088_amd import recon
    geoms, slices = case(kind)
    M, beta, n_pre, n_ref, n_cold = 4, 1e-3, 6, 5, 9
    counts = [torch.from_numpy(s.counts).to(dev) for s in slices]
    i0s = [s.i0 for s in slices]
    # the residual limit at the median ratio, so some slices fall back and some do not
    probe = recon.Batch(geoms, M, beta)
    _, res, flo, _ = probe.warm_start(net, counts, i0s, None, n_pre, n_ref, n_cold, 1e6, check_stride=stride)
    r = np.sort(res / flo)
    k = len(geoms) // 2
    limit = float(0.5 * (r[k - 1] + r[k]))
    ref_b = recon.Batch(geoms, M, beta)
    ref = ref_b.warm_start(net, counts, i0s, None, n_pre, n_ref, n_cold, limit, check_stride=stride)
    torch.cuda.synchronize()
    ref_imgs = [r.clone() for r in ref[0]]
    # a fresh batch (no epoch graphs yet: every sub-iteration launched directly) and the reference
    # batch again (its graphs replayed)
    for label, B in (("fresh batch", recon.Batch(geoms, M, beta)), ("same batch", ref_b)):
        out = B.warm_start(net, counts, i0s, None, n_pre, n_ref, n_cold, limit, noalloc=True, check_stride=stride)
        torch.cuda.synchronize()
        print(f"{kind}, {label}, check stride {stride}: {len(geoms)} slices, fallbacks {out[3].tolist()}",
              flush=True)
        assert 0 < out[3].sum() < len(geoms)
        for k in range(len(geoms)):
            assert torch.equal(out[0][k], ref_imgs[k]), (kind, label, k)
        assert np.array_equal(out[1], ref[1]) and np.array_equal(out[2], ref[2])
        assert np.array_equal(out[3], ref[3])


def test_noalloc_warm_start_equals_warm_start(dev):
    from paper_1903_10088_amd import recon
    theta = ph.cnn_initial_params(7, zero_last=False, last_std=0.05)
    big = recon.Cnn(theta, max_batch=2, max_n=1024, mu_scale=ph.MU_WATER_PER_MM)
    compare(dev, "chunked", big)
    small = recon.Cnn(theta, max_batch=2, max_n=128, mu_scale=ph.MU_WATER_PER_MM)
    compare(dev, "mixed", small)
    compare(dev, "smaller", small, stride=2)


def test_noalloc_rejects_images_beyond_the_scratch(dev):
    """An image above 2048 x 2048 does not fit the scratch stage: RECON_INVALID_ARG, nothing run."""
    from paper_1903_10088_amd import recon
    g = ph.Geometry(n=2050, pixel_mm=400 / 2050, n_views=8, n_channels=33)
    B = recon.Batch([g], 4, 1e-3)
    net = recon.Cnn(None, max_batch=1, max_n=64, mu_scale=ph.MU_WATER_PER_MM)
    counts = [torch.full((g.n_views, g.n_channels), 1e3, device=dev)]
    with pytest.raises(recon.ReconError) as ei:
        B.warm_start(net, counts, [1e4], None, 1, 1, 1, 1.0, noalloc=True)
    assert ei.value.status == recon.RECON_INVALID_ARG
    assert "2048" in str(ei.value)
