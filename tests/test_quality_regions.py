"""Host logic of the image-quality study: the background and insert regions come from the
phantom's own ellipses, are disjoint, and hold uniform true values (water in the background, one
insert value in each insert region)."""
import numpy as np

from paper_1903_10088_amd import phantom as ph
from paper_1903_10088_amd import quality_study as qs


def test_regions_are_disjoint_and_uniform():
    g = ph.config1_geometry()
    sl = ph.make_slice(g, 100, 2e3, low_contrast=True, supersample=1)
    bg, masks = qs.regions(sl)
    assert bg.sum() > 10000 and len(masks) >= 2
    assert np.allclose(sl.truth[bg], ph.MU_WATER_PER_MM)
    seen = bg.copy()
    for m in masks:
        assert not (seen & m).any()
        seen |= m
        vals = sl.truth[m]
        assert np.ptp(vals) == 0.0 and abs(vals[0] / ph.MU_WATER_PER_MM - 1) >= 0.01
    # the study's metrics on the truth itself: no noise, so an infinite SNR / CNR is avoided by a tiny ripple
    rng = np.random.default_rng(0)
    img = sl.truth + rng.normal(0, 1e-5, sl.truth.shape)
    disc = np.ones_like(bg)
    m = qs.metrics(img, sl, bg, masks, disc)
    # contrasts are 1-3 % of water (4.9e-5 .. 1.5e-4 / mm) over a 1e-5 ripple
    assert m["snr"] > 400 and m["cnr"] > 4.5 and m["rmse_truth"] < 0.01
