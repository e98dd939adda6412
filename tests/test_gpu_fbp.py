"""GPU parity of the filtered-backprojection baseline (recon_fbp) against the FP64 oracle.

Bar: relative L2 error over the whole image <= 1e-5 against oracle.fbp of the same measured line
integrals ln(I0 / max(y, 1)); bitwise determinism; the channel limit of the filter.
"""
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


GEOMS = {
    "config0": ph.config0_geometry(),
    "odd-rotated": ph.Geometry(n=37, pixel_mm=10.0, n_views=33, n_channels=51, start_angle_rad=0.3),
    "n200": ph.Geometry(n=200, pixel_mm=2.0, n_views=90, n_channels=301),
    "config1": ph.config1_geometry(),
}


@pytest.mark.parametrize("name", list(GEOMS))
def test_fbp_matches_oracle(dev, name):
    from paper_1903_10088_amd import recon
    g = GEOMS[name]
    print(f"fbp parity {name}: {g.n}^2, {g.n_views} views x {g.n_channels} channels", flush=True)
    sl = ph.make_slice(g, 41, 5e3, low_contrast=True, supersample=1)
    R = recon.Recon(g, 1, 1e-3)
    out = R.fbp(torch.from_numpy(sl.counts).to(dev), sl.i0).cpu().numpy().astype(np.float64)
    ref = oracle.fbp(g, oracle.line_integrals(sl.counts, sl.i0))
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    print(f"  relative L2 {err:.2e}", flush=True)
    assert err <= 1e-5


def test_fbp_is_deterministic_and_reconstructs_the_phantom(dev):
    from paper_1903_10088_amd import recon
    g = ph.config0_geometry()
    sl = ph.make_slice(g, 42, 1e5, supersample=2)
    R = recon.Recon(g, 10, 1e-3)
    counts = torch.from_numpy(sl.counts).to(dev)
    a, b = R.fbp(counts, sl.i0), R.fbp(counts, sl.i0)
    assert torch.equal(a, b)
    # at a high dose the image is the phantom up to the band limit (interior of the body)
    disc = oracle.initial_image(g, 1.0) > 0
    err = np.sqrt(np.mean((a.cpu().numpy() - sl.truth)[disc] ** 2)) / ph.MU_WATER_PER_MM
    assert err < 0.1


def test_fbp_channel_limit(dev):
    from paper_1903_10088_amd import recon
    g = ph.Geometry(n=64, pixel_mm=6.25, n_views=2, n_channels=20000)
    R = recon.Recon(g, 1, 1e-3)
    with pytest.raises(recon.ReconError) as ei:
        R.fbp(torch.ones((2, 20000), device=dev), 1e4)
    assert ei.value.status == recon.RECON_INVALID_ARG
