"""GPU parity of the helical rebinning (recon_rebin_helical) against the FP64 oracle.

Bar: every output element within 1e-6 relative of oracle.rebin_helical on the same float32 counts
and the same float32 I0 (both form the bracket and weight in double precision; the GPU's log and
exp differ from numpy's by ulps of double, which rounding to float32 hides or turns into one float
ulp).  Cases: a small helical scan with Poisson counts (ragged 256-thread tail), a full-size scan
(800 views x 738 channels per turn, 3 turns) on 8 slices, slices at the ends of the valid range, a
z-invariant object whose rebinned counts equal its fan counts, and refusal of unbracketed slices.
"""
import math

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


def run(dev, g, counts, i0, pitch, z0, zs):
    from paper_1903_10088_amd import recon
    out = recon.rebin_helical(g, torch.from_numpy(counts).to(dev), i0, pitch, z0, zs).cpu().numpy()
    ref = oracle.rebin_helical(g, counts, float(np.float32(i0)), pitch, z0, zs)
    err = np.max(np.abs(out.astype(np.float64) / ref - 1))
    print(f"  {len(zs)} slices of {g.n_views} x {g.n_channels}: max relative {err:.2e}", flush=True)
    return out, ref, err


CASES = {
    "small": (ph.Geometry(n=64, pixel_mm=6.25, n_views=36, n_channels=47, start_angle_rad=0.2), 3, 20.0, -30.0, 0.5),
    "full": (ph.config1_geometry(), 3, 10.0, -15.0, 1.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_rebin_matches_oracle(dev, name):
    g, turns, pitch, z0, scale = CASES[name]
    nh = turns * g.n_views
    print(f"rebin parity {name}: {nh} helical views x {g.n_channels} channels, pitch {pitch} mm", flush=True)
    ell = ph.helical_line_integrals(ph.random_helical_phantom(11, scale=scale), g, nh, pitch, z0)
    i0 = 3.7e3
    counts = ph.poisson_counts(ell, i0, 11)
    lo = z0 + pitch * (g.n_views - 1) / g.n_views + 1e-6
    hi = z0 + pitch * (nh - g.n_views) / g.n_views - 1e-6
    zs = list(np.linspace(lo, hi, 8))
    _, _, err = run(dev, g, counts, i0, pitch, z0, zs)
    assert err <= 1e-6


def test_z_invariant_object_rebins_to_its_fan_counts(dev):
    g, turns, pitch, z0 = CASES["small"][0], 3, 20.0, -30.0
    cyl = [ph.Ellipsoid(3.0, -2.0, 0.0, 60.0, 45.0, math.inf, 0.3, ph.MU_WATER_PER_MM)]
    nh = turns * g.n_views
    counts = (1e4 * np.exp(-ph.helical_line_integrals(cyl, g, nh, pitch, z0))).astype(np.float32)
    out, _, _ = run(dev, g, counts, 1e4, pitch, z0, [-7.0, 2.5])
    fan = counts[:g.n_views].astype(np.float64)  # the first turn: the same object at the same angles
    assert np.max(np.abs(out / fan - 1)) <= 1e-6


def test_unbracketed_slice_is_refused(dev):
    from paper_1903_10088_amd import recon
    g = CASES["small"][0]
    counts = torch.ones((3 * g.n_views, g.n_channels), device=dev)
    with pytest.raises(recon.ReconError) as ei:
        recon.rebin_helical(g, counts, 1e4, 20.0, -30.0, [0.0, 50.0])
    assert ei.value.status == recon.RECON_INVALID_ARG


def test_rebinned_slices_reconstruct_like_the_oracle(dev):
    """The chain a helical scan takes: GPU rebinning into three slices, then the batched
    iteration on them, against the oracle's rebinning and iteration of the same slices."""
    from paper_1903_10088_amd import recon
    g = ph.Geometry(n=64, pixel_mm=6.25, n_views=60, n_channels=64)
    turns, pitch, z0, M, n_iter = 3, 12.0, -18.0, 5, 10
    nh = turns * g.n_views
    ell = ph.helical_line_integrals(ph.random_helical_phantom(12, scale=0.8, length_mm=30.0), g, nh, pitch, z0)
    i0 = 4096.0
    counts = ph.poisson_counts(ell, i0, 12)
    zs = [-5.0, 0.0, 5.5]
    print(f"rebin + batch: {len(zs)} slices, {n_iter} sub-iterations", flush=True)
    reb = recon.rebin_helical(g, torch.from_numpy(counts).to(dev), i0, pitch, z0, zs)
    B = recon.Batch([g] * len(zs), M, 1e-3)
    imgs, _ = B.run([reb[s] for s in range(len(zs))], [i0] * len(zs), None, n_iter)
    ref_counts = oracle.rebin_helical(g, counts, i0, pitch, z0, zs)
    disc = oracle.initial_image(g, 1.0) > 0
    for s in range(len(zs)):
        ref, _ = oracle.os_iterate(g, M, 1e-3, ref_counts[s].astype(np.float32), i0, None, n_iter)
        rmse = float(np.sqrt(np.mean((imgs[s].cpu().numpy() - ref)[disc] ** 2)))
        print(f"  slice z = {zs[s]}: rmse {rmse:.2e}", flush=True)
        assert rmse <= 1e-4 * ph.MU_WATER_PER_MM
