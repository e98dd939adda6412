"""Pins of the oracle's helical rebinning (360-degree linear interpolation along z, the textbook
method; the paper reconstructs helical MVCT slices without stating its rebinning).

Exact cases: an object constant along z rebins to its own fan sinogram at every slice; an object
whose line integrals are linear in z rebins to the fan sinogram of its cross-section at the slice
(linear interpolation is exact there, so a swapped weight or a wrong turn shows at once); a slice
at a helical view's own z returns that view.  Brute force: a plain search over the helical views
of each angle for the bracketing pair.  Convergence: on a curved object the error falls with the
square of the pitch.  Slices without helical views on both sides are refused.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1903_10088_amd import phantom as ph

G = ph.Geometry(n=64, pixel_mm=6.25, n_views=36, n_channels=48, start_angle_rad=0.2)
I0 = 1e4
PITCH, Z0, TURNS = 20.0, -30.0, 3
NH = TURNS * G.n_views
Z_OK = [-10.5, -3.3, 0.0, 4.72, 9.9]  # inside [z0 + pitch (nv-1)/nv, z0 + pitch (nh-nv)/nv)


def section_sinogram(ellipsoids, z):
    return ph.analytic_sinogram([e for e in (q.section(z) for q in ellipsoids) if e is not None], G)


def noise_free(ellipsoids, pitch=PITCH):
    return I0 * np.exp(-ph.helical_line_integrals(ellipsoids, G, NH, pitch, Z0))


def test_z_invariant_object_rebins_to_its_fan_sinogram():
    cyl = [ph.Ellipsoid(3.0, -2.0, 0.0, 150.0 * 0.4, 110.0 * 0.4, math.inf, 0.3, ph.MU_WATER_PER_MM),
           ph.Ellipsoid(20.0, 5.0, 0.0, 12.0, 7.0, math.inf, 1.1, 0.002)]
    out = oracle.rebin_helical(G, noise_free(cyl), I0, PITCH, Z0, Z_OK)
    ref = I0 * np.exp(-section_sinogram(cyl, 0.0))
    for s in range(len(Z_OK)):
        assert np.max(np.abs(out[s] / ref - 1)) < 1e-12


def test_linear_in_z_object_rebins_exactly():
    obj = [ph.Ellipsoid(0.0, 0.0, 0.0, 55.0, 45.0, math.inf, 0.0, ph.MU_WATER_PER_MM, 2e-5),
           ph.Ellipsoid(-15.0, 10.0, 4.0, 10.0, 14.0, math.inf, 0.7, 0.001, -3e-5)]
    out = oracle.rebin_helical(G, noise_free(obj), I0, PITCH, Z0, Z_OK)
    for s, z in enumerate(Z_OK):
        ell = np.log(I0 / out[s])
        assert np.max(np.abs(ell - section_sinogram(obj, z))) < 1e-11


def test_slice_at_a_view_returns_that_view():
    rng = np.random.default_rng(3)
    counts = rng.uniform(50, 5000, (NH, G.n_channels))
    m = 1
    z = Z0 + PITCH * m  # helical view m * nv (view angle 0 of turn m)
    out = oracle.rebin_helical(G, counts, I0, PITCH, Z0, [z])
    assert np.max(np.abs(out[0, 0] / counts[m * G.n_views] - 1)) < 1e-12


def test_matches_a_brute_force_search():
    rng = np.random.default_rng(4)
    counts = rng.uniform(0.0, 8000, (NH, G.n_channels))  # includes y < 1 (guarded)
    zh = ph.helical_view_z(G, NH, PITCH, Z0)
    out = oracle.rebin_helical(G, counts, I0, PITCH, Z0, Z_OK)
    ell = np.log(I0 / np.maximum(counts, 1.0))
    for s, z in enumerate(Z_OK):
        for v in range(G.n_views):
            same = [h for h in range(NH) if h % G.n_views == v]
            lower = max(h for h in same if zh[h] <= z)
            upper = min(h for h in same if zh[h] > z)
            w = (z - zh[lower]) / (zh[upper] - zh[lower])
            ref = I0 * np.exp(-((1 - w) * ell[lower] + w * ell[upper]))
            np.testing.assert_allclose(out[s, v], ref, rtol=1e-12)


def test_error_falls_with_the_square_of_the_pitch():
    # long in z against the pitch, so its line integrals are smooth in z (the RMS over the rays;
    # rays grazing a cross-section's edge vary like a square root and would dominate a maximum)
    ball = [ph.Ellipsoid(0.0, 0.0, 0.0, 60.0, 50.0, 200.0, 0.4, ph.MU_WATER_PER_MM)]
    errs = []
    for pitch in (16.0, 8.0):
        z0 = -pitch * 1.5
        counts = I0 * np.exp(-ph.helical_line_integrals(ball, G, NH, pitch, z0))
        out = oracle.rebin_helical(G, counts, I0, pitch, z0, [0.3 * pitch])
        d = np.log(I0 / out[0]) - section_sinogram(ball, 0.3 * pitch)
        errs.append(np.sqrt(np.mean(d * d)))
    assert 3.5 < errs[0] / errs[1] < 4.8


def test_unbracketed_slices_are_refused():
    counts = np.full((NH, G.n_channels), 100.0)
    lo = Z0 + PITCH * (G.n_views - 1) / G.n_views
    hi = Z0 + PITCH * (NH - G.n_views) / G.n_views  # exclusive
    oracle.rebin_helical(G, counts, I0, PITCH, Z0, [lo + 1e-9, hi - 1e-9])
    for z in (lo - 1e-6, hi + 1e-6, Z0 - 50.0):
        with pytest.raises(ValueError):
            oracle.rebin_helical(G, counts, I0, PITCH, Z0, [z])
