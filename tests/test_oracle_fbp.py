"""Pins of the oracle's fan-beam filtered backprojection (the baseline the paper compares with;
the algorithm is the textbook equiangular one, which the paper does not spell out).

Analytic line integrals of ellipse phantoms (closed-form chords, from the phantom module) must
come back as the phantom: a uniform disc to its value in the interior, an off-centre rotated
ellipse with an insert at its place and orientation; a quarter turn of the object (a shift of the
sinogram by N_v/4 views, the projector's pinned convention) must turn the image by a quarter turn,
which a mirrored fan angle or a wrong view angle would break; and the filter's scale is fixed by the
disc's value (a missing factor of 2, D or dbeta shows at once).
"""
import math

import numpy as np

import oracle
from paper_1903_10088_amd import phantom as ph

G = ph.Geometry(n=128, pixel_mm=3.125, n_views=360, n_channels=384)


def radius_map(g):
    c = 0.5 * (g.n - 1)
    x = (np.arange(g.n) - c) * g.pixel_mm
    X, Y = np.meshgrid(x, x, indexing="xy")
    return X, Y, np.hypot(X, Y)


def test_uniform_disc_comes_back_at_its_value():
    mu = 0.02
    disc = [ph.Ellipse(0.0, 0.0, 100.0, 100.0, 0.0, mu)]
    img = oracle.fbp(G, ph.analytic_sinogram(disc, G))
    _, _, r = radius_map(G)
    inner = img[r < 85.0]
    assert abs(inner.mean() / mu - 1) < 0.005
    assert inner.std() / mu < 0.01
    ring = img[(r > 115.0) & (r < 190.0)]
    assert np.abs(ring).mean() / mu < 0.02


def test_off_centre_ellipse_at_its_place_and_orientation():
    ells = [ph.Ellipse(30.0, -20.0, 120.0, 60.0, 0.5, 0.015), ph.Ellipse(60.0, -10.0, 20.0, 10.0, 1.2, 0.01)]
    img = oracle.fbp(G, ph.analytic_sinogram(ells, G))
    truth = ph.rasterize(ells, G.n, G.pixel_mm, supersample=4)
    # away from the edges (where pixel averages and the band-limited reconstruction differ)
    X, Y, r = radius_map(G)
    edge = np.zeros_like(truth, dtype=bool)
    for e in ells:
        for d in (-2.0, 2.0):
            grown = ph.Ellipse(e.cx, e.cy, e.a + d * G.pixel_mm, e.b + d * G.pixel_mm, e.phi, 1.0)
            edge ^= ph.rasterize([grown], G.n, G.pixel_mm, supersample=1) > 0
    keep = (r < 190.0) & ~edge
    err = np.sqrt(np.mean((img - truth)[keep] ** 2)) / 0.015
    assert err < 0.02
    # the mirrored or rotated placement is far off
    assert np.sqrt(np.mean((img[::-1, :] - truth)[keep] ** 2)) / 0.015 > 0.3


def test_quarter_turn():
    rng = np.random.default_rng(5)
    s = rng.uniform(0.0, 1.0, (G.n_views, G.n_channels))
    a = oracle.fbp(G, np.roll(s, -G.n_views // 4, axis=0))
    b = np.rot90(oracle.fbp(G, s))
    assert np.max(np.abs(a - b)) <= 1e-9 * np.max(np.abs(b))


def test_filter_kernel_has_no_dc():
    """A constant sinogram row filters to ~zero in the interior channels (the ramp has no DC), so
    a constant offset of all line integrals barely moves the interior of the image."""
    mu = 0.02
    disc = [ph.Ellipse(0.0, 0.0, 100.0, 100.0, 0.0, mu)]
    s = ph.analytic_sinogram(disc, G)
    img0 = oracle.fbp(G, s)
    img1 = oracle.fbp(G, s + 0.1)  # 0.1 is five times the disc's peak line integral
    _, _, r = radius_map(G)
    assert np.abs(img1 - img0)[r < 150.0].max() / mu < 0.2
    assert math.isfinite(float(img1.sum()))
