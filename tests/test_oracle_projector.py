"""Pins of the oracle's fan-beam Joseph projector and its transpose.

Each test checks the oracle against something other than itself: a closed form
for axis-aligned rays, the exact line integrals of ellipses computed by the
separate input generator, symmetries of the geometry, the adjoint identity and
a dense brute-force transpose.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1903_10088_amd import phantom as ph


def small_geom(n=8, nv=4, nc=5, px=1.0, sad=100.0):
    return ph.Geometry(n=n, pixel_mm=px, n_views=nv, n_channels=nc, sad_mm=sad, sdd_mm=2 * sad)


def test_axis_aligned_closed_form():
    """Central ray (odd channel count) of view 0 runs along y = 0: for even N it samples halfway
    between rows N/2-1 and N/2 with weight 1/2 each and unit path length per column; view N_v/4
    runs along x = 0 and does the same over columns."""
    g = small_geom()
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 1, (8, 8))
    sino = oracle.project(g, img)
    k = 2  # (n_ch - 1) / 2
    expect_v0 = g.pixel_mm * np.sum(0.5 * img[3, :] + 0.5 * img[4, :])
    expect_v1 = g.pixel_mm * np.sum(0.5 * img[:, 3] + 0.5 * img[:, 4])
    assert sino[0, k] == pytest.approx(expect_v0, rel=1e-12)
    assert sino[1, k] == pytest.approx(expect_v1, rel=1e-12)
    # the opposite views see the same lines
    assert sino[2, k] == pytest.approx(expect_v0, rel=1e-12)
    assert sino[3, k] == pytest.approx(expect_v1, rel=1e-12)


def test_unit_image_path_length_scale():
    """A uniform image of 1/mm inside a wide square: the central ray of view 0 crosses N columns of
    width pixel_mm, so its line integral is N * pixel_mm (pins the per-column length)."""
    g = small_geom(n=16, px=2.5)
    img = np.ones((16, 16))
    sino = oracle.project(g, img)
    assert sino[0, 2] == pytest.approx(16 * 2.5, rel=1e-12)


def test_analytic_ellipses_config0():
    """Joseph projection of the supersampled ellipse phantom agrees with the exact chord integrals
    within 2% (relative L2) at the 128^2 configuration; this fixes orientation, angle origin,
    channel order and length scale."""
    g = ph.config0_geometry()
    sl = ph.make_slice(g, 0, 1e4)
    A = oracle.project(g, sl.truth)
    rel = np.linalg.norm(A - sl.line_integrals) / np.linalg.norm(sl.line_integrals)
    assert rel < 0.02
    # a wrong channel order or a mirrored geometry is far off
    rel_flip = np.linalg.norm(A[:, ::-1] - sl.line_integrals) / np.linalg.norm(sl.line_integrals)
    assert rel_flip > 5 * rel


def test_analytic_error_shrinks_with_resolution():
    """Discretisation error falls as the pixel shrinks at fixed FOV (about first order)."""
    errs = []
    for n in (64, 128, 256):
        g = ph.Geometry(n=n, pixel_mm=400.0 / n, n_views=90, n_channels=3 * n // 2)
        sl = ph.make_slice(g, 5, 1e4)
        A = oracle.project(g, sl.truth)
        errs.append(np.linalg.norm(A - sl.line_integrals) / np.linalg.norm(sl.line_integrals))
    assert errs[0] > 1.5 * errs[1] > 1.5 * 1.5 * errs[2] * 0.99


def test_rotation_by_quarter_turn():
    """Rotating the image by a quarter turn shifts the sinogram by N_v/4 views."""
    g = ph.config0_geometry()
    rng = np.random.default_rng(11)
    img = rng.uniform(0, 0.01, (g.n, g.n))
    p0 = oracle.project(g, img)
    p1 = oracle.project(g, np.rot90(img))
    shift = g.n_views // 4
    expect = np.roll(p0, -shift, axis=0)
    assert np.max(np.abs(p1 - expect)) <= 1e-10 * np.max(np.abs(p0))


def test_vertical_flip():
    """Mirroring y -> -y maps view v to -v and channel k to n_ch-1-k."""
    g = ph.config0_geometry()
    rng = np.random.default_rng(12)
    img = rng.uniform(0, 0.01, (g.n, g.n))
    p0 = oracle.project(g, img)
    p1 = oracle.project(g, np.flipud(img))
    v = (-np.arange(g.n_views)) % g.n_views
    expect = p0[v][:, ::-1]
    assert np.max(np.abs(p1 - expect)) <= 1e-10 * np.max(np.abs(p0))


@pytest.mark.parametrize("geom", ["config0", "n32"])
def test_adjoint_identity(geom):
    """<A x, y> = <x, A^T y> to 1e-12 relative."""
    if geom == "config0":
        g = ph.config0_geometry()
    else:
        g = ph.Geometry(n=32, pixel_mm=12.5, n_views=40, n_channels=48)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((g.n, g.n))
    y = rng.standard_normal((g.n_views, g.n_channels))
    lhs = np.sum(oracle.project(g, x) * y)
    rhs = np.sum(x * oracle.backproject(g, y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    views = oracle.subset_views(g.n_views, 10, 3)
    ys = rng.standard_normal((len(views), g.n_channels))
    lhs = np.sum(oracle.project(g, x, views) * ys)
    rhs = np.sum(x * oracle.backproject(g, ys, views))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_dense_transpose_brute_force():
    """On an 8x8 image the backprojector equals the transpose of the dense projection matrix."""
    g = ph.Geometry(n=8, pixel_mm=25.0, n_views=12, n_channels=10)
    npix, nray = 64, 120
    A = np.zeros((nray, npix))
    for r in range(npix):
        e = np.zeros(npix)
        e[r] = 1.0
        A[:, r] = oracle.project(g, e.reshape(8, 8)).ravel()
    B = np.zeros((npix, nray))
    for q in range(nray):
        e = np.zeros(nray)
        e[q] = 1.0
        B[:, q] = oracle.backproject(g, e.reshape(12, 10)).ravel()
    assert np.max(np.abs(B - A.T)) <= 1e-14 * np.max(np.abs(A))
    # every ray crosses the image with non-negative weights
    assert A.min() >= 0
    nnz = int(np.count_nonzero(A))
    pairs = oracle.count_pairs(g)
    assert nnz <= pairs <= nnz + nray  # zero weights only where a sample falls exactly on a row


def test_major_axis_split():
    """Each view's rays switch major axis at most once (fan narrower than 90 degrees), central rays
    at 0 and 90 degrees are x- and y-major, and about half of all rays are x-major."""
    g = ph.config1_geometry()
    m = oracle.ray_major(g)
    flips = np.abs(np.diff(m, axis=1)).sum(axis=1)
    assert flips.max() <= 1
    c = (g.n_channels - 1) // 2
    assert m[0, c] == 0 and m[g.n_views // 4, c] == 1
    assert 0.45 < (m == 0).mean() < 0.55


# ---------------------------------------------------------------------------
# Limited-angle data (section 4, reconstructed images: fewer projection data)
# ---------------------------------------------------------------------------

def test_partial_arc_is_the_first_views_of_a_full_turn():
    """K views over an arc of 2 pi K / N sit at the angles of the first K views of a full turn of N
    views: the sinogram equals those rows, and the same arc started N/3 steps later equals rows
    N/3 .. N/3 + K - 1 (a wrong step, arc / (K - 1) or 2 pi / K, moves every view but the first)."""
    n_full, k = 60, 23
    full = ph.Geometry(n=32, pixel_mm=6.25, n_views=n_full, n_channels=41)
    rng = np.random.default_rng(11)
    img = rng.uniform(0, 0.01, (32, 32))
    sino_full = oracle.project(full, img)
    arc = 2 * math.pi * k / n_full
    part = ph.Geometry(n=32, pixel_mm=6.25, n_views=k, n_channels=41, scan_arc_rad=arc)
    sino = oracle.project(part, img)
    np.testing.assert_allclose(sino, sino_full[:k], rtol=1e-12, atol=1e-15)
    s0 = n_full // 3
    later = ph.Geometry(n=32, pixel_mm=6.25, n_views=k, n_channels=41, scan_arc_rad=arc,
                        start_angle_rad=2 * math.pi * s0 / n_full)
    np.testing.assert_allclose(oracle.project(later, img), sino_full[s0:s0 + k], rtol=1e-12, atol=1e-15)
    # the arc is honoured: a full turn of K views differs from every row but the first
    other = oracle.project(ph.Geometry(n=32, pixel_mm=6.25, n_views=k, n_channels=41), img)
    assert np.allclose(other[0], sino[0], rtol=1e-12)
    assert all(not np.allclose(other[v], sino[v], rtol=1e-6) for v in range(1, k))


def test_partial_arc_matches_analytic_ellipses():
    """A short scan (half a turn plus the fan) of the config-0 phantom: the Joseph projection of
    the rasterised phantom agrees with the generator's exact chord integrals of the same arc
    within the full-turn bar, and the transpose stays exact (adjoint identity)."""
    g0 = ph.config0_geometry()
    arc = math.pi + 2 * g0.gamma_max
    g = ph.Geometry(n=g0.n, pixel_mm=g0.pixel_mm, n_views=100, n_channels=g0.n_channels, scan_arc_rad=arc)
    sl = ph.make_slice(g, 0, 1e4)
    A = oracle.project(g, sl.truth)
    rel = np.linalg.norm(A - sl.line_integrals) / np.linalg.norm(sl.line_integrals)
    assert rel < 0.02
    rng = np.random.default_rng(5)
    x = rng.standard_normal((g.n, g.n))
    y = rng.standard_normal((g.n_views, g.n_channels))
    lhs = float(np.sum(oracle.project(g, x) * y))
    rhs = float(np.sum(x * oracle.backproject(g, y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_partial_arc_bounds_and_fbp_refusal():
    """Arcs outside (0, 2 pi] are refused; the filtered backprojection takes full turns only (a
    partial arc would need redundancy weights, which are not stated)."""
    img = np.zeros((16, 16))
    for bad in (-0.5, 2 * math.pi + 1e-3):
        with pytest.raises(RuntimeError):
            oracle.project(ph.Geometry(n=16, pixel_mm=5.0, n_views=8, n_channels=9, scan_arc_rad=bad), img)
    g = ph.Geometry(n=16, pixel_mm=5.0, n_views=8, n_channels=9, scan_arc_rad=math.pi)
    with pytest.raises(RuntimeError):
        oracle.fbp(g, np.zeros((8, 9)))
    # exactly 2 pi is a full turn, bit for bit
    full = ph.Geometry(n=16, pixel_mm=5.0, n_views=8, n_channels=9)
    img = np.random.default_rng(2).uniform(0, 0.01, (16, 16))
    two_pi = ph.Geometry(n=16, pixel_mm=5.0, n_views=8, n_channels=9, scan_arc_rad=2 * math.pi)
    assert np.array_equal(oracle.project(two_pi, img), oracle.project(full, img))
