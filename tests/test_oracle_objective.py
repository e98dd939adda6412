"""Pins of the oracle's TV prior, likelihood, step rule and ordered-subset iteration.

Pins come from mathematics: finite differences, closed forms for a step edge,
the textbook Poisson log-pmf, the descent lemma for projected gradient steps,
noise-free data, and the constants the paper prints (tests/golden).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1903_10088_amd import phantom as ph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


# ----------------------------------------------------------------------------- TV

def test_tv_constant_image_has_zero_gradient():
    val, g = oracle.tv(np.full((12, 12), 0.05), eps=1e-3)
    assert np.all(g == 0.0)
    assert val == pytest.approx(144 * 1e-3, rel=1e-14)


def test_tv_step_edge_closed_form():
    """Vertical step from a to b between columns m-1 and m: only those two columns get a gradient,
    +-(b-a)/sqrt((b-a)^2+eps^2), and TV = N*sqrt((b-a)^2+eps^2) + (N^2-N)*eps."""
    n, m, a, b, eps = 10, 4, 0.02, 0.05, 1e-3
    img = np.full((n, n), a)
    img[:, m:] = b
    val, g = oracle.tv(img, eps)
    phi = math.sqrt((b - a) ** 2 + eps**2)
    expect = np.zeros((n, n))
    expect[:, m - 1] = (b - a) / phi
    expect[:, m] = -(b - a) / phi
    assert np.max(np.abs(g - expect)) < 1e-14
    assert val == pytest.approx(n * phi + (n * n - n) * eps, rel=1e-14)


def test_tv_gradient_matches_finite_differences():
    """Central differences of TV along random directions and at single pixels (corners, edges,
    interior) agree with -g_R to 1e-8 relative."""
    rng = np.random.default_rng(4)
    n, eps = 16, 2e-3
    img = 0.05 + 0.01 * rng.standard_normal((n, n))
    _, g = oracle.tv(img, eps)
    h = 1e-5

    def fd5(d):  # fourth-order central difference
        f = [oracle.tv(img + s * h * d, eps)[0] for s in (-2, -1, 1, 2)]
        return (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)

    for _ in range(4):
        d = rng.standard_normal((n, n))
        an = -np.sum(g * d)
        assert abs(fd5(d) - an) <= 1e-8 * abs(an)
    for (j, i) in [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1), (0, 5), (7, 0), (n - 1, 6), (5, n - 1), (8, 9)]:
        e = np.zeros((n, n))
        e[j, i] = 1
        assert fd5(e) == pytest.approx(-g[j, i], rel=1e-8, abs=1e-9)


# ----------------------------------------------------------------------------- likelihood

def test_loglik_is_poisson_logpmf_up_to_constants():
    """I0 * L + sum(y ln I0 - ln y!) equals the Poisson log-pmf of counts with mean I0 exp(-l)."""
    rng = np.random.default_rng(5)
    i0 = 2000.0
    ell = rng.uniform(0.0, 2.0, 500)
    y = rng.poisson(i0 * np.exp(-ell)).astype(np.float64)
    L = oracle.loglik(ell, y / i0)
    const = np.sum(y * math.log(i0) - np.array([math.lgamma(v + 1) for v in y]))
    ref = np.sum(stats.poisson.logpmf(y, i0 * np.exp(-ell)))
    assert i0 * L + const == pytest.approx(ref, rel=1e-12)


def _geom16():
    return ph.Geometry(n=16, pixel_mm=25.0, n_views=24, n_channels=24)


def _phi(g, mu_mm, counts, i0, beta, eps_mm):
    """Objective -L + beta*TV in the paper's units (cm, 1/cm)."""
    ell = oracle.project(g, mu_mm)  # dimensionless
    L = oracle.loglik(ell, counts / i0)
    tvv, _ = oracle.tv(10 * mu_mm, 10 * eps_mm)
    return -L + beta * tvv


def test_iteration_step_is_likelihood_gradient():
    """One sub-iteration with beta=0, M=1 and a given lambda moves the image (inside the mask, away
    from the clamp) by lambda * dL/dmu, with dL/dmu in cm units checked by central differences
    of the likelihood."""
    g = _geom16()
    sl = ph.make_slice(g, 3, 5e3)
    i0 = 5e3
    mu0 = oracle.initial_image(g, 0.005)
    lam = 1e-3
    mu1, _ = oracle.os_iterate(g, 1, 0.0, sl.counts, i0, mu0, 1, lambda_schedule=[lam])
    mask = mu0 > 0
    step_cm = 10 * (mu1 - mu0) / lam  # dL/dmu_cm inside the mask
    rng = np.random.default_rng(6)
    h = 1e-7
    for _ in range(3):
        d = rng.standard_normal(mu0.shape) * mask  # direction in 1/cm
        Lp = oracle.loglik(oracle.project(g, mu0 + h * d / 10), sl.counts / i0)
        Lm = oracle.loglik(oracle.project(g, mu0 - h * d / 10), sl.counts / i0)
        fd = (Lp - Lm) / (2 * h)
        an = np.sum(step_cm * d)
        assert fd == pytest.approx(an, rel=1e-6)


def test_consistent_data_is_a_fixed_point():
    """If y/I0 = exp(-A mu) exactly and beta = 0 the gradient vanishes and mu does not move."""
    g = _geom16()
    sl = ph.make_slice(g, 4, 1e4)
    mu = np.where(oracle.initial_image(g, 1.0) > 0, sl.truth + 0.001, 0.0)
    i0 = 1e4
    counts = i0 * np.exp(-oracle.project(g, mu))
    mu1, _ = oracle.os_iterate(g, 4, 0.0, counts, i0, mu, 4, lambda_schedule=[0.01] * 4)
    assert np.max(np.abs(mu1 - mu)) <= 1e-14


def test_monotone_objective_decrease():
    """M = 1 with constant lambda = 1/(|A|^2 + 8 beta/eps) (cm units): projected gradient descent with
    a step below the inverse Lipschitz constant decreases -L + beta*TV at every step."""
    g = _geom16()
    sl = ph.make_slice(g, 7, 3e3)
    i0, beta, eps_mm = 3e3, 1e-3, 1e-4
    # |A_cm|^2 by power iteration (A_cm = A_mm / 10)
    rng = np.random.default_rng(8)
    x = rng.uniform(size=(16, 16))
    for _ in range(60):
        x = oracle.backproject(g, oracle.project(g, x))
        nrm = np.linalg.norm(x)
        x /= nrm
    a2_cm = nrm / 100.0
    lam = 1.0 / (a2_cm * 1.01 + 8 * beta / (10 * eps_mm))
    params = dict(tv_eps_per_mm=eps_mm)
    mu = oracle.initial_image(g, 0.005)
    phis = [_phi(g, mu, sl.counts, i0, beta, eps_mm)]
    for _ in range(25):
        mu, _ = oracle.os_iterate(g, 1, beta, sl.counts, i0, mu, 1, lambda_schedule=[lam], params=params)
        phis.append(_phi(g, mu, sl.counts, i0, beta, eps_mm))
    d = np.diff(phis)
    assert np.all(d < 0), d


def test_noise_free_residual_goes_to_zero():
    """Noise-free data from the discrete model and beta = 0: the squared difference falls by
    orders of magnitude."""
    g = ph.Geometry(n=24, pixel_mm=400 / 24, n_views=48, n_channels=36)
    sl = ph.make_slice(g, 9, 1e4)
    mu_true = np.where(oracle.initial_image(g, 1.0) > 0, sl.truth, 0.0)
    i0 = 1e4
    counts = i0 * np.exp(-oracle.project(g, mu_true))
    _, tr = oracle.os_iterate(g, 4, 0.0, counts, i0, None, 400)
    assert tr[-1, 0] < 1e-4 * tr[0, 0]


# ----------------------------------------------------------------------------- step rule

def test_paper_constants_are_the_defaults():
    gold = json.load(open(GOLDEN))
    assert oracle.DEFAULT_PARAMS["lambda0"] == gold["lambda0"]["value"]
    assert oracle.DEFAULT_PARAMS["lambda_inc"] == gold["lambda_inc"]["value"]
    assert oracle.DEFAULT_PARAMS["lambda_dec"] == gold["lambda_dec"]["value"]
    assert oracle.DEFAULT_PARAMS["mu0_per_mm"] * 10 == pytest.approx(gold["mu0_per_cm_best"]["value"])


def test_lambda_rule_scripted():
    """Eqs. 4-5 on a scripted sequence: start 0.01; decrease +1e-4; tie or increase -2e-4; floor."""
    lam = oracle.lambda_next(True, 0.0, 5.0, 0.0)
    assert lam == 0.01
    seq = [(4.0, 5.0, 0.0101), (3.0, 4.0, 0.0102), (3.0, 3.0, 0.0100), (3.5, 3.0, 0.0098)]
    for f_n, f_prev, expect in seq:
        lam = oracle.lambda_next(False, lam, f_n, f_prev)
        assert lam == pytest.approx(expect, abs=1e-15)
    assert oracle.lambda_next(False, 2e-4, 2.0, 1.0) == pytest.approx(1e-4)
    assert oracle.lambda_next(False, 1e-4, 2.0, 1.0) == pytest.approx(1e-4)


def test_iteration_lambda_trace_follows_rule():
    g = ph.config0_geometry()
    sl = ph.make_slice(g, 1, 1e4)
    _, tr = oracle.os_iterate(g, 10, 1e-3, sl.counts, 1e4, None, 30)
    assert tr[0, 1] == 0.01
    for n in range(1, 30):
        dl = tr[n, 1] - tr[n - 1, 1]
        if tr[n, 0] < tr[n - 1, 0]:
            assert dl == pytest.approx(1e-4, abs=1e-14)
        else:
            assert dl == pytest.approx(-2e-4, abs=1e-14) or tr[n, 1] == pytest.approx(1e-4)


def test_subsets_are_interleaved_views():
    """f_n is the mean squared difference over the views v = s (mod M) of subset s = n mod M."""
    g = ph.config0_geometry()
    sl = ph.make_slice(g, 2, 1e4)
    M, i0 = 10, 1e4
    mu0 = oracle.initial_image(g, 0.005)
    st = oracle.State()
    st._s.n_done = 3
    st._s.lambda_ = 0.01
    _, tr = oracle.os_iterate(g, M, 1e-3, sl.counts, i0, mu0, 1, state=st)
    views = np.arange(3, g.n_views, M)
    ell = oracle.project(g, mu0, views)
    p = np.log(i0 / np.maximum(sl.counts[views].astype(np.float64), 1.0))
    assert tr[0, 0] == pytest.approx(np.mean((ell - p) ** 2), rel=1e-12)
    assert st.n_done == 4


def test_resume_equals_uninterrupted():
    g = ph.config0_geometry()
    sl = ph.make_slice(g, 6, 1e4)
    a, ta = oracle.os_iterate(g, 10, 1e-3, sl.counts, 1e4, None, 20)
    st = oracle.State()
    b, tb1 = oracle.os_iterate(g, 10, 1e-3, sl.counts, 1e4, None, 12, state=st)
    b, tb2 = oracle.os_iterate(g, 10, 1e-3, sl.counts, 1e4, b, 8, state=st)
    # the image crosses the 1/mm <-> 1/cm conversion once more, so allow a few ulps
    assert np.allclose(a, b, rtol=1e-12, atol=1e-16)
    tb = np.vstack([tb1, tb2])
    assert np.array_equal(ta[:, 1], tb[:, 1])
    assert np.allclose(ta[:, 0], tb[:, 0], rtol=1e-12, atol=0)


def test_step_limit_reading():
    """The reading of the likelihood normalisation (divide by I0, cm units) makes the paper's
    lambda_0 = 0.01 a stable but not tiny step on a config-0 subset: below 2 / |A_s^T T A_s|,
    the inverse curvature of -L_s at the phantom (T = diag(exp(-l))), and above a tenth of it."""
    g = ph.config0_geometry()
    sl = ph.make_slice(g, 0, 1e4)
    views = oracle.subset_views(g.n_views, 10, 0)
    t = np.exp(-sl.line_integrals[views])
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(g.n, g.n))
    for _ in range(40):
        x = oracle.backproject(g, t * oracle.project(g, x, views), views)
        nrm = np.linalg.norm(x)
        x /= nrm
    h_cm = nrm / 100.0  # A_cm = A_mm / 10
    assert 0.1 * 2.0 / h_cm < 0.01 < 2.0 / h_cm


# ----------------------------------------------------------------------------- prior weight and support

def _subset_loglik(g, mu_mm, counts, i0, views):
    """L_s of section 2 restricted to the rays of the listed views (blank-scan normalised)."""
    return oracle.loglik(oracle.project(g, mu_mm, views), counts[views] / i0)


def _one_step(g, M, beta, counts, i0, mu0, n_done, lam, eps_mm):
    st = oracle.State()
    st._s.n_done = n_done
    st._s.lambda_ = 0.01
    mu1, _ = oracle.os_iterate(g, M, beta, counts, i0, mu0, 1, state=st, lambda_schedule=[lam],
                               params=dict(tv_eps_per_mm=eps_mm))
    return mu1


def test_step_with_subsets_uses_thinned_prior_weight():
    """Section 3.D: in ordered-subset mode the TV weight is multiplied by the thinning factor 1/M.
    One sub-iteration with M = 4, beta > 0 and a given lambda, started at sub-iteration 5 (subset
    s = 1), from a textured positive image: inside the disc (no pixel reaches the clamp) the
    image moves by lambda * (dL_s/dmu + (beta/M) g_R) in cm units.  Both gradients come from
    central differences outside the iteration: L_s of subset 1's views only, and TV of the image
    in 1/cm.  The prior's share alone (the beta run minus the beta = 0 run) is checked against
    -(beta/M) dTV/dmu on its own, so a weight of beta (or beta/M^2) fails by a factor M."""
    g = _geom16()
    sl = ph.make_slice(g, 11, 5e3)
    i0, M, beta, eps_mm, lam, n_done = 5e3, 4, 2e-2, 1e-4, 2e-4, 5
    rng = np.random.default_rng(12)
    disc = oracle.initial_image(g, 1.0) > 0
    mu0 = np.where(disc, 0.005 * (1.0 + 0.2 * rng.uniform(-1, 1, (g.n, g.n))), 0.0)
    views = oracle.subset_views(g.n_views, M, n_done % M)

    mu_b = _one_step(g, M, beta, sl.counts, i0, mu0, n_done, lam, eps_mm)
    mu_0 = _one_step(g, M, 0.0, sl.counts, i0, mu0, n_done, lam, eps_mm)
    assert np.all(mu_b[disc] > 0) and np.all(mu_0[disc] > 0)  # away from the clamp
    step_b = 10 * (mu_b - mu0) / lam  # per 1/cm of image, as Eq. 3 is written
    step_prior = 10 * (mu_b - mu_0) / lam

    h = 1e-6
    for _ in range(4):
        d = rng.standard_normal((g.n, g.n)) * disc  # direction in 1/cm
        fd_l = (_subset_loglik(g, mu0 + h * d / 10, sl.counts, i0, views)
                - _subset_loglik(g, mu0 - h * d / 10, sl.counts, i0, views)) / (2 * h)
        tv_p = oracle.tv(10 * mu0 + h * d, 10 * eps_mm)[0]
        tv_m = oracle.tv(10 * mu0 - h * d, 10 * eps_mm)[0]
        fd_r = -(tv_p - tv_m) / (2 * h)  # directional derivative of R = -TV
        full = fd_l + (beta / M) * fd_r
        assert np.sum(step_b * d) == pytest.approx(full, rel=1e-6)
        assert np.sum(step_prior * d) == pytest.approx((beta / M) * fd_r, rel=1e-5)
        # the prior's share is far above the 1e-6 tolerance: a weight off by M would show in both
        assert abs((beta / M) * fd_r) > 1e-4 * abs(full)


def _integer_disc(n):
    """Pixel centres inside the reconstruction circle of radius N*pixel/2, decided in integers:
    with centre offsets (i - (N-1)/2, j - (N-1)/2) in pixels, the test doubled is
    (2i - N + 1)^2 + (2j - N + 1)^2 <= N^2 (no centre lies exactly on the circle: the two
    squares are both even for odd N and both odd for even N, while N^2 is odd or 0 mod 4)."""
    a = 2 * np.arange(n, dtype=np.int64) - n + 1
    return a[None, :] ** 2 + a[:, None] ** 2 <= n * n


def _integer_disc_count(n):
    """Number of pixel centres in the circle, counted row by row with integer square roots."""
    import math as _m
    total = 0
    for j in range(n):
        b = 2 * j - n + 1
        rem = n * n - b * b
        if rem < 0:
            continue
        r = _m.isqrt(rem)  # largest |a| with a^2 <= rem
        # a = 2i - n + 1 runs over values of the parity of n - 1 in [-(n-1), n-1]
        lo = -min(r, n - 1)
        hi = min(r, n - 1)
        par = (n - 1) % 2
        if (lo - par) % 2:
            lo += 1
        if (hi - par) % 2:
            hi -= 1
        if hi >= lo:
            total += (hi - lo) // 2 + 1
    return total


@pytest.mark.parametrize("n,px", [(5, 25.0), (16, 25.0), (17, 400 / 17), (128, 3.125), (200, 2.0), (512, 0.78125)])
def test_initial_image_support_is_the_reconstruction_disc(n, px):
    """Section 3.C.2: the homogeneous start image fills the reconstruction circle x^2 + y^2 <=
    (N*pixel/2)^2 and is zero outside; the pixel set equals the integer-arithmetic disc and its
    size equals an independent row-by-row isqrt count.  A radius of (N-1)*pixel/2 drops
    a ring of boundary pixels and fails."""
    g = ph.Geometry(n=n, pixel_mm=px, n_views=8, n_channels=8)
    img = oracle.initial_image(g, 0.005)
    disc = _integer_disc(n)
    assert np.array_equal(img > 0, disc)
    assert np.all(img[disc] == 0.005) and np.all(img[~disc] == 0.0)
    assert int(disc.sum()) == _integer_disc_count(n)


def test_iteration_holds_the_image_at_zero_outside_the_disc():
    """The iterate is zero outside the reconstruction circle and the start image is taken as zero
    there too: a start image positive everywhere (corners included) gives, after one small step,
    exactly zero on the pixels outside the integer-arithmetic disc and positive values inside."""
    g = ph.Geometry(n=17, pixel_mm=400 / 17, n_views=24, n_channels=24)
    sl = ph.make_slice(g, 13, 5e3)
    mu0 = np.full((g.n, g.n), 0.005)
    mu1, _ = oracle.os_iterate(g, 3, 1e-3, sl.counts, 5e3, mu0, 1, lambda_schedule=[1e-4])
    disc = _integer_disc(g.n)
    assert np.all(mu1[~disc] == 0.0)
    assert np.all(mu1[disc] > 0.0)
