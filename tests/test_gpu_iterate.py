"""GPU parity of the full ordered-subset iteration against the FP64 oracle.

Bar: image RMSE over the reconstruction disc <= 1e-4 * mu_water (4.9e-7 / mm)
after the full iteration count, the GPU taking its own step-rule decisions, and
the lambda traces equal to the oracle's, decision for decision (a differing
decision fails the test and names the first differing sub-iteration and the
oracle's margin there).
"""
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


def run_both(dev, g, M, beta, sl, n_iter, schedule=None, segments=None):
    from paper_1903_10088_amd import recon
    R = recon.Recon(g, M, beta)
    if segments:
        R.set_launch(fp_segments=segments)
    counts = torch.from_numpy(sl.counts).to(dev)
    img, tr = R.os_iterate(counts, sl.i0, None, n_iter, trace=True, lambda_schedule=schedule)
    torch.cuda.synchronize()
    ref, rtr = oracle.os_iterate(g, M, beta, sl.counts, sl.i0, None, n_iter, lambda_schedule=schedule)
    return img.cpu().numpy().astype(np.float64), tr.cpu().numpy(), ref, rtr


def disc_rmse(g, a, b):
    m = oracle.initial_image(g, 1.0) > 0
    return float(np.sqrt(np.mean((a - b)[m] ** 2)))


def check_parity(dev, g, M, beta, sl, n_iter, label):
    """GPU run (own step-rule decisions) against the oracle: the lambda traces must be equal, and
    a differing decision fails with the first differing sub-iteration, the oracle's relative
    margin |f_n - f_ref| / f_n there and the GPU-vs-oracle agreement of f up to it (a near-tie
    shows as a margin below that agreement)."""
    print(f"os_iterate parity {label}: n={g.n} views={g.n_views} M={M} beta={beta} iters={n_iter}", flush=True)
    img, tr, ref, rtr = run_both(dev, g, M, beta, sl, n_iter)
    same = np.array_equal(tr[:, 1], rtr[:, 1])
    if not same:
        first = int(np.argmax(tr[:, 1] != rtr[:, 1]))
        margin = abs(rtr[first, 0] - rtr[first - 1, 0]) / rtr[first, 0] if first > 0 else np.inf
        fdiff = np.max(np.abs(tr[:first + 1, 0] - rtr[:first + 1, 0]) / rtr[:first + 1, 0])
        raise AssertionError(f"lambda decision differs first at sub-iteration {first}: oracle margin {margin:.2e}, "
                             f"f agreement up to there {fdiff:.2e}")
    rmse = disc_rmse(g, img, ref)
    frel = np.max(np.abs(tr[:, 0] - rtr[:, 0]) / rtr[:, 0])
    print(f"  rmse {rmse:.3e} (tol {RMSE_TOL:.2e}), max rel f diff {frel:.2e}, same lambda: {same}", flush=True)
    assert rmse <= RMSE_TOL
    assert frel <= 1e-4
    return same


def test_config0_full(dev):
    g = ph.config0_geometry()
    sl = ph.make_slice(g, 0, 1e4)
    check_parity(dev, g, 10, 1e-3, sl, 20, "config0")


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_config0_seeds(dev, seed):
    g = ph.config0_geometry()
    sl = ph.make_slice(g, seed, 1e4)
    check_parity(dev, g, 10, 1e-3, sl, 20, f"config0 seed {seed}")


@pytest.mark.parametrize("M,n_iter", [(1, 6), (5, 13), (33, 40)])
def test_degenerate_subsets(dev, M, n_iter):
    """One subset with every view, an odd subset count (graph parity flips), and one view per subset."""
    g = ph.Geometry(n=37, pixel_mm=10.0, n_views=33, n_channels=51, start_angle_rad=0.3)
    sl = ph.make_slice(g, 5, 5e3)
    check_parity(dev, g, M, 1e-3, sl, n_iter, f"odd geometry M={M}")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("beta", [3e-4, 1e-3, 3e-3])
def test_config1_full_500(dev, beta):
    """The clinical-scale slice over its full 500 sub-iterations for every TV weight of the sweep
    (the weight sets the TV curvature 8 beta / (M eps), where step-rule branches would part)."""
    g = ph.config1_geometry()
    sl = ph.make_slice(g, 100, 2e3, low_contrast=True)
    check_parity(dev, g, 20, beta, sl, 500, f"config1 full beta={beta}")


def test_resume_is_bitwise_and_deterministic(dev):
    from paper_1903_10088_amd import recon
    g = ph.config0_geometry()
    sl = ph.make_slice(g, 6, 1e4)
    R = recon.Recon(g, 10, 1e-3)
    counts = torch.from_numpy(sl.counts).to(dev)
    a, ta = R.os_iterate(counts, sl.i0, None, 20, trace=True)
    a2, _ = R.os_iterate(counts, sl.i0, None, 20)
    st = recon.State()
    b, tb1 = R.os_iterate(counts, sl.i0, None, 12, state=st, trace=True)
    assert st.n_done == 12
    b, tb2 = R.os_iterate(counts, sl.i0, b, 8, state=st, trace=True)
    assert st.n_done == 20
    assert torch.equal(a, a2)
    assert torch.equal(a, b)
    assert torch.equal(ta, torch.cat([tb1, tb2]))
    assert st.lam == float(ta[-1, 1]) and st.f_prev == float(ta[-1, 0])


@pytest.mark.parametrize("name", ["config0", "config1"])
def test_launch_shapes_give_identical_bits(dev, name):
    """Every projector segment count and both backprojector variants (global reads, LDS staging)
    give the same bits, so launch-shape tuning cannot change a reconstruction."""
    from paper_1903_10088_amd import recon
    if name == "config0":
        g, M, sl, n = ph.config0_geometry(), 10, ph.make_slice(ph.config0_geometry(), 8, 1e4), 20
    else:
        g, M, n = ph.config1_geometry(), 20, 40
        sl = ph.make_slice(g, 101, 2e3, low_contrast=True, supersample=2)
    counts = torch.from_numpy(sl.counts).to(dev)
    R = recon.Recon(g, M, 1e-3)
    ref = None
    shapes = [(seg, 2) for seg in (1, 2, 4, 8, 16)] + [(8, bpv) for bpv in (1, 3, 4, 5, 6)]
    for seg, bpv in shapes:
        print(f"{name}: fp_segments={seg} bp_variant={bpv}", flush=True)
        R.set_launch(fp_segments=seg, bp_variant=bpv)
        img, tr = R.os_iterate(counts, sl.i0, None, n, trace=True)
        if ref is None:
            ref = (img.clone(), tr.clone())
        else:
            assert torch.equal(img, ref[0]), (seg, bpv)
            assert torch.equal(tr, ref[1]), (seg, bpv)


def test_start_image_is_held_at_zero_outside_the_disc(dev):
    """Zero sub-iterations return the start image with the outside of the reconstruction disc
    zeroed (the iterate lives on the disc); from an arbitrary start the run matches the oracle,
    which takes the start the same way."""
    from paper_1903_10088_amd import recon
    g = ph.config0_geometry()
    sl = ph.make_slice(g, 6, 1e4)
    R = recon.Recon(g, 10, 1e-3)
    x = torch.rand((g.n, g.n), device=dev) * 0.01
    y = x.clone()
    counts = torch.from_numpy(sl.counts).to(dev)
    R.os_iterate(counts, sl.i0, y, 0)
    disc = torch.from_numpy(oracle.initial_image(g, 1.0) > 0).to(dev)
    assert torch.equal(y[disc], x[disc]) and not y[~disc].any()
    z = x.clone()
    R.os_iterate(counts, sl.i0, z, 7)
    ref, _ = oracle.os_iterate(g, 10, 1e-3, sl.counts, sl.i0, x.cpu().numpy().astype(np.float64), 7)
    rmse = float(np.sqrt(np.mean((z.cpu().numpy() - ref)[disc.cpu().numpy()] ** 2)))
    assert rmse <= RMSE_TOL


def test_nonfinite_image_flags_numeric(dev):
    """A non-finite pixel makes the squared difference non-finite: the run reports RECON_NUMERIC."""
    from paper_1903_10088_amd import recon
    g = ph.config0_geometry()
    sl = ph.make_slice(g, 6, 1e4)
    R = recon.Recon(g, 10, 1e-3)
    img = R.initial_image(dev)
    img[64, 64] = float("nan")
    st = recon.State()
    with pytest.raises(recon.ReconError) as ei:
        R.os_iterate(torch.from_numpy(sl.counts).to(dev), sl.i0, img, 10, state=st)
    assert ei.value.status == recon.RECON_NUMERIC
    assert st.flags & 1


def test_initial_image_matches_oracle(dev):
    from paper_1903_10088_amd import recon
    for g in (ph.config0_geometry(), ph.Geometry(n=37, pixel_mm=10.0, n_views=33, n_channels=51)):
        R = recon.Recon(g, 3, 1e-3)
        a = R.initial_image(dev).cpu().numpy()
        b = oracle.initial_image(g, 0.005).astype(np.float32)
        assert np.array_equal(a, b)
