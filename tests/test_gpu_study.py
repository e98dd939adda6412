"""The convergence-study driver on a small slice: its bookkeeping against the library's own
outputs (chunked tracking equals an uninterrupted run, the kept epoch, a constant step stays
constant, the thinning timer runs)."""
import numpy as np
import pytest

from paper_1903_10088_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_10088_amd import conv_study as cs
    return cs.Case(ph.config0_geometry(), 3, 1e4, torch.device("cuda:0"))


def test_tracking_in_chunks_matches_one_run(case):
    from paper_1903_10088_amd import conv_study as cs
    from paper_1903_10088_amd import recon
    print("study: config0 tracking, 100 sub-iterations", flush=True)
    t = cs.track(case, 10, 1e-3, 100, dict(keep_best=1, lambda_compare=1))
    assert t["n"] == cs.checkpoints(100) and t["diverged_at"] is None
    R = recon.Recon(case.g, 10, 1e-3, dict(lambda_compare=1))
    img, tr = R.os_iterate(case.counts, case.i0, None, 100, trace=True)
    res = R.data_residual(case.counts, case.i0, img).cpu().numpy()
    assert t["r_over_v"][-1] == float(res[0] / res[1])  # bitwise: the chunked run is the same run
    f = tr[:, 0].cpu().numpy()
    assert np.allclose(t["epoch_mean_f"], f.reshape(10, 10).mean(axis=1), rtol=0, atol=0)
    assert t["kept"]["best_n"] == 10 * (int(np.argmin(f.reshape(10, 10).sum(axis=1))) + 1)
    assert t["r_over_v"][-1] < t["r_over_v"][0]


def test_constant_step_and_timer(case):
    from paper_1903_10088_amd import conv_study as cs
    t = cs.track(case, 10, 1e-3, 30, dict(lambda_inc=0.0, lambda_dec=0.0))
    assert set(t["lambda"]) == {0.01}
    assert np.allclose(t["epoch_mean_lambda"], 0.01, rtol=1e-15, atol=0)
    s = cs.time_slice(case, 5, 1e-3, 20, reps=2)
    assert 0 < s < 1.0
    assert cs.first_reaching(t, t["r_over_v"][-1]) <= 30


def test_limited_angle_case_takes_the_first_views():
    """The study's limited-angle case: the first views of the turn's own data at the turn's spacing,
    and tracking it equals an uninterrupted run on that arc."""
    import math

    from paper_1903_10088_amd import conv_study as cs
    from paper_1903_10088_amd import recon
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    g = ph.config0_geometry()
    full = cs.Case(g, 3, 1e4, dev)
    part = cs.Case(g, 3, 1e4, dev, first_views=100)
    assert part.g.n_views == 100 and part.g.scan_arc_rad == 2 * math.pi * 100 / 180
    assert torch.equal(part.counts, full.counts[:100])
    print("study: limited-angle case, 20 sub-iterations", flush=True)
    t = cs.track(part, 5, 1e-3, 20)
    R = recon.Recon(part.g, 5, 1e-3)
    img, _ = R.os_iterate(part.counts, part.i0, None, 20)
    res = R.data_residual(part.counts, part.i0, img).cpu().numpy()
    assert t["r_over_v"][-1] == float(res[0] / res[1])
