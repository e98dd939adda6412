"""GPU parity of the single operators against the FP64 oracle, through the C ABI.

Tolerances: projection <= 1e-5 relative L2 per view; backprojection and TV
gradient <= 1e-5 relative L2 over the image.  Inputs are float32-rounded once
and the oracle is fed exactly those values.
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
    "config0": (ph.config0_geometry(), 10),
    "config1": (ph.config1_geometry(), 20),
    "odd-rotated": (ph.Geometry(n=37, pixel_mm=10.0, n_views=33, n_channels=51, start_angle_rad=0.3), 5),
    "n200": (ph.Geometry(n=200, pixel_mm=2.0, n_views=90, n_channels=301), 7),
}


def f32(a):
    return np.asarray(a, dtype=np.float32)


def test_name_case(dev):
    print("gpu parity on", torch.cuda.get_device_name(0), flush=True)


def images(g, seed):
    rng = np.random.default_rng(seed)
    sl = ph.make_slice(g, seed, 1e4, supersample=2)
    disc = oracle.initial_image(g, 1.0) > 0
    rnd = np.where(disc, rng.uniform(0, 0.01, (g.n, g.n)), 0.0)
    full = rng.uniform(0, 0.01, (g.n, g.n))  # nonzero up to the grid corners
    return {"phantom": f32(sl.truth), "random-disc": f32(rnd), "random-full": f32(full)}


@pytest.mark.parametrize("name", list(GEOMS))
@pytest.mark.parametrize("segments", [1, 4, 8])
def test_project_per_view(dev, name, segments):
    from paper_1903_10088_amd import recon
    g, M = GEOMS[name]
    print(f"project {name} segments={segments}", flush=True)
    R = recon.Recon(g, M, 1e-3)
    R.set_launch(fp_segments=segments)
    for kind, img in images(g, 1).items():
        ref = oracle.project(g, img.astype(np.float64))
        out = R.project(torch.from_numpy(img).to(dev), -1).cpu().numpy().astype(np.float64)
        err = np.linalg.norm(out - ref, axis=1) / np.linalg.norm(ref, axis=1)
        assert err.max() <= 1e-5, (kind, err.max())
        s = M - 1  # a subset, in subset order
        views = oracle.subset_views(g.n_views, M, s)
        outs = R.project(torch.from_numpy(img).to(dev), s).cpu().numpy()
        assert np.array_equal(outs, out[views].astype(np.float32))


@pytest.mark.parametrize("name", list(GEOMS))
def test_backproject(dev, name):
    from paper_1903_10088_amd import recon
    g, M = GEOMS[name]
    print(f"backproject {name}", flush=True)
    R = recon.Recon(g, M, 1e-3)
    rng = np.random.default_rng(2)
    sl = ph.make_slice(g, 2, 2e3, supersample=2)
    # a likelihood-gradient-like sinogram and a random one
    w_like = f32(np.exp(-sl.line_integrals) - sl.counts / 2e3)
    rnd = f32(rng.uniform(-1, 1, (g.n_views, g.n_channels)))
    for kind, sino in {"residual": w_like, "random": rnd}.items():
        ref = oracle.backproject(g, sino.astype(np.float64))
        out = R.backproject(torch.from_numpy(sino).to(dev), -1).cpu().numpy().astype(np.float64)
        err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
        assert err <= 1e-5, (kind, err)
        s = 1 % M
        views = oracle.subset_views(g.n_views, M, s)
        ref_s = oracle.backproject(g, sino[views].astype(np.float64), views)
        out_s = R.backproject(torch.from_numpy(np.ascontiguousarray(sino[views])).to(dev), s).cpu().numpy()
        err = np.linalg.norm(out_s - ref_s) / np.linalg.norm(ref_s)
        assert err <= 1e-5, (kind, "subset", err)


@pytest.mark.parametrize("name", ["config0", "odd-rotated"])
def test_gpu_adjoint_identity(dev, name):
    from paper_1903_10088_amd import recon
    g, M = GEOMS[name]
    R = recon.Recon(g, M, 1e-3)
    rng = np.random.default_rng(3)
    x = torch.from_numpy(f32(rng.uniform(0, 1, (g.n, g.n)))).to(dev)
    y = torch.from_numpy(f32(rng.uniform(0, 1, (g.n_views, g.n_channels)))).to(dev)
    lhs = float((R.project(x).double() * y.double()).sum())
    rhs = float((x.double() * R.backproject(y).double()).sum())
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


@pytest.mark.parametrize("name", ["config0", "config1", "odd-rotated"])
def test_tv_grad(dev, name):
    from paper_1903_10088_amd import recon
    g, M = GEOMS[name]
    R = recon.Recon(g, M, 1e-3, params=dict(tv_eps_per_mm=1e-4))
    rng = np.random.default_rng(4)
    sl = ph.make_slice(g, 4, 1e4, supersample=2)
    cases = {"phantom+noise": f32(sl.truth + 2e-4 * rng.standard_normal((g.n, g.n))),
             "random": f32(rng.uniform(0, 0.01, (g.n, g.n)))}
    for kind, img in cases.items():
        _, ref = oracle.tv(img.astype(np.float64), 1e-4)
        out = R.tv_grad(torch.from_numpy(img).to(dev)).cpu().numpy().astype(np.float64)
        err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
        assert err <= 1e-5, (kind, err)


def test_backprojection_is_deterministic(dev):
    from paper_1903_10088_amd import recon
    g, M = GEOMS["config1"]
    R = recon.Recon(g, M, 1e-3)
    rng = np.random.default_rng(5)
    y = torch.from_numpy(f32(rng.uniform(-1, 1, (g.n_views, g.n_channels)))).to(dev)
    a = R.backproject(y).clone()
    b = R.backproject(y).clone()
    assert torch.equal(a, b)


def test_empty_image_projects_to_zero(dev):
    from paper_1903_10088_amd import recon
    g, M = GEOMS["odd-rotated"]
    R = recon.Recon(g, M, 1e-3)
    z = torch.zeros((g.n, g.n), dtype=torch.float32, device=dev)
    assert float(R.project(z).abs().max()) == 0.0
    assert float(R.backproject(torch.zeros((g.n_views, g.n_channels), device=dev)).abs().max()) == 0.0


def test_bad_shapes_raise(dev):
    from paper_1903_10088_amd import recon
    g, M = GEOMS["config0"]
    R = recon.Recon(g, M, 1e-3)
    with pytest.raises(ValueError):
        R.project(torch.zeros((g.n, g.n + 1), device=dev))
    with pytest.raises(recon.ReconError):
        R.project(torch.zeros((g.n, g.n), device=dev), subset=M)
