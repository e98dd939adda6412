"""Pins of the CNN oracle (oracle/cnn.py) against what is fixed independently of it:
scipy's 2-D correlation, adjoint identities, finite differences of the pure FP64 network,
torch's float32 -> bfloat16 conversion, torch's Adam, and the identity at zero last layer."""
import numpy as np
import pytest
import scipy.signal

from oracle import cnn


def rng(seed):
    return np.random.default_rng(seed)


def rand_theta(seed, scale=0.3, zero_last=False):
    r = rng(seed)
    layers = []
    for c, o in cnn.LAYERS:
        W = r.normal(0, scale / np.sqrt(c * 9), (o, c, 3, 3))
        b = r.normal(0, 0.05, o)
        layers.append((W, b))
    if zero_last:
        layers[-1] = (np.zeros_like(layers[-1][0]), np.zeros_like(layers[-1][1]))
    return cnn.pack(layers)


def test_param_count_and_layout():
    assert cnn.param_count() == (32 * 9 + 32) + 6 * (32 * 32 * 9 + 32) + (32 * 9 + 1) == 56097
    th = np.arange(cnn.param_count(), dtype=np.float64)
    layers = cnn.unpack(th)
    assert layers[0][0].shape == (32, 1, 3, 3) and layers[7][0].shape == (1, 32, 3, 3)
    assert layers[0][1][0] == 288 and layers[1][0][0, 0, 0, 0] == 320  # b_1 follows W_1
    assert np.array_equal(cnn.pack(layers), th)


def test_conv_equals_scipy_correlate2d():
    r = rng(1)
    a = r.normal(size=(2, 3, 11, 7))
    W = r.normal(size=(4, 3, 3, 3))
    z = cnn.conv(a, W)
    for b in range(2):
        for o in range(4):
            ref = sum(scipy.signal.correlate2d(a[b, c], W[o, c], mode="same", boundary="fill", fillvalue=0)
                      for c in range(3))
            np.testing.assert_allclose(z[b, o], ref, rtol=0, atol=1e-12)


def test_conv_transpose_and_wgrad_are_adjoints():
    r = rng(2)
    a = r.normal(size=(2, 5, 9, 13))
    g = r.normal(size=(2, 6, 9, 13))
    W = r.normal(size=(6, 5, 3, 3))
    lhs = np.vdot(cnn.conv(a, W), g)
    np.testing.assert_allclose(np.vdot(a, cnn.conv_t(g, W)), lhs, rtol=1e-12)
    np.testing.assert_allclose(np.vdot(W, cnn.wgrad(a, g)), lhs, rtol=1e-12)


def test_conv_single_tap_is_a_shift():
    """A kernel with one nonzero tap at (dy, dx) reads the pixel (i + dy, j + dx): orientation."""
    a = np.arange(20.0).reshape(1, 1, 4, 5)
    W = np.zeros((1, 1, 3, 3))
    W[0, 0, 2, 0] = 1.0  # dy = +1, dx = -1
    z = cnn.conv(a, W)[0, 0]
    assert z[0, 1] == a[0, 0, 1, 0] and z[2, 4] == a[0, 0, 3, 3]
    assert z[3, 2] == 0.0 and z[1, 0] == 0.0  # reads past the last row / first column are zero


def test_bf16_round_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    r = rng(3)
    x = np.concatenate([r.normal(size=20000) * 10.0 ** r.uniform(-6, 6, 20000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 1.0 - 2 ** -10,
                                  0.0, 65504.0, 3.0e-30])]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16_round(x.astype(np.float64)), ref)
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert cnn.bf16_round(1.0 + 2 ** -8) == 1.0
    assert cnn.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def test_zero_last_layer_is_identity():
    th = rand_theta(4, zero_last=True)
    mu = rng(5).uniform(0, 0.01, size=(2, 12, 12))
    for emulate in (True, False):
        out, _ = cnn.forward(th, mu, 0.0049, emulate_bf16=emulate)
        np.testing.assert_allclose(out, mu, rtol=1e-15, atol=0)


def test_loss_at_identity_is_masked_mse():
    th = rand_theta(6, zero_last=True)
    r = rng(7)
    mu = r.uniform(0, 0.01, size=(3, 10, 10))
    t = r.uniform(0, 0.01, size=(3, 10, 10))
    loss, _, _ = cnn.loss_and_grad(th, mu, t, 0.005)
    D = cnn.disc_mask(10)
    assert D.sum() == 80  # 5 + 5 + 4 + 4 + 2 centres per quadrant within 5 px
    ref = np.mean([((mu[b] - t[b])[D] / 0.005) ** 2 for b in range(3)])
    np.testing.assert_allclose(loss, ref, rtol=1e-13)


@pytest.mark.parametrize("n", [7, 10])
def test_gradient_matches_finite_differences(n):
    """Pure FP64 network (no rounding): dL/dtheta along random directions by 4th-order central
    differences, and the gradient of every layer separately."""
    th = rand_theta(8, scale=1.0)
    r = rng(9)
    mu = r.uniform(0.002, 0.008, size=(2, n, n))
    t = mu + r.normal(0, 0.0005, size=mu.shape)
    loss, g, _ = cnn.loss_and_grad(th, mu, t, 0.0049, emulate_bf16=False)
    k = 0
    for l, (c, o) in enumerate(cnn.LAYERS):
        size = o * c * 9 + o
        d = np.zeros_like(th)
        d[k:k + size] = r.normal(size=size)
        k += size
        h = 1e-6 / np.linalg.norm(d)  # small enough that no pre-activation crosses its ReLU kink

        def L(s):
            return cnn.loss_and_grad(th + s * h * d, mu, t, 0.0049, emulate_bf16=False)[0]

        fd = (-L(2) + 8 * L(1) - 8 * L(-1) + L(-2)) / (12 * h)
        an = float(np.dot(g, d))
        assert abs(fd - an) <= 1e-6 * abs(an), (l, fd, an)


def test_emulated_gradient_is_close_to_exact():
    """The bfloat16 rounding points (about 2^-9 relative each, at 15 places through the network
    and back) change the gradient by a few percent, neither nothing nor everything."""
    th = rand_theta(10, scale=1.0)
    r = rng(11)
    mu = r.uniform(0.002, 0.008, size=(2, 16, 16))
    t = mu + r.normal(0, 0.0005, size=mu.shape)
    _, g0, _ = cnn.loss_and_grad(th, mu, t, 0.0049, emulate_bf16=False)
    _, g1, info = cnn.loss_and_grad(th, mu, t, 0.0049, emulate_bf16=True)
    rel = np.linalg.norm(g1 - g0) / np.linalg.norm(g0)
    assert 1e-4 < rel < 1e-1
    for a in info["acts"]:
        assert np.array_equal(cnn.bf16_round(a), a)
    for gl in info["gs"][1:8]:
        assert np.array_equal(cnn.bf16_round(gl), gl)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    r = rng(12)
    th = r.normal(size=50)
    p = torch.tensor(th.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for step in range(1, 6):
        g = r.normal(size=50)
        p.grad = torch.tensor(g.copy(), dtype=torch.float64)
        opt.step()
        th, m, v = cnn.adam_step(th, m, v, g, step, 3e-3)
        np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-14, atol=1e-15)


def test_adam_first_step_closed_form():
    """With zero moments the bias-corrected first step is -lr g / (|g| + eps)."""
    g = np.array([1e-3, -2.0, 0.0, 5e-9])
    th, _, _ = cnn.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, 0.01)
    np.testing.assert_allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
