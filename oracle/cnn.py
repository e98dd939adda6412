"""FP64 CPU oracle of the learned warm start: a residual CNN on reconstructed slices.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg.  The GPU library never imports or links it, and it
shares no code with the HIP kernels.

The paper's method has no network; this is the project's learned warm start for
the ordered-subset iteration.  What it computes, written out from definitions:

Network (8 layers, 3x3 kernels, 32 channels, zero "same" padding):
    x    = mu / mu_scale                           (normalised slice, float)
    a0   = bf(x)
    z_l  = conv(a_{l-1}, bf(W_l)) + b_l            l = 1..8
    a_l  = bf(relu(z_l))                            l = 1..7
    y    = x + z_8                                  (residual output)
    mu'  = mu + mu_scale * z_8                      (= mu_scale * y)
conv is the 2-D cross-correlation summed over input channels,
    conv(a, W)[o, i, j] = sum_c sum_{dy,dx in -1..1} W[o, c, dy+1, dx+1] a[c, i+dy, j+dx],
with a read as 0 outside the image.  bf() rounds to bfloat16 (8 significant
bits, round to nearest, ties to even): the network stores weights and hidden
activations in bfloat16 and accumulates in higher precision, and the oracle
rounds at exactly those points (emulate_bf16=True) or nowhere (False, for
finite-difference checks).

Training loss on the reconstruction disc D of each n x n image:
    L = 1 / (B |D|) sum_b sum_{p in D} (y_b[p] - t_b[p])^2,   t = target / mu_scale.
Backward pass (rounding points as in the forward pass):
    g_8  = dL/dz_8 = 2 (y - t) [p in D] / (B |D|)          (not rounded)
    g_7  = bf(convT(g_8, bf(W_8)) * [a_7 > 0])
    g_l  = bf(convT(g_{l+1}, bf(W_{l+1})) * [a_l > 0])     l = 6..1
    dW_l = wgrad(a_{l-1}, g_l),  db_l = sum_p g_l
convT is the adjoint of conv in its input, wgrad its adjoint in the weights:
    convT(g, W)[c, i, j] = sum_o sum_{dy,dx} W[o, c, dy+1, dx+1] g[o, i-dy, j-dx]
    wgrad(a, g)[o, c, dy+1, dx+1] = sum_{i,j} g[o, i, j] a[c, i+dy, j+dx].

Optimiser: Adam (Kingma and Ba, "Adam: A Method for Stochastic Optimization",
ICLR 2015, Algorithm 1) on float master parameters.

Parameter vector layout (float, shared with the C ABI): for l = 1..8 in turn,
W_l as [out][in][3][3] followed by b_l [out]; channel counts (in, out) are
(1, 32), (32, 32) x 6, (32, 1).
"""
from __future__ import annotations

import numpy as np

CH = 32
LAYERS = [(1, CH)] + [(CH, CH)] * 6 + [(CH, 1)]


def param_count() -> int:
    return sum(o * c * 9 + o for c, o in LAYERS)


def unpack(theta: np.ndarray):
    """Flat parameter vector -> list of (W [out][in][3][3], b [out]) float64 views."""
    theta = np.asarray(theta, dtype=np.float64)
    out, k = [], 0
    for c, o in LAYERS:
        W = theta[k:k + o * c * 9].reshape(o, c, 3, 3)
        k += o * c * 9
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    assert k == theta.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers]).astype(np.float64)


# ---------------------------------------------------------------------------
# bfloat16 rounding
# ---------------------------------------------------------------------------

def bf16_round(x) -> np.ndarray:
    """Round to the nearest value with 8 significant bits (ties to even), i.e. to bfloat16.

    Finite values of normal magnitude only (the network never meets others):
    x = m 2^e with 0.5 <= |m| < 1; m 2^8 is rounded to an integer, ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0), e - 8)


def _r(x, emulate: bool):
    return bf16_round(x) if emulate else np.asarray(x, dtype=np.float64)


# ---------------------------------------------------------------------------
# The three convolution forms (batched: arrays are [B][C][H][W])
# ---------------------------------------------------------------------------

def _pad(x: np.ndarray) -> np.ndarray:
    B, Cc, H, Wd = x.shape
    xp = np.zeros((B, Cc, H + 2, Wd + 2))
    xp[:, :, 1:-1, 1:-1] = np.asarray(x, dtype=np.float64)
    return xp


def _windows(x: np.ndarray, flip: bool = False) -> np.ndarray:
    """[B][C][H][W] -> [B][C*9][H*W]: row (c, ky, kx) holds x shifted by (dy, dx) = (ky - 1, kx - 1),
    i.e. X[b, (c, ky, kx), (i, j)] = x[b, c, i + dy, j + dx] (0 outside); flip=True shifts by
    (-dy, -dx) instead."""
    B, Cc, H, Wd = x.shape
    xp = _pad(x)
    X = np.empty((B, Cc, 3, 3, H * Wd))
    for ky in range(3):
        for kx in range(3):
            oy, ox = (2 - ky, 2 - kx) if flip else (ky, kx)
            X[:, :, ky, kx] = xp[:, :, oy:oy + H, ox:ox + Wd].reshape(B, Cc, H * Wd)
    return X.reshape(B, Cc * 9, H * Wd)


def conv(a: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Cross-correlation with zero padding: [B][C][H][W] x [O][C][3][3] -> [B][O][H][W].

    z[o, p] = sum over (c, ky, kx) of W[o, c, ky, kx] times a[c] at p + (ky - 1, kx - 1):
    one matrix product of W (as [O][C*9]) with the shifted copies of a."""
    B, Cc, H, Wd = a.shape
    z = np.matmul(W.reshape(W.shape[0], Cc * 9), _windows(a))
    return z.reshape(B, W.shape[0], H, Wd)


def conv_t(g: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Adjoint of conv in its input: [B][O][H][W] x [O][C][3][3] -> [B][C][H][W].

    a[c, p] = sum over (o, ky, kx) of W[o, c, ky, kx] times g[o] at p - (ky - 1, kx - 1)."""
    B, O, H, Wd = g.shape
    Wt = np.ascontiguousarray(W.transpose(1, 0, 2, 3)).reshape(W.shape[1], O * 9)
    a = np.matmul(Wt, _windows(g, flip=True))
    return a.reshape(B, W.shape[1], H, Wd)


def wgrad(a: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Adjoint of conv in its weights: [B][C][H][W], [B][O][H][W] -> [O][C][3][3].

    dW[o, c, ky, kx] = sum over images and pixels p of g[o, p] times a[c] at p + (ky - 1, kx - 1)."""
    B, Cc, H, Wd = a.shape
    gf = np.asarray(g, dtype=np.float64).reshape(B, g.shape[1], H * Wd)
    dW = np.matmul(gf, _windows(a).transpose(0, 2, 1)).sum(axis=0)
    return dW.reshape(g.shape[1], Cc, 3, 3)


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------

def disc_mask(n: int) -> np.ndarray:
    """Reconstruction disc of an n x n grid: pixel centres within n/2 pixels of the grid centre."""
    c = np.arange(n) - 0.5 * (n - 1)
    return (c[None, :] ** 2 + c[:, None] ** 2) <= (0.5 * n) ** 2


def forward(theta, mu, mu_scale: float, emulate_bf16: bool = True):
    """mu: [B][n][n] (1/mm).  Returns (mu_out [B][n][n], cache) with cache holding x, the
    stored activations a_0..a_7 ([B][C][n][n]) and the rounded weights."""
    layers = unpack(theta)
    x = np.asarray(mu, dtype=np.float64) / mu_scale
    Wr = [_r(W, emulate_bf16) for W, _ in layers]
    acts = [_r(x[:, None], emulate_bf16)]
    for l in range(7):
        z = conv(acts[-1], Wr[l]) + layers[l][1][None, :, None, None]
        acts.append(_r(np.maximum(z, 0.0), emulate_bf16))
    z8 = conv(acts[-1], Wr[7]) + layers[7][1][None, :, None, None]
    y = x + z8[:, 0]
    return np.asarray(mu, dtype=np.float64) + mu_scale * z8[:, 0], dict(x=x, acts=acts, Wr=Wr, y=y)


def loss_and_grad(theta, mu, target, mu_scale: float, emulate_bf16: bool = True):
    """Loss and its gradient (flat, parameter layout) for a batch of n x n slices.

    Returns (loss, grad, info) with info holding the output y, the stored
    activations a_l and the stored backward signals g_l (l = 1..8)."""
    mu = np.asarray(mu, dtype=np.float64)
    B, n, _ = mu.shape
    _, cache = forward(theta, mu, mu_scale, emulate_bf16)
    y, acts, Wr = cache["y"], cache["acts"], cache["Wr"]
    t = np.asarray(target, dtype=np.float64) / mu_scale
    D = disc_mask(n)[None]
    count = B * int(D.sum())
    diff = np.where(D, y - t, 0.0)
    loss = float(np.sum(diff * diff)) / count
    gs = [None] * 9
    gs[8] = (2.0 / count) * diff[:, None]
    grads = [None] * 8
    for l in range(8, 0, -1):
        g = gs[l]
        dW = wgrad(acts[l - 1], g)
        db = g.sum(axis=(0, 2, 3))
        grads[l - 1] = (dW, db)
        if l > 1:
            da = conv_t(g, Wr[l - 1])
            gs[l - 1] = _r(da * (acts[l - 1] > 0), emulate_bf16)
    return loss, pack(grads), dict(y=y, acts=acts, gs=gs)


def adam_step(theta, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Algorithm 1 of Kingma and Ba); `step` is the 1-based step count.
    Returns new (theta, m, v)."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    theta = np.asarray(theta, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v
