"""FP64 reference of the frequency surrogate network.

Test infrastructure only (see the package docstring).

The surrogate is not part of the paper: it maps a wavenumber k to the surface
unknowns of a fixed geometry, trained on solutions the direct method produces,
and every prediction is accepted only when the float64 residual of the
discrete equation (Eq. BRIEF discretised) is below tolerance.

Definition (written out plainly):
  features   gamma(k) = [sin(2^l pi k / K), cos(2^l pi k / K)], l = 0..L-1
  hidden     h_{i+1} = silu(h_i W_i + b_i), silu(z) = z / (1 + e^{-z})
  output     y = h_last W_out + b_out           (no activation)
  loss       mean over batch and outputs of (y - t)^2
  Adam       m = b1 m + (1-b1) g ; v = b2 v + (1-b2) g^2 ;
             p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
             (Kingma & Ba, 2015, Algorithm 1)
Weights are stored [in, out] row-major; a batch is [B, features].
"""
from __future__ import annotations

import numpy as np


def features(k, n_oct: int, kscale: float):
    k = np.asarray(k, dtype=np.float64)
    f = (2.0 ** np.arange(n_oct))[None, :] * np.pi * k[:, None] / kscale
    return np.concatenate([np.sin(f), np.cos(f)], axis=1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(sizes, seed: int):
    """He-style uniform init, seeded; sizes = [in, h1, ..., out]."""
    rng = np.random.default_rng(seed)
    params = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / a)
        params.append([rng.uniform(-lim, lim, (a, b)), np.zeros(b)])
    return params


def forward(params, x):
    """Returns (y, cache) with cache = list of (input, pre-activation) per layer."""
    cache = []
    h = x
    L = len(params)
    for i, (W, b) in enumerate(params):
        z = h @ W + b
        cache.append((h, z))
        h = silu(z) if i < L - 1 else z
    return h, cache


def mse(y, t):
    return float(np.mean((y - t) ** 2))


def backward(params, cache, y, t):
    """Gradients of the mean-squared loss with respect to every W, b."""
    B, O = y.shape
    g = 2.0 * (y - t) / (B * O)
    grads = [None] * len(params)
    L = len(params)
    for i in range(L - 1, -1, -1):
        h, z = cache[i]
        if i < L - 1:
            g = g * silu_grad(z)
        W, _ = params[i]
        grads[i] = [h.T @ g, g.sum(axis=0)]
        g = g @ W.T
    return grads


def adam_step(params, grads, state, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    if state is None:
        state = [[(np.zeros_like(p), np.zeros_like(p)) for p in layer] for layer in params]
    for li, layer in enumerate(params):
        for pi, p in enumerate(layer):
            m, v = state[li][pi]
            gr = grads[li][pi]
            m = b1 * m + (1 - b1) * gr
            v = b2 * v + (1 - b2) * gr * gr
            state[li][pi] = (m, v)
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            p -= lr * mh / (np.sqrt(vh) + eps)
    return state
