"""Pins of the surrogate network reference: gradients against central finite
differences, the activation derivative against its closed form, and one Adam
step against the published update written out by hand."""
import numpy as np

from oracle import mlp


def test_features_shape_and_values():
    f = mlp.features([0.0, 6.0, 12.0], 3, 12.0)
    assert f.shape == (3, 6)
    assert np.allclose(f[0], [0, 0, 0, 1, 1, 1])
    assert np.allclose(f[1], [1, 0, 0, 0, -1, 1], atol=1e-15)


def test_silu_grad_closed_form():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.silu_grad(z))) < 1e-9


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    sizes = [6, 9, 7, 5]
    params = mlp.init_params(sizes, 1)
    for layer in params:
        layer[1] += rng.standard_normal(layer[1].shape) * 0.1
    x = rng.standard_normal((4, 6))
    t = rng.standard_normal((4, 5))
    y, cache = mlp.forward(params, x)
    grads = mlp.backward(params, cache, y, t)
    h = 1e-6
    for li, layer in enumerate(params):
        for pi, p in enumerate(layer):
            flat = p.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = mlp.mse(mlp.forward(params, x)[0], t)
                flat[idx] = old - h
                lm = mlp.mse(mlp.forward(params, x)[0], t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                an = grads[li][pi].reshape(-1)[idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (li, pi, idx, fd, an)


def test_adam_first_steps_by_hand():
    p = [[np.array([[1.0, -2.0]]), np.array([0.5, 0.0])]]
    g = [[np.array([[0.1, -0.3]]), np.array([2.0, 0.0])]]
    st = mlp.adam_step(p, g, None, 1, lr=0.01)
    # first step: m_hat = g, v_hat = g^2 -> p -= lr * g / (|g| + eps) = p - lr*sign(g)
    assert np.allclose(p[0][0], [[1.0 - 0.01, -2.0 + 0.01]], atol=1e-9)
    assert np.allclose(p[0][1], [0.5 - 0.01, 0.0])
    st = mlp.adam_step(p, g, st, 2, lr=0.01)
    m = 0.9 * 0.1 * 0.1 + 0.1 * 0.1       # m after two identical gradients on W[0,0]
    v = 0.999 * 0.001 * 0.01 + 0.001 * 0.01
    step = 0.01 * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    step1 = 0.01 * 0.1 / (0.1 + 1e-8)
    assert abs(p[0][0][0, 0] - (1.0 - step1 - step)) < 1e-13


def test_training_reduces_loss_on_smooth_target():
    k = np.linspace(0.05, 12, 64)
    x = mlp.features(k, 4, 12.0)
    t = np.stack([np.cos(0.7 * k), np.sin(0.4 * k) * k / 12], axis=1)
    params = mlp.init_params([8, 32, 32, 2], 3)
    st = None
    y, _ = mlp.forward(params, x)
    l0 = mlp.mse(y, t)
    for it in range(1, 301):
        y, cache = mlp.forward(params, x)
        st = mlp.adam_step(params, mlp.backward(params, cache, y, t), st, it, lr=3e-3)
    assert mlp.mse(mlp.forward(params, x)[0], t) < 0.05 * l0
