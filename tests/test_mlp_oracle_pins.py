"""Pins of the cost-model MLP oracle: its gradient against central finite
differences, its forward pass against a hand-built network, Adam's first step
against the closed form lr * sign(g)."""
import numpy as np

from oracle import mlp


def _theta(seed=0, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, mlp.NPARAM)


def test_parameter_count():
    assert mlp.NPARAM == 8 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4801


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    th = _theta(2)
    X = rng.normal(size=(37, 8))
    T = rng.normal(size=37)
    _, g = mlp.loss_grad(th, X, T)
    idx = rng.choice(mlp.NPARAM, 120, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAM - 1, 0, 8 * 64 + 63]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss(th + e, X, T) - mlp.loss(th - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_forward_on_hand_built_network():
    # one active path: x0 -> h1[0] -> h2[0] -> y, all weights 1, biases 0
    p = {name: np.zeros(shape) for name, shape in mlp.SIZES}
    p["W1"][0, 0] = 2.0
    p["W2"][0, 0] = 3.0
    p["W3"][0] = 5.0
    p["b3"][0] = 0.5
    th = mlp.pack(p)
    y, _ = mlp.forward(th, np.array([[1.5, 9, 9, 9, 9, 9, 9, 9], [-1.0, 0, 0, 0, 0, 0, 0, 0]]))
    assert np.allclose(y, [2 * 1.5 * 3 * 5 + 0.5, 0.5])  # ReLU blocks the negative input


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th = np.zeros(4)
    out, m, v = mlp.adam(th, g, np.zeros(4), np.zeros(4), step=1, lr=0.01)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> lr * g / (|g| + eps)
    assert np.allclose(out, -0.01 * g / (np.abs(g) + 1e-8))
