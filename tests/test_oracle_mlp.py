"""Pins of the surrogate-network oracle (oracle/mlp.py) to facts independent of it."""
import numpy as np

from oracle import mlp

DIMS = (3, 5, 3, 4)  # n_in, width, n_hidden, n_out


def _rand(seed=0):
    rng = np.random.default_rng(seed)
    th = rng.normal(scale=0.7, size=mlp.num_params(*DIMS))
    X = rng.uniform(-1, 1, size=(6, 3))
    T = rng.normal(size=(6, 4))
    return th, X, T


def test_param_count():
    # 3->5, 5->5, 5->5, 5->4 with biases
    assert mlp.num_params(*DIMS) == (15 + 5) + 2 * (25 + 5) + (20 + 4)


def test_gradient_vs_central_differences():
    """Back-propagation against central differences of the loss (every parameter)."""
    th, X, T = _rand()
    L, g = mlp.loss_and_grad(th, X, T, DIMS)
    h = 1e-6
    fd = np.empty_like(th)
    for i in range(th.size):
        e = np.zeros_like(th)
        e[i] = h
        fd[i] = (mlp.loss_and_grad(th + e, X, T, DIMS)[0] - mlp.loss_and_grad(th - e, X, T, DIMS)[0]) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-8 * max(1.0, np.max(np.abs(fd)))


def test_forward_special_cases():
    """Zero hidden weights and biases: every hidden unit is tanh(0) = 0, so y = b_out;
    a single path x -> unit -> output reproduces w2 tanh(w1 x + b1) + b2."""
    th = np.zeros(mlp.num_params(*DIMS))
    layers = mlp.unpack(th, DIMS)
    layers[-1][1][:] = [1.0, -2.0, 0.5, 3.0]
    y, _ = mlp.forward(th, np.ones((2, 3)), DIMS)
    assert np.array_equal(y, np.tile([1.0, -2.0, 0.5, 3.0], (2, 1)))
    dims = (1, 1, 1, 1)
    th = np.array([0.7, -0.2, 1.5, 0.25])  # W0, b0, Wout, bout
    x = np.array([[0.3], [-1.1]])
    y, _ = mlp.forward(th, x, dims)
    assert np.allclose(y[:, 0], 1.5 * np.tanh(0.7 * x[:, 0] - 0.2) + 0.25, rtol=0, atol=1e-15)


def test_adam_first_step_closed_form():
    """From zero moments, the bias-corrected first step is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th0 = np.array([1.0, 2.0, 3.0, 4.0])
    th, m, v = mlp.adam_step(th0, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(th, th0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    """Plain full-batch Adam on the oracle decreases the loss (sanity of the pieces together)."""
    th, X, T = _rand(3)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    L0 = mlp.loss_and_grad(th, X, T, DIMS)[0]
    for t in range(1, 201):
        L, g = mlp.loss_and_grad(th, X, T, DIMS)
        th, m, v = mlp.adam_step(th, g, m, v, t, lr=1e-2)
    assert mlp.loss_and_grad(th, X, T, DIMS)[0] < 0.2 * L0
