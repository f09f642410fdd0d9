"""Surrogate network kernels (BF16 MFMA products, FP32 accumulation) vs the FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DIMS = (3, 128, 4, 200)  # widths of the surrogate; 200 outputs keep the test small


def _setup(seed=0, n=777):
    import torch
    from oracle import mlp as om
    from paper_1902_05875_amd import api
    net = api.MLP(*DIMS, seed=seed)
    rng = np.random.default_rng(seed)
    th = net.get_params().astype(np.float64)
    # non-zero biases so that every parameter class is exercised
    layers = om.unpack(th, DIMS)
    for _, b in layers:
        b[:] = rng.normal(scale=0.1, size=b.shape)
    net.set_params(th.astype(np.float32))
    th = net.get_params().astype(np.float64)
    X = rng.uniform(-1, 1, size=(n, 3))
    T = rng.normal(scale=0.5, size=(n, DIMS[3]))
    return net, th, X, T, torch.from_numpy(X).float().cuda(), torch.from_numpy(T).float().cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_forward_vs_oracle():
    """n = 777 rows (ragged against the 64-row tiles), 200 outputs (ragged against 64)."""
    from oracle import mlp as om
    net, th, X, T, x, t = _setup()
    y = net.forward(x).cpu().numpy()
    ref, _ = om.forward(th, X, DIMS)
    e = _rel(y, ref)
    print("mlp forward rel err (BF16 products)", e)
    assert e < 1e-2


def test_gradient_vs_oracle():
    from oracle import mlp as om
    net, th, X, T, x, t = _setup(1)
    L, g = net.loss_grad(x, t)
    Lr, gr = om.loss_and_grad(th, X, T, DIMS)
    e = _rel(g, gr)
    print(f"mlp loss {L:.6f} vs {Lr:.6f}; gradient rel err {e:.3e}")
    assert abs(L - Lr) < 2e-2 * Lr
    assert e < 1e-2
    # per-layer check: every block of the gradient carries the right values
    o = 0
    for r, c in om.shapes(*DIMS):
        for size in (r * c, r):
            assert _rel(g[o:o + size], gr[o:o + size]) < 1e-1
            o += size


def test_adam_step_vs_oracle():
    from oracle import mlp as om
    net, th, X, T, x, t = _setup(2)
    _, g = net.loss_grad(x, t)
    net.adam_step(1e-3)
    th1 = net.get_params().astype(np.float64)
    ref, _, _ = om.adam_step(th, g.astype(np.float64), np.zeros_like(th), np.zeros_like(th), 1, lr=1e-3)
    assert np.max(np.abs(th1 - ref)) < 1e-6


def test_training_fits_smooth_function():
    """Minibatch Adam on the GPU fits a smooth 3 -> 200 map (loss falls 30x)."""
    import torch
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, size=(8192, 3))
    freq = rng.normal(size=(3, DIMS[3]))
    T = np.sin(X @ freq) + 0.3 * np.cos(2 * X @ freq)
    from paper_1902_05875_amd import api
    net = api.MLP(*DIMS, seed=4)
    x = torch.from_numpy(X).float().cuda()
    t = torch.from_numpy(T).float().cuda()
    losses = net.train(x, t, epochs=40, batch=512, lr=2e-3, seed=5)
    print("training losses", losses[0], losses[-1])
    assert losses[-1] < losses[0] / 30


def test_split_products_vs_oracle():
    """Hidden products with each operand as a BF16 hi + lo pair (three MFMAs, FP32
    accumulation): forward and gradient close to the FP64 oracle at the level of ~16
    mantissa bits per operand, and much closer than one BF16 product per pair."""
    from oracle import mlp as om
    net, th, X, T, x, t = _setup(5)
    y1 = net.forward(x).cpu().numpy()
    net.set_split(1)
    y3 = net.forward(x).cpu().numpy()
    ref, _ = om.forward(th, X, DIMS)
    e1, e3 = _rel(y1, ref), _rel(y3, ref)
    L, g = net.loss_grad(x, t)
    Lr, gr = om.loss_and_grad(th, X, T, DIMS)
    eg = _rel(g, gr)
    print(f"mlp forward rel err: one BF16 product {e1:.2e}, split {e3:.2e}; split gradient {eg:.2e}")
    assert e3 < 1e-4 and e3 < 0.1 * e1
    assert abs(L - Lr) < 1e-4 * Lr and eg < 1e-3
    with pytest.raises(Exception):
        net.set_split(2)
