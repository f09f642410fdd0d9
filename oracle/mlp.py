"""Plain FP64 reference of the surrogate network and its training step.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Network (the surrogate for the reaction derivative tables): a fully connected
tanh network
    a_0 = x                                    (n_in inputs)
    a_{l+1} = tanh(W_l a_l + b_l),  l = 0 .. n_hidden-1   (width units each)
    y = W_out a_{n_hidden} + b_out              (n_out outputs)
with the mean-squared loss  L = (1 / (n n_out)) sum_{samples, outputs} (y - t)^2,
gradients by the chain rule, and Adam (Kingma & Ba, 2015) with bias correction.

Parameter vector layout (float, row-major matrices, W[j][i] = weight from input
i to unit j): W_0, b_0, W_1, b_1, ..., W_out, b_out.
"""
from __future__ import annotations

import numpy as np


def shapes(n_in, width, n_hidden, n_out):
    """[(rows, cols) of W_l, ...] for every layer including the output layer."""
    s = [(width, n_in)] + [(width, width)] * (n_hidden - 1) + [(n_out, width)]
    return s


def num_params(n_in, width, n_hidden, n_out):
    return sum(r * c + r for r, c in shapes(n_in, width, n_hidden, n_out))


def unpack(theta, dims):
    """List of (W, b) views of the flat parameter vector."""
    out, o = [], 0
    for r, c in shapes(*dims):
        W = theta[o:o + r * c].reshape(r, c)
        o += r * c
        b = theta[o:o + r]
        o += r
        out.append((W, b))
    assert o == theta.size
    return out


def forward(theta, X, dims):
    """Outputs y (n x n_out) and the activations a_0 .. a_{n_hidden}."""
    layers = unpack(np.asarray(theta, np.float64), dims)
    a = [np.asarray(X, np.float64)]
    for W, b in layers[:-1]:
        a.append(np.tanh(a[-1] @ W.T + b))
    W, b = layers[-1]
    return a[-1] @ W.T + b, a


def loss_and_grad(theta, X, T, dims):
    """Mean-squared loss and its gradient with respect to the parameter vector."""
    theta = np.asarray(theta, np.float64)
    y, a = forward(theta, X, dims)
    n, n_out = y.shape
    r = y - np.asarray(T, np.float64)
    L = float(np.sum(r * r) / (n * n_out))
    layers = unpack(theta, dims)
    grads = [None] * len(layers)
    d = 2.0 * r / (n * n_out)                      # dL/dy
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        grads[li] = (d.T @ a[li], d.sum(axis=0))   # dL/dW_l, dL/db_l
        if li > 0:
            d = (d @ W) * (1.0 - a[li] ** 2)       # back through tanh of layer li-1
    g = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return L, g


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
