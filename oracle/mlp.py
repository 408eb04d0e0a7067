"""Warm-start network oracle: plain FP64 numpy MLP -- TEST INFRASTRUCTURE ONLY.

The network maps a LASSO problem of one bootstrap and one penalty to an ADMM
starting point: input [c / lambda_max, log(lambda / lambda_max)] (p + 1
values), two ReLU hidden layers, output z / lambda_max (p values).  This is
not part of the paper; the paper's ADMM starts cold.

Layers are y = x W' + b with W stored (out, in).  Loss = mean over samples and
outputs of (y - t)^2.  ``bf16=True`` rounds, like the GPU path, the GEMM
operands (inputs, weights, hidden activations, back-propagated gradients) to
bfloat16 with round-to-nearest-even; all arithmetic stays float64.
"""
from __future__ import annotations

import numpy as np

__all__ = ["init_params", "flat", "unflat", "forward", "loss_and_grads", "adam_step", "bf16_round"]


def bf16_round(x):
    """Round float32-representable values to bfloat16 (nearest, ties to even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out[nan] = np.nan
    return out


def shapes(n_in, hidden, n_out):
    return [(hidden, n_in), (hidden,), (hidden, hidden), (hidden,), (n_out, hidden), (n_out,)]


def init_params(n_in, hidden, n_out, seed=0):
    """He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    ps = []
    for shp in shapes(n_in, hidden, n_out):
        if len(shp) == 2:
            lim = np.sqrt(6.0 / shp[1])
            ps.append(rng.uniform(-lim, lim, size=shp))
        else:
            ps.append(np.zeros(shp))
    return ps


def flat(ps):
    return np.concatenate([p.reshape(-1) for p in ps])


def unflat(v, n_in, hidden, n_out):
    out, o = [], 0
    for shp in shapes(n_in, hidden, n_out):
        k = int(np.prod(shp))
        out.append(np.asarray(v[o:o + k], dtype=np.float64).reshape(shp))
        o += k
    return out


def _r(x, bf16):
    return bf16_round(x) if bf16 else x


def forward(ps, X, bf16=False):
    W1, b1, W2, b2, W3, b3 = ps
    x0 = _r(X, bf16)
    a1 = x0 @ _r(W1, bf16).T + b1
    h1 = _r(np.maximum(a1, 0.0), bf16)
    a2 = h1 @ _r(W2, bf16).T + b2
    h2 = _r(np.maximum(a2, 0.0), bf16)
    y = h2 @ _r(W3, bf16).T + b3
    return y, (x0, h1, h2)


def loss_and_grads(ps, X, T, bf16=False):
    """MSE loss and its gradient with respect to every parameter (analytic)."""
    W1, b1, W2, b2, W3, b3 = ps
    y, (x0, h1, h2) = forward(ps, X, bf16)
    n, m = y.shape
    d = y - T
    loss = float(np.sum(d * d) / (n * m))
    dy = _r(2.0 * d / (n * m), bf16)
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dh2 = dy @ _r(W3, bf16)
    da2 = _r(dh2 * (h2 > 0), bf16)
    gW2 = da2.T @ h1
    gb2 = da2.sum(0)
    dh1 = da2 @ _r(W2, bf16)
    da1 = _r(dh1 * (h1 > 0), bf16)
    gW1 = da1.T @ x0
    gb1 = da1.sum(0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma and Ba, 2015) on flat vectors; t counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
