"""Reference surrogate network: a multilayer perceptron with SiLU hidden
layers that maps a parameter vector to a standardised log-likelihood, its
MSE loss, gradients and Adam update (Kingma & Ba 2015).

TEST INFRASTRUCTURE ONLY.

Arithmetic model it emulates (FP64 with explicit BF16 rounding): the input
(mapped from the prior box to [-1, 1]), the weights of the hidden layers and
every hidden activation are rounded to bfloat16 (round to nearest even);
products of BF16 values are exact and are summed here in FP64; biases, the
output layer and all optimiser state are FP32 values. With emulate=False
nothing is rounded (plain FP64), which is what the pins compare against
PyTorch and finite differences.

Packed parameter layout (FP32 master copy), for input d and width w:
    W1 [w, d], b1 [w], W2 [w, w], b2 [w], W3 [w, w], b3 [w], W4 [w], b4 [1]
(weights row-major, output-by-input).
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to bfloat16 (via FP32, nearest even); returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    rnd = ((b >> 16) & 1) + 0x7FFF
    b = ((b + rnd) & 0xFFFF0000).astype(np.uint32)
    out = b.view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def layout(d_in, width):
    """(name, shape) of each packed block."""
    return [("W1", (width, d_in)), ("b1", (width,)), ("W2", (width, width)), ("b2", (width,)),
            ("W3", (width, width)), ("b3", (width,)), ("W4", (width,)), ("b4", (1,))]


def n_params(d_in, width):
    return sum(int(np.prod(s)) for _, s in layout(d_in, width))


def unpack(flat, d_in, width):
    out, o = {}, 0
    for name, shape in layout(d_in, width):
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p, d_in, width):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in layout(d_in, width)])


def standardise_inputs(theta, lo, hi):
    """Map the prior box to [-1, 1]."""
    return 2.0 * (np.asarray(theta, np.float64) - lo) / (hi - lo) - 1.0


def affine_inputs(theta, center, T):
    """General affine input map x = T (theta - center), one row per sample."""
    return (np.asarray(theta, np.float64) - center) @ np.asarray(T, np.float64).T


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(flat, x, d_in, width, emulate=True):
    """x: standardised inputs [B, d]. Returns (output [B], cache)."""
    p = unpack(flat, d_in, width)
    r = bf16 if emulate else (lambda v: np.asarray(v, np.float64))
    a = r(x)
    cache = {"a0": a}
    for l in (1, 2, 3):
        z = a @ r(p["W%d" % l]).T + p["b%d" % l]
        a = r(silu(z))
        cache["z%d" % l], cache["a%d" % l] = z, a
    out = a @ p["W4"] + p["b4"][0]
    cache["out"] = out
    return out, cache


def loss_and_grad(flat, x, t, d_in, width, emulate=True):
    """MSE over the batch, mean((out - t)^2), and its gradient (packed).
    With emulate, the backpropagated pre-activation gradients entering the
    BF16 products are rounded to BF16 as well."""
    p = unpack(flat, d_in, width)
    r = bf16 if emulate else (lambda v: np.asarray(v, np.float64))
    out, c = forward(flat, x, d_in, width, emulate)
    B = x.shape[0]
    diff = out - t
    loss = np.mean(diff ** 2)
    g = {}
    dout = 2.0 * diff / B
    g["W4"] = c["a3"].T @ dout
    g["b4"] = np.array([dout.sum()])
    da = np.outer(dout, p["W4"])
    for l in (3, 2, 1):
        dz = r(da * dsilu(c["z%d" % l]))
        g["W%d" % l] = dz.T @ c["a%d" % (l - 1)]
        g["b%d" % l] = dz.sum(0)
        if l > 1:
            da = dz @ r(p["W%d" % l])
    return loss, pack(g, d_in, width)


def adam(flat, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (flat, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v
