"""FP64 reference of the queue-ordering network (forward, loss, gradients).

TEST INFRASTRUCTURE ONLY: the GPU network's forward pass and gradients are
checked against this module; the product path never imports it.

Network: 20 -> 128 -> 128 -> 128 -> 1, GELU after each hidden layer
(GELU(z) = z Phi(z) with Phi the standard normal CDF), mean squared error.
Parameters are packed as W1 [128 x 20], b1 [128], W2 [128 x 128], b2, W3
[128 x 128], b3, W4 [1 x 128], b4 [1] (row-major, 35,841 numbers).

The GPU stores weights and activations in bfloat16 and accumulates in FP32.
`forward(..., bf16=True)` rounds at the same points (weights, the input
features and every layer output after the activation) so that the
remaining difference is FP32 accumulation order; with bf16=False it is the
plain FP64 network used to pin the gradients by finite differences.
"""
from __future__ import annotations

import math

import numpy as np

IN, HID, OUT = 20, 128, 1
SHAPES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (HID, HID)),
          ("b3", (HID,)), ("W4", (OUT, HID)), ("b4", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    assert o == theta.size == N_PARAMS
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round to bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _erf(x):
    return np.vectorize(math.erf)(x)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X, bf16_storage=False):
    """Returns (y [n], cache).  X: [n, 20]."""
    p = unpack(theta)
    r = bf16 if bf16_storage else (lambda a: np.asarray(a, dtype=np.float64))
    W = {k: r(v) if k.startswith("W") else v for k, v in p.items()}
    h0 = r(X)
    z1 = h0 @ W["W1"].T + p["b1"]
    h1 = r(gelu(z1))
    z2 = h1 @ W["W2"].T + p["b2"]
    h2 = r(gelu(z2))
    z3 = h2 @ W["W3"].T + p["b3"]
    h3 = r(gelu(z3))
    y = (h3 @ W["W4"].T + p["b4"])[:, 0]
    return y, dict(h0=h0, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3, W=W)


def loss_and_grad(theta, X, t, bf16_storage=False):
    """Mean squared error and its gradient with respect to the packed parameters."""
    y, c = forward(theta, X, bf16_storage)
    n = X.shape[0]
    r = bf16 if bf16_storage else (lambda a: a)
    W = c["W"]
    dy = r(2.0 * (y - t) / n)                   # [n]; stored like the other layer gradients
    g = {}
    g["W4"] = dy[None, :] @ c["h3"]
    g["b4"] = np.array([dy.sum()])
    dz3 = r((dy[:, None] @ W["W4"]) * gelu_prime(c["z3"]))
    g["W3"] = dz3.T @ c["h2"]
    g["b3"] = dz3.sum(0)
    dz2 = r((dz3 @ W["W3"]) * gelu_prime(c["z2"]))
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(0)
    dz1 = r((dz2 @ W["W2"]) * gelu_prime(c["z1"]))
    g["W1"] = dz1.T @ c["h0"]
    g["b1"] = dz1.sum(0)
    return float(np.mean((y - t) ** 2)), pack(g)


def init_params(seed):
    """He-style initialisation (for tests; the library has its own)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            p[name] = rng.standard_normal(shp) * math.sqrt(2.0 / shp[1])
        else:
            p[name] = rng.standard_normal(shp) * 0.01
    return pack(p)
