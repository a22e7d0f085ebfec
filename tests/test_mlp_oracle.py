"""Pins of the FP64 network oracle: GELU closed forms and finite differences."""
import math

import numpy as np

from oracle import mlp_oracle as mo


def test_gelu_values():
    # GELU(z) = z Phi(z): Phi(0) = 1/2, Phi(1) = 0.841344746..., symmetric identity
    assert mo.gelu(np.array([0.0]))[0] == 0.0
    assert mo.gelu(np.array([1.0]))[0] == np.float64(0.8413447460685429)
    z = np.linspace(-4, 4, 17)
    assert np.allclose(mo.gelu(z) - mo.gelu(-z), z)
    h = 1e-6
    assert np.allclose((mo.gelu(z + h) - mo.gelu(z - h)) / (2 * h), mo.gelu_prime(z), atol=1e-8)


def test_pack_roundtrip_and_count():
    th = mo.init_params(0)
    assert th.size == mo.N_PARAMS == 35841
    assert np.array_equal(mo.pack(mo.unpack(th)), th)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    th = mo.init_params(1)
    X = rng.standard_normal((24, mo.IN))
    t = rng.standard_normal(24)
    L, g = mo.loss_and_grad(th, X, t)
    idx = rng.choice(th.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(th)
        e[i] = 1e-6
        fd = (mo.loss_and_grad(th + e, X, t)[0] - mo.loss_and_grad(th - e, X, t)[0]) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, -3.14159, 1e-3])
    r = mo.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7    # ties to even
    assert np.all(np.abs(r - x) <= 2 ** -8 * np.abs(x))
