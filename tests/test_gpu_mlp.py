"""The queue-ordering network on the GPU against the FP64 oracle.

The oracle rounds weights and activations to bf16 at the same points as the
kernels, so forward values and gradients differ only by FP32 accumulation
order and the rare activation whose rounding falls the other way.
"""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as mo

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_01232_amd import Context
    c = Context(0)
    yield c
    c.close()


def _features(rng, n):
    X = rng.standard_normal((n, mo.IN)) * 0.8
    X[:, 6:10] = rng.uniform(0, 1, (n, 4))
    return X


@pytest.mark.parametrize("n", [1, 17, 1000, 4099])
def test_forward_matches_oracle(ctx, n):
    rng = np.random.default_rng(n)
    th = mo.init_params(7).astype(np.float32).astype(np.float64)
    ctx.mlp_set_params(th)
    X = _features(rng, n)
    y = ctx.mlp_predict(X)
    yo, _ = mo.forward(th, X.astype(np.float32).astype(np.float64), bf16_storage=True)
    err = np.abs(y - yo)
    scale = np.abs(yo).mean() + 1e-3
    print(f"n={n}: max err {err.max():.3e} median {np.median(err):.3e} scale {scale:.3e}")
    # measured on MI355X: median 3e-8 of the scale, largest 1.7e-3 (an activation
    # whose bf16 rounding falls the other way)
    assert np.median(err) <= 1e-6 * scale
    assert err.max() <= 5e-3 * scale


def test_gradient_matches_oracle(ctx):
    rng = np.random.default_rng(11)
    n = 777
    th = mo.init_params(3).astype(np.float32).astype(np.float64)
    ctx.mlp_set_params(th)
    X = _features(rng, n).astype(np.float32).astype(np.float64)
    t = rng.standard_normal(n).astype(np.float32).astype(np.float64)
    loss, g = ctx.mlp_loss_grad(X, t)
    lo, go = mo.loss_and_grad(th, X, t, bf16_storage=True)
    assert loss == pytest.approx(lo, rel=1e-3)
    for name, sl in _slices():
        a, b = g[sl], go[sl]
        rel = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30))
        print(f"{name}: rel {rel:.3e} cos {cos:.6f}")
        # measured on MI355X: relative error at most 3.6e-6, cosine 1 - 1e-12
        assert rel <= 2e-5 and cos >= 0.99999, name


def _slices():
    o = 0
    for name, shp in mo.SHAPES:
        k = int(np.prod(shp))
        yield name, slice(o, o + k)
        o += k


def test_training_reduces_loss(ctx):
    rng = np.random.default_rng(5)
    n = 20000
    X = _features(rng, n)
    t = np.tanh(X[:, 0] - 0.5 * X[:, 3]) + 0.3 * X[:, 11] ** 2 + 0.1 * X[:, 7]
    ctx.mlp_init(1)
    hist = ctx.mlp_train(X, t, epochs=12, batch=1024, lr=2e-3, seed=3)
    print("loss per epoch", hist)
    assert hist[-1] < 0.1 * hist[0]
    y = ctx.mlp_predict(X[:2000])
    assert np.mean((y - t[:2000]) ** 2) < 0.1 * np.var(t)


def test_params_roundtrip_and_errors(ctx):
    from paper_1812_01232_amd import GosmaError
    th = mo.init_params(9).astype(np.float32)
    ctx.mlp_set_params(th)
    assert np.array_equal(ctx.mlp_get_params(), th)
    with pytest.raises(GosmaError):
        ctx.mlp_train(np.zeros((4, mo.IN)), np.zeros(4), epochs=0)
