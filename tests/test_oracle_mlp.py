"""Pins of the FP64 screener-MLP oracle: finite differences of the loss,
BF16 rounding against torch's bfloat16 cast, Adam's first step in closed
form, and the bounded effect of the BF16 roundings."""
import numpy as np
import torch

from oracle import mlp_oracle as mo
from paper_2607_04310_amd import inputs


def _data(seed, B=64):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (B, 4)).astype(np.float32)
    t = rng.uniform(0, 1.5, B).astype(np.float32)
    theta = inputs.mlp_init_params(seed).astype(np.float64)
    theta[mo.H * mo.N_IN:mo.H * mo.N_IN + mo.H] = rng.normal(0, 0.1, mo.H)   # non-zero b1
    return X, t, theta


def test_parameter_layout():
    assert mo.N_PARAMS == inputs.MLP_PARAMS == 4545
    theta = np.arange(mo.N_PARAMS, dtype=np.float64)
    assert np.array_equal(mo.pack(*mo.unpack(theta)), theta)


def test_gradient_finite_differences():
    X, t, theta = _data(1)
    g = mo.backward(theta, X, t, bf16_on=False)
    rng = np.random.default_rng(2)
    idx = rng.choice(mo.N_PARAMS, 80, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(theta)
        e[k] = h
        fd = (mo.loss(theta + e, X, t, False) - mo.loss(theta - e, X, t, False)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 10, 10000), rng.normal(0, 1e-3, 1000),
                        [0.0, -0.0, 1.0, 3.14159, 65504.0, 1e-40]]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mo.bf16(x), ref)


def test_bf16_effect_is_bounded():
    X, t, theta = _data(4, B=256)
    y1, _ = mo.forward(theta, X, True)
    y0, _ = mo.forward(theta, X, False)
    assert np.max(np.abs(y1 - y0)) <= 0.05 * max(1.0, np.max(np.abs(y0)))


def test_adam_first_step_closed_form():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    th, m, v = mo.adam(theta, np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    # step 1: m_hat = g, v_hat = g^2, update = lr * g / (|g| + eps)
    np.testing.assert_allclose(th, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)
