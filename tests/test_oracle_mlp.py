"""Pins of the surrogate's FP64 oracle: GELU at closed-form points, backward pass
against central finite differences of the forward pass, and Adam's first step."""
import numpy as np
import pytest
from scipy.stats import norm

from oracle import mlp as M
from paper_1812_10375_amd import scenarios as S


def test_gelu_closed_forms():
    z = np.array([-2.0, -1.0, 0.0, 0.5, 1.0, 3.0])
    # g(z) = z Phi(z) with the standard normal CDF
    assert np.allclose(M.gelu(z), z * norm.cdf(z), rtol=0, atol=1e-15)
    assert M.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-15)
    assert M.gelu_grad(0.0) == 0.5
    # derivative by central differences
    h = 1e-6
    assert np.allclose(M.gelu_grad(z), (M.gelu(z + h) - M.gelu(z - h)) / (2 * h), atol=1e-9)


def test_parameter_layout_matches_the_generator():
    assert M.N_PARAMS == 17410
    v = S.mlp_init_params(1, 2)
    assert v.shape == (2, M.N_PARAMS)
    p = M.unpack(v[0])
    assert np.all(p["b1"] == 0) and np.all(p["b3"] == 0)
    assert np.abs(p["W2"]).max() <= np.sqrt(6.0 / 256)
    assert np.array_equal(M.pack(p), v[0])


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    vec = S.mlp_init_params(4, 1)[0] + 0.01 * rng.standard_normal(M.N_PARAMS)
    X = rng.uniform(-1, 1, size=(7, 4))
    T = rng.standard_normal((7, 2))
    loss, g = M.loss_and_grad(vec, X, T)
    idx = np.concatenate([rng.choice(np.arange(0, 512), 6, replace=False),             # W1
                          rng.choice(np.arange(512, 640), 3, replace=False),           # b1
                          rng.choice(np.arange(640, 640 + 16384), 8, replace=False),   # W2
                          rng.choice(np.arange(17024, 17152), 3, replace=False),       # b2
                          rng.choice(np.arange(17152, 17408), 5, replace=False),       # W3
                          [17408, 17409]])                                             # b3
    h = 1e-6
    for i in idx:
        e = np.zeros_like(vec)
        e[i] = h
        fd = (M.loss_and_grad(vec + e, X, T)[0] - M.loss_and_grad(vec - e, X, T)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i


def test_adam_first_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(5)
    vec = rng.standard_normal(100)
    grad = rng.standard_normal(100)
    new, m, v = M.adam_step(vec, grad, np.zeros(100), np.zeros(100), 1, lr=1e-3, eps=1e-12)
    assert np.allclose(new - vec, -1e-3 * np.sign(grad), rtol=1e-9)
    assert np.allclose(m, 0.1 * grad) and np.allclose(v, 0.001 * grad * grad)
