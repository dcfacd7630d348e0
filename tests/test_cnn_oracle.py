"""Pins of the learned-propagator oracle (oracle/cnn_oracle.py) against independent routes:
library correlation with wrap-around, translation equivariance, central differences of the
loss and of Psi, Adam's closed form under a constant gradient, and bfloat16 rounding."""
import numpy as np
import pytest
import scipy.signal

import workloads as W
from oracle import cnn_oracle as C


def small_params(seed=3, scale=1.0):
    v = W.cnn_init(seed).astype(np.float64)
    return v * scale


def test_param_count_matches_layout():
    assert C.N_PARAMS == W.CNN_N_PARAMS == 19105


def test_convolution_is_wraparound_correlation():
    """One input and one output channel: the oracle's convolution equals scipy's 2D correlation with
    periodic boundary on the 3x3 kernel k[dy + 1][dx + 1] = W[t]."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 7, 9, 1))
    Wt = rng.standard_normal((9, 1, 1))
    got = C.conv_multi(x, Wt)[0, :, :, 0]
    k = Wt[:, 0, 0].reshape(3, 3)
    ref = scipy.signal.correlate2d(x[0, :, :, 0], k, mode="same", boundary="wrap")
    assert np.max(np.abs(got - ref)) <= 1e-13


def test_conv_transpose_is_adjoint():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 5, 6, 4))
    g = rng.standard_normal((2, 5, 6, 3))
    Wt = rng.standard_normal((9, 3, 4))
    lhs = np.sum(g * C.conv_multi(x, Wt))
    rhs = np.sum(C.conv_transpose_multi(g, Wt) * x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_translation_equivariance():
    """Circular padding: shifting the input field shifts f by the same amount."""
    v = small_params()
    x = np.random.default_rng(3).uniform(-0.5, 0.5, size=(2, 8, 10))
    f = C.forward(v, x)[0]
    fs = C.forward(v, np.roll(x, (3, -2), axis=(1, 2)))[0]
    assert np.max(np.abs(fs - np.roll(f, (3, -2), axis=(1, 2)))) <= 1e-13


def test_zero_network_loss():
    v = np.zeros(C.N_PARAMS)
    rng = np.random.default_rng(4)
    x, y = rng.standard_normal((2, 6, 6)), rng.standard_normal((2, 6, 6))
    loss, g = C.loss_and_grad(v, x, y)
    assert abs(loss - np.mean((x - y) ** 2)) <= 1e-15
    assert g[-1] == pytest.approx(2 * np.mean(x - y), rel=1e-12)   # db4


def _mask_pattern(v, x):
    _, c = C.forward(v, x)
    return [c[k] > 0 for k in ("a1", "a2", "a3")]


def test_gradient_matches_central_differences():
    """dL/dparams against central differences along random directions (FP64; directions that move a
    pre-activation across zero within the step are skipped)."""
    v = small_params(seed=8)
    v[C.N_PARAMS - 1] = 0.01
    rng = np.random.default_rng(5)
    x = rng.uniform(-0.6, 0.6, size=(2, 6, 7))
    y = x + 0.1 * rng.standard_normal(x.shape)
    loss, g = C.loss_and_grad(v, x, y)
    h = 1e-6
    checked = 0
    for _ in range(12):
        d = rng.standard_normal(C.N_PARAMS)
        m0 = _mask_pattern(v, x)
        if any(np.any(a != b) for a, b in zip(m0, _mask_pattern(v + h * d, x))) or \
           any(np.any(a != b) for a, b in zip(m0, _mask_pattern(v - h * d, x))):
            continue
        lp, _ = C.loss_and_grad(v + h * d, x, y)
        lm, _ = C.loss_and_grad(v - h * d, x, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * max(abs(fd), 1e-12), (fd, g @ d)
        checked += 1
    assert checked >= 8
    # every coordinate of the small first and last layers individually
    for k in list(range(0, 9 * 32, 37)) + list(range(C.N_PARAMS - 289, C.N_PARAMS)):
        e = np.zeros(C.N_PARAMS)
        e[k] = 1.0
        lp, _ = C.loss_and_grad(v + h * e, x, y)
        lm, _ = C.loss_and_grad(v - h * e, x, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1e-9) + 1e-12


def test_jvp_matches_central_differences():
    v = small_params(seed=9)
    rng = np.random.default_rng(6)
    x = rng.uniform(-0.6, 0.6, size=(1, 8, 8))
    e = rng.standard_normal(x.shape)
    h = 1e-7
    m0 = _mask_pattern(v, x)
    assert all(np.all(a == b) for a, b in zip(m0, _mask_pattern(v, x + h * e)))
    fd = (C.psi(v, x + h * e) - C.psi(v, x - h * e)) / (2 * h)
    got = C.jvp(v, x, e)
    assert np.max(np.abs(got - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g, the bias-corrected moments are g and g^2, so every Adam step moves a
    parameter by lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    vec, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for step in range(1, 4):
        new, m, v = C.adam(vec, g, m, v, step, lr=1e-2)
        np.testing.assert_allclose(new - vec, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)
        vec = new


def test_bf16_rounding():
    import torch
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -3.14159, 1e-30, 65504.0, 2.0 ** -130])
    got = C.bf16(vals)
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1 + 2 ** -6   # ties to even
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(got, ref)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000)
    np.testing.assert_array_equal(C.bf16(x), torch.tensor(x, dtype=torch.float32).to(torch.bfloat16)
                                  .to(torch.float64).numpy())
