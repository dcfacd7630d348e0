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


# ---------------------------------------------------------------------------
# the learned windows (FAS form of Alg. 2 at the coarsest level, section 2.1 local grids)
# ---------------------------------------------------------------------------

def window_inputs(nt_c=9, h=6, w=8, seed=11):
    rng = np.random.default_rng(seed)
    states = rng.uniform(-1, 1, size=(nt_c + 1, h, w))
    r = rng.standard_normal((nt_c + 1, h, w))
    r[0] = 0.0
    return states, r


def windowed_residual_sums(r, k):
    """e_p = r_s + r_{s+1} + ... + r_p, s = max(0, p - k + 1), by a running sum over the residuals."""
    c = np.concatenate([np.zeros((1,) + r.shape[1:]), np.cumsum(r, axis=0)])
    return np.stack([c[p + 1] - c[max(0, p - k + 1)] for p in range(r.shape[0])])


@pytest.mark.parametrize("k", [1, 2, 4, 10, 11])
def test_learned_windows_zero_network_sum_residuals(k):
    """A zero network gives Psi = I; the FAS window then telescopes to the sum of the residuals over
    the window's C-points (v cancels).  Pins the start s, the first row (v_s + r_s) and tau's index."""
    states, r = window_inputs()
    got = C.learned_local_solves(np.zeros(C.N_PARAMS), states, r, k, bf16_mode=False)
    ref = windowed_residual_sums(r, k)
    assert np.max(np.abs(got - ref)) <= 1e-13


@pytest.mark.parametrize("bf16_mode", [False, True])
def test_learned_windows_constant_bias_cancels(bf16_mode):
    """Only the output bias set (f = c): Psi(x) = x + c, and c cancels between Psi(w) and tau's
    -Psi(v): the same residual sums.  A sign error in tau would leave (p - s) c."""
    states, r = window_inputs(seed=12)
    P = C.unpack(np.zeros(C.N_PARAMS))
    P["b4"][0] = 0.375
    P["b1"][...] = 0.2     # hidden biases do not reach f while the weights are zero
    got = C.learned_local_solves(C.pack(P), states, r, 4, bf16_mode=bf16_mode)
    assert np.max(np.abs(got - windowed_residual_sums(r, 4))) <= 1e-13


def test_fas_windows_equal_c_oracle_local_solves(orc):
    """With the re-discretised coarse step as Psi, the windows equal the C oracle's FAS local solves
    (written separately, pinned by the windows of Figs. 1, 2 and 5 and the E_cc closed form), bit for bit."""
    p, u0 = W.small_problem(W.AC2D, seed=3, nt=40, nx=6, ny=5)
    o = W.Options(m=4, k=3, coarse_form=2, coarse_substeps=2)
    NT = p.nt // o.m
    rng = np.random.default_rng(5)
    vc = rng.uniform(-0.5, 0.5, size=(NT + 1, p.n))
    rc = 1e-2 * rng.standard_normal((NT + 1, p.n))
    rc[0] = 0.0
    ref = orc.local_solves(p, o, rc, vc)
    got = C.fas_local_solves(lambda x: orc.coarse_step(p, o, x.reshape(-1)).reshape(p.ny, p.nx),
                             vc.reshape(NT + 1, p.ny, p.nx), rc.reshape(NT + 1, p.ny, p.nx), o.k)
    np.testing.assert_array_equal(got.reshape(NT + 1, p.n), ref)


def test_planted_window_off_by_one_is_caught():
    """A window loop started one C-point early (s = max(0, p - k)) fails the zero-network pin."""
    states, r = window_inputs(seed=13)
    k = 3

    def planted(psi_fn, states, r, k):
        NT = r.shape[0] - 1
        tau = np.zeros_like(states)
        for j in range(1, NT + 1):
            tau[j] = (states[j] - psi_fn(states[j - 1])) + r[j]
        out = np.zeros_like(states)
        for p in range(NT + 1):
            s = max(0, p - k)
            w = states[s] + r[s]
            for j in range(s + 1, p + 1):
                w = psi_fn(w) + tau[j]
            out[p] = w - states[p]
        return out

    bad = planted(lambda x: x, states, r, k)
    assert np.max(np.abs(bad - windowed_residual_sums(r, k))) > 1e-3
    good = C.fas_local_solves(lambda x: x, states, r, k)
    assert np.max(np.abs(good - windowed_residual_sums(r, k))) <= 1e-13
