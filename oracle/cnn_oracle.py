"""CPU oracle of the learned coarse propagator -- TEST INFRASTRUCTURE ONLY.

Psi(u) = u + f(u), f a four-layer 3x3 convolutional network on the periodic
grid: 1 -> 32 -> 32 -> 32 -> 1 channels, ReLU after the first three layers,
circular padding (the Allen-Cahn grid is periodic).  The paper lets the
coarse propagator be any approximation of Phi over a coarse step (section
2.1); this one is learned from pairs (u_n, u_{n+m}) of the fine propagator.

Plain numpy in FP64: a convolution is the sum over the nine taps of the
shifted input times that tap's weight matrix, out(p) = sum_t W[t] in(p + t),
t = (dy, dx) in {-1, 0, 1}^2, tap index (dy + 1) * 3 + (dx + 1).

`bf16=True` rounds weights, activations and back-propagated signals to
bfloat16 (round to nearest even) at the points where the GPU kernels store
them, so the GPU path can be checked at its own precision; products and sums
stay FP64 here.  Only tests/ and the smoke check import this module.

Parameter vector layout (float, 19105 entries):
  W1[9][32] (tap, out channel), b1[32], W2[9][32][32] (tap, out, in), b2[32],
  W3[9][32][32], b3[32], W4[9][32] (tap, in channel), b4[1].
"""
from __future__ import annotations

import numpy as np

C = 32
SIZES = [("W1", (9, C)), ("b1", (C,)), ("W2", (9, C, C)), ("b2", (C,)), ("W3", (9, C, C)), ("b3", (C,)),
         ("W4", (9, C)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)
TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def unpack(vec):
    """Split the flat parameter vector into named FP64 arrays."""
    vec = np.asarray(vec, dtype=np.float64)
    assert vec.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = vec[o:o + n].reshape(shape)
        o += n
    return out


def pack(params):
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    rounded = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def shift(x, dy, dx):
    """x(p + (dy, dx)) on the periodic grid; x is [B, H, W, ...]."""
    return np.roll(x, shift=(-dy, -dx), axis=(1, 2))


def conv_multi(x, W):
    """out(p)[o] = sum_t sum_i W[t][o][i] x(p + t)[i]; x [B,H,W,Cin], W [9,Cout,Cin]."""
    out = 0.0
    for t, (dy, dx) in enumerate(TAPS):
        out = out + shift(x, dy, dx) @ W[t].T
    return out


def conv_transpose_multi(g, W):
    """Adjoint of conv_multi: out(p)[i] = sum_t sum_o W[t][o][i] g(p - t)[o]."""
    out = 0.0
    for t, (dy, dx) in enumerate(TAPS):
        out = out + shift(g, -dy, -dx) @ W[t]
    return out


def forward(vec, x, bf16_mode=False):
    """f(x) for x [B, H, W]; returns (f, cache)."""
    P = unpack(vec)
    q = bf16 if bf16_mode else (lambda v: np.asarray(v, dtype=np.float64))
    W1, W2, W3, W4 = q(P["W1"]), q(P["W2"]), q(P["W3"]), q(P["W4"])
    x0 = q(x)[..., None]                                   # [B,H,W,1]
    z1 = conv_multi(x0, W1[:, :, None]) + P["b1"]          # W1 as [9, 32, 1]
    a1 = q(np.maximum(z1, 0.0))
    z2 = conv_multi(a1, W2) + P["b2"]
    a2 = q(np.maximum(z2, 0.0))
    z3 = conv_multi(a2, W3) + P["b3"]
    a3 = q(np.maximum(z3, 0.0))
    f = conv_multi(a3, W4[:, None, :])[..., 0] + P["b4"][0]  # W4 as [9, 1, 32]
    cache = dict(x0=x0, a1=a1, a2=a2, a3=a3, W1=W1, W2=W2, W3=W3, W4=W4, q=q)
    return f, cache


def psi(vec, x, bf16_mode=False):
    """The learned coarse propagator Psi(x) = x + f(x)."""
    return np.asarray(x, dtype=np.float64) + forward(vec, x, bf16_mode)[0]


def loss_and_grad(vec, x, y, bf16_mode=False):
    """MSE loss L = mean((x + f(x) - y)^2) and dL/dparams (flat), by back-propagation."""
    f, c = forward(vec, x, bf16_mode)
    q = c["q"]
    n = f.size
    d = np.asarray(x, dtype=np.float64) + f - y
    loss = float(np.sum(d * d) / n)
    g4 = 2.0 * d / n                                        # dL/df, [B,H,W]
    grads = {}
    # layer 4 (32 -> 1)
    grads["W4"] = np.stack([np.einsum("bhw,bhwc->c", g4, shift(c["a3"], dy, dx)) for dy, dx in TAPS])
    grads["b4"] = np.array([g4.sum()])
    g3 = conv_transpose_multi(g4[..., None], c["W4"][:, None, :])
    g3 = q(g3 * (c["a3"] > 0))
    # layer 3 (32 -> 32)
    grads["W3"] = np.stack([np.einsum("bhwo,bhwi->oi", g3, shift(c["a2"], dy, dx)) for dy, dx in TAPS])
    grads["b3"] = g3.sum(axis=(0, 1, 2))
    g2 = q(conv_transpose_multi(g3, c["W3"]) * (c["a2"] > 0))
    # layer 2
    grads["W2"] = np.stack([np.einsum("bhwo,bhwi->oi", g2, shift(c["a1"], dy, dx)) for dy, dx in TAPS])
    grads["b2"] = g2.sum(axis=(0, 1, 2))
    g1 = q(conv_transpose_multi(g2, c["W2"]) * (c["a1"] > 0))
    # layer 1 (1 -> 32)
    grads["W1"] = np.stack([np.einsum("bhwc,bhw->c", g1, shift(c["x0"], dy, dx)[..., 0]) for dy, dx in TAPS])
    grads["b1"] = g1.sum(axis=(0, 1, 2))
    return loss, pack(grads)


def jvp(vec, v, e, bf16_mode=False):
    """The derivative of Psi at v applied to e: e + J_f(v) e (ReLU masks of the forward pass at v)."""
    _, c = forward(vec, v, bf16_mode)
    q = c["q"]
    d0 = q(e)[..., None]
    d1 = q(conv_multi(d0, c["W1"][:, :, None]) * (c["a1"] > 0))
    d2 = q(conv_multi(d1, c["W2"]) * (c["a2"] > 0))
    d3 = q(conv_multi(d2, c["W3"]) * (c["a3"] > 0))
    df = conv_multi(d3, c["W4"][:, None, :])[..., 0]
    return np.asarray(e, dtype=np.float64) + df


def adam(vec, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba); step counts from 1.  Returns (vec, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return vec - lr * mhat / (np.sqrt(vhat) + eps), m, v


def fas_local_solves(psi_fn, states, r, k):
    """Every window's correction in the FAS form (Alg. 2, coarsest level; section 2.1 local grids) with
    the coarse propagator psi_fn (one C-point state [h, w] -> the next):
    tau_j = (v_j - Psi(v_{j-1})) + r_j for j = 1..N_T; window p covers s = max(0, p - k + 1) .. p and
    starts from w = v_s + r_s, then w = Psi(w) + tau_j for j = s+1..p; e_p = w - v_p.
    states: [N_T+1, h, w] C-point values v_j; r: [N_T+1, h, w] C-point residuals (r_0 = 0)."""
    NT = r.shape[0] - 1
    states = np.asarray(states, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    tau = np.zeros_like(states)
    for j in range(1, NT + 1):
        tau[j] = (states[j] - psi_fn(states[j - 1])) + r[j]
    e_all = np.zeros_like(states)
    for p in range(NT + 1):
        s = max(0, p - k + 1)
        w = states[s] + r[s]
        for j in range(s + 1, p + 1):
            w = psi_fn(w) + tau[j]
        e_all[p] = w - states[p]
    return e_all


def learned_local_solves(vec, states, r, k, bf16_mode=True):
    """The FAS windows above with the learned Psi(x) = x + f(x)."""
    return fas_local_solves(lambda x: psi(vec, x[None], bf16_mode)[0], states, r, k)
