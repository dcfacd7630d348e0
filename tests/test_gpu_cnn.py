"""GPU parity of the learned coarse propagator's kernels (through the C-ABI) against the CPU oracle
in bf16 mode (same rounding points, FP64 sums), element by element: the GPU sums in FP32, so a BF16
rounding falls the other way now and then; those flips are counted and bounded (tests/bf16_parity.py)."""
import numpy as np
import pytest

import workloads as W
from oracle import cnn_oracle as CO
from tests.bf16_parity import ULP, elementwise
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def atm():
    import paper_2107_09596_amd as atm
    return atm


def dev32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def params(seed=3):
    v = W.cnn_init(seed, last_scale=1.0).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    P = CO.unpack(v.copy())
    for name in ("b1", "b2", "b3", "b4"):
        P[name][...] = rng.uniform(-0.1, 0.1, size=P[name].shape)
    return CO.pack(P).astype(np.float32)


SHAPES = [(3, 16, 32), (1, 5, 16), (2, 128, 128)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_forward_matches_oracle(atm, shape):
    b, h, w = shape
    pv = params()
    x = np.random.default_rng(1).uniform(-1, 1, size=shape).astype(np.float32)
    ws = atm.workspace(atm.atm_cnn_workspace_bytes(b, h, w))
    out = dev32(np.zeros(shape))
    atm.atm_cnn_forward(dev32(pv), dev32(x), out, ws)
    ref = CO.forward(pv.astype(np.float64), x.astype(np.float64), bf16_mode=True)[0]
    elementwise(host(out), ref, f"forward {shape}")
    # far from the FP64 network only by the BF16 rounding of weights and activations (four layers of
    # sums over up to 288 terms, each rounded input off by at most half an ulp): a few percent of the scale
    ref64 = CO.forward(pv.astype(np.float64), x.astype(np.float64))[0]
    elementwise(host(out), ref64, f"forward {shape} vs FP64 network", tight=ULP, loose=16 * ULP, max_flip_frac=1.0)


@pytest.mark.parametrize("shape", SHAPES[:2], ids=lambda s: "x".join(map(str, s)))
def test_jvp_matches_oracle(atm, shape):
    b, h, w = shape
    pv = params(4)
    rng = np.random.default_rng(2)
    v = rng.uniform(-1, 1, size=shape).astype(np.float32)
    e = (1e-6 * rng.standard_normal(shape)).astype(np.float32)   # a small correction: scale-free
    ws = atm.workspace(atm.atm_cnn_workspace_bytes(b, h, w))
    out = dev32(np.zeros(shape))
    atm.atm_cnn_jvp(dev32(pv), dev32(v), dev32(e), out, ws)
    ref = CO.jvp(pv.astype(np.float64), v.astype(np.float64), e.astype(np.float64), bf16_mode=True)
    got = host(out)
    elementwise(got - e, ref - e, f"jvp {shape}")
    # linear in e: doubling e doubles the product (up to the BF16 rounding of e's signals)
    out2 = dev32(np.zeros(shape))
    atm.atm_cnn_jvp(dev32(pv), dev32(v), dev32(2 * e), out2, ws)
    # (a power-of-two scaling commutes with every rounding, so the products agree far below the ulp)
    elementwise(host(out2) - 2 * e, 2 * (got - e), f"jvp linearity {shape}", tight=1e-6, loose=1e-6, max_flip_frac=0.0,
                footprint=0)


@pytest.mark.parametrize("shape", [(4, 16, 32), (2, 128, 128)], ids=lambda s: "x".join(map(str, s)))
def test_gradients_match_oracle(atm, shape):
    b, h, w = shape
    pv = params(5)
    rng = np.random.default_rng(3)
    frames = rng.uniform(-1, 1, size=(b + 3, h, w)).astype(np.float32)
    idx_x = [0, 2, 4, 1][:b]
    idx_y = [3, 1, 0, 4][:b]
    ws = atm.workspace(atm.atm_cnn_workspace_bytes(b, h, w))
    grad = dev32(np.zeros(CO.N_PARAMS))
    loss = dev32(np.zeros(1))
    atm.atm_cnn_gradients(dev32(pv), dev32(frames), idx_x, idx_y, grad, ws, loss_out=loss)
    ref_loss, ref_g = CO.loss_and_grad(pv.astype(np.float64), frames[idx_x].astype(np.float64),
                                       frames[idx_y].astype(np.float64), bf16_mode=True)
    assert abs(host(loss)[0] - ref_loss) <= 1e-5 * ref_loss
    g = host(grad)
    P, R = CO.unpack(g), CO.unpack(ref_g)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"):
        elementwise(P[name], R[name], f"gradient {name} {shape}")


def test_train_step_is_adam_on_the_gradient(atm):
    b, h, w = 4, 16, 32
    pv = params(6)
    frames = np.random.default_rng(4).uniform(-1, 1, size=(6, h, w)).astype(np.float32)
    idx_x, idx_y = [0, 1, 2, 3], [4, 5, 1, 0]
    ws = atm.workspace(atm.atm_cnn_workspace_bytes(b, h, w))
    grad = dev32(np.zeros(CO.N_PARAMS))
    atm.atm_cnn_gradients(dev32(pv), dev32(frames), idx_x, idx_y, grad, ws)
    g = host(grad)
    p = dev32(pv)
    m = dev32(np.zeros(CO.N_PARAMS))
    v = dev32(np.zeros(CO.N_PARAMS))
    loss = dev32(np.zeros(1))
    atm.atm_cnn_train_step(p, m, v, 1, 1e-3, dev32(frames), idx_x, idx_y, ws, loss_out=loss)
    ref, rm, rv = CO.adam(pv.astype(np.float64), g, np.zeros(CO.N_PARAMS), np.zeros(CO.N_PARAMS), 1, lr=1e-3)
    np.testing.assert_allclose(host(p), ref, rtol=0, atol=2e-6)
    np.testing.assert_allclose(host(m), rm, rtol=1e-5, atol=1e-12)


def test_training_lowers_the_loss(atm):
    """A few Adam steps on a fixed batch of smooth fields reduce the loss."""
    b, h, w = 8, 16, 32
    rng = np.random.default_rng(7)
    yy, xx = np.meshgrid(np.arange(h) / h, np.arange(w) / w, indexing="ij")
    frames = np.stack([np.sin(2 * np.pi * (k % 3 + 1) * xx + k) * np.cos(2 * np.pi * yy) for k in range(16)])
    frames = frames.astype(np.float32)
    idx_x = list(range(8))
    idx_y = list(range(8, 16))
    ws = atm.workspace(atm.atm_cnn_workspace_bytes(b, h, w))
    p = dev32(W.cnn_init(11))
    m = dev32(np.zeros(CO.N_PARAMS))
    v = dev32(np.zeros(CO.N_PARAMS))
    loss = dev32(np.zeros(1))
    losses = []
    for step in range(1, 41):
        atm.atm_cnn_train_step(p, m, v, step, 3e-3, dev32(frames), idx_x, idx_y, ws, loss_out=loss)
        losses.append(host(loss)[0])
    assert losses[-1] < 0.5 * losses[0], losses[::8]
    del rng


def test_cnn_error_paths(atm):
    assert atm.atm_cnn_workspace_bytes(2, 16, 24) == 0
    ws = atm.workspace(atm.atm_cnn_workspace_bytes(2, 16, 32))
    with pytest.raises(atm.AtmError) as ei:
        atm.atm_cnn_forward(dev32(params()), dev32(np.zeros((2, 16, 24))), dev32(np.zeros((2, 16, 24))), ws)
    assert ei.value.status == atm.ATM_ERR_UNSUPPORTED
    frames = dev32(np.zeros((3, 16, 32)))
    with pytest.raises(atm.AtmError) as ei:
        atm.atm_cnn_gradients(dev32(params()), frames, [0, 3], [1, 2], dev32(np.zeros(CO.N_PARAMS)), ws)
    assert ei.value.status == atm.ATM_ERR_INVALID_ARG
