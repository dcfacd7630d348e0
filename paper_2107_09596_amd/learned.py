"""Training the learned coarse propagator on the GPU (marshalling only).

The training pairs (u_n, u_{n+lag}) come from trajectories of the library's
own fine propagator (atm_sequential); every optimisation step is one call of
atm_cnn_train_step (forward, back-propagation and Adam in the library's
kernels).  Shuffling orders are inputs: the caller draws them.
"""
from __future__ import annotations

import time

import numpy as np

from . import (atm_cnn_gradients, atm_cnn_train_step, atm_cnn_workspace_bytes, atm_sequential,
               atm_sequential_workspace_bytes, workspace)


def trajectory_frames(prob, fields, stride: int, device="cuda"):
    """Run the fine propagator from each initial field and keep every stride-th state as FP32.

    Returns a [len(fields) * (nt // stride + 1), ny, nx] float32 device tensor,
    trajectory-major.
    """
    import torch
    per = prob.nt // stride + 1
    out = torch.empty((len(fields) * per, prob.ny, prob.nx), dtype=torch.float32, device=device)
    u = torch.zeros((prob.nt + 1, prob.n), dtype=torch.float64, device=device)
    ws = workspace(atm_sequential_workspace_bytes(prob), device=device)
    for i, f in enumerate(fields):
        u.zero_()
        u[0].copy_(torch.as_tensor(np.asarray(f, dtype=np.float64), device=device))
        atm_sequential(prob, u, ws)
        out[i * per:(i + 1) * per].copy_(u[::stride][:per].reshape(per, prob.ny, prob.nx))
    torch.cuda.synchronize()
    return out


def pair_indices(n_traj: int, per_traj: int, lag_frames: int, n_pairs: int):
    """Frame indices (x, y) of the pairs (u_n, u_{n+lag}) trajectory by trajectory, the first n_pairs."""
    xs, ys = [], []
    for t in range(n_traj):
        for i in range(per_traj - lag_frames):
            xs.append(t * per_traj + i)
            ys.append(t * per_traj + i + lag_frames)
    xs, ys = np.asarray(xs[:n_pairs], dtype=np.int32), np.asarray(ys[:n_pairs], dtype=np.int32)
    if len(xs) < n_pairs:
        raise ValueError(f"only {len(xs)} pairs available, {n_pairs} asked for")
    return xs, ys


def mean_loss(params, frames, idx_x, idx_y, batch: int = 64):
    """Mean of the batch losses over the given pairs (one gradient pass per batch)."""
    import torch
    n, h, w = frames.shape
    ws = workspace(atm_cnn_workspace_bytes(batch, h, w), device=frames.device)
    grad = torch.empty(params.numel(), dtype=torch.float32, device=frames.device)
    loss = torch.zeros(1, dtype=torch.float32, device=frames.device)
    total, count = 0.0, 0
    for s in range(0, len(idx_x) - batch + 1, batch):
        atm_cnn_gradients(params, frames, idx_x[s:s + batch], idx_y[s:s + batch], grad, ws, loss_out=loss)
        total += float(loss.item())
        count += 1
    return total / max(count, 1)


def train(params, frames, idx_x, idx_y, orders, batch: int = 64, lr: float = 1e-3, log=None):
    """Adam on the MSE of Psi(u_n) = u_n + f(u_n) against u_{n+lag}.

    params: FP32 device vector (updated in place).  orders: one permutation of
    range(len(idx_x)) per epoch.  Returns (per-epoch mean training loss, seconds).
    """
    import torch
    n, h, w = frames.shape
    dev = frames.device
    ws = workspace(atm_cnn_workspace_bytes(batch, h, w), device=dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    acc = torch.zeros(1, dtype=torch.float64, device=dev)
    step = 0
    history = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for epoch, order in enumerate(orders):
        acc.zero_()
        nb = 0
        for s in range(0, len(order) - batch + 1, batch):
            sel = order[s:s + batch]
            step += 1
            atm_cnn_train_step(params, m, v, step, lr, frames, idx_x[sel], idx_y[sel], ws, loss_out=loss)
            acc += loss
            nb += 1
        history.append(float(acc.item()) / max(nb, 1))
        if log:
            log(f"epoch {epoch + 1}/{len(orders)}: training loss {history[-1]:.4e}")
    torch.cuda.synchronize()
    return history, time.perf_counter() - t0
