"""Two-level AT-MGRIT (arXiv 2107.09596) on one MI355X: thin Python binding.

The functions below carry the names of the C-ABI in include/atm.h and only
marshal arguments: torch tensors (device memory) become pointers, the current
torch stream becomes the hipStream_t.  All arithmetic of the hot path runs in
the HIP kernels of libatmgrit.so; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes

from . import _abi
from ._abi import (ATM_AC2D, ATM_ERR_DEVICE, ATM_ERR_DIVERGED, ATM_ERR_INNER_SOLVE, ATM_ERR_INVALID_ARG,
                   ATM_ERR_UNSUPPORTED, ATM_ERR_WORKSPACE, ATM_HEAT1D, ATM_HEAT2D, ATM_NOT_CONVERGED, ATM_OK,
                   AtmError)

__all__ = [
    "atm_num_intervals", "atm_window_start", "atm_workspace_bytes", "atm_sweep", "atm_coarse_solve",
    "atm_coarse_solve_static", "atm_static_scratch_bytes", "atm_sweep_kernel", "atm_coarse_kernel",
    "atm_residual_norm", "atm_implicit_residual_norm", "atm_step_residual_norm", "atm_sequential", "atm_sequential_workspace_bytes", "atm_solve", "atm_status_string",
    "atm_last_error", "workspace", "atm_cnn_param_count", "atm_cnn_workspace_bytes", "atm_cnn_forward",
    "atm_cnn_jvp", "atm_cnn_gradients", "atm_cnn_train_step", "Batch", "AtmError", "ATM_OK", "ATM_NOT_CONVERGED", "ATM_ERR_INVALID_ARG",
    "ATM_ERR_UNSUPPORTED", "ATM_ERR_DEVICE", "ATM_ERR_DIVERGED", "ATM_ERR_INNER_SOLVE", "ATM_ERR_WORKSPACE",
    "ATM_HEAT1D", "ATM_HEAT2D", "ATM_AC2D",
]


def _torch():
    import torch
    return torch


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    torch = _torch()
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    del torch
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def atm_num_intervals(prob, opts) -> int:
    return int(_abi.lib().atm_num_intervals(ctypes.byref(_abi.problem(prob)), ctypes.byref(_abi.options(opts))))


def atm_window_start(p: int, k: int) -> int:
    return int(_abi.lib().atm_window_start(int(p), int(k)))


def atm_workspace_bytes(prob, opts) -> int:
    return int(_abi.lib().atm_workspace_bytes(ctypes.byref(_abi.problem(prob)), ctypes.byref(_abi.options(opts))))


def atm_sequential_workspace_bytes(prob) -> int:
    return int(_abi.lib().atm_sequential_workspace_bytes(ctypes.byref(_abi.problem(prob))))


def workspace(nbytes: int, device="cuda"):
    """A zero-filled device byte buffer usable as the workspace (torch allocations are 512-byte aligned)."""
    torch = _torch()
    if nbytes <= 0:
        raise ValueError("workspace size is 0: the problem or options are invalid (see atm_last_error())")
    return torch.zeros(int(nbytes), dtype=torch.uint8, device=device)


def _f64():
    return _torch().float64


def atm_sweep(prob, opts, mode: int, u, aux, y, ws, stream=None, source=None) -> None:
    st = _abi.lib().atm_sweep(ctypes.byref(_abi.problem(prob, source)), ctypes.byref(_abi.options(opts)), int(mode),
                              _ptr(u, _f64(), "u"), _ptr(aux, _f64(), "aux"), _ptr(y, _f64(), "y"),
                              _ptr(ws, None, "ws"), ws.numel() * ws.element_size(), _stream(stream))
    _abi.check(st, "atm_sweep")


def atm_coarse_solve(prob, opts, u, y, e, ws, stream=None) -> None:
    st = _abi.lib().atm_coarse_solve(ctypes.byref(_abi.problem(prob)), ctypes.byref(_abi.options(opts)),
                                     _ptr(u, _f64(), "u"), _ptr(y, _f64(), "y"), _ptr(e, _f64(), "e"),
                                     _ptr(ws, None, "ws"), ws.numel() * ws.element_size(), _stream(stream))
    _abi.check(st, "atm_coarse_solve")


def atm_coarse_solve_static(prob, opts, u, y, e, stream=None) -> None:
    """atm_coarse_solve on the library's static device scratch (no workspace argument)."""
    st = _abi.lib().atm_coarse_solve_static(ctypes.byref(_abi.problem(prob)), ctypes.byref(_abi.options(opts)),
                                            _ptr(u, _f64(), "u"), _ptr(y, _f64(), "y"), _ptr(e, _f64(), "e"),
                                            _stream(stream))
    _abi.check(st, "atm_coarse_solve_static")


def atm_sweep_kernel(prob, opts) -> str:
    """The kernel that runs the relaxation sweeps for these arguments on the current device."""
    return _abi.lib().atm_sweep_kernel(ctypes.byref(_abi.problem(prob)), ctypes.byref(_abi.options(opts))).decode()


def atm_coarse_kernel(prob, opts) -> str:
    """The kernel that runs the local solves (the windows) for these arguments on the current device."""
    return _abi.lib().atm_coarse_kernel(ctypes.byref(_abi.problem(prob)), ctypes.byref(_abi.options(opts))).decode()


def atm_static_scratch_bytes() -> int:
    return int(_abi.lib().atm_static_scratch_bytes())


def atm_residual_norm(prob, opts, u, y, ws, stream=None) -> float:
    out = ctypes.c_double(0.0)
    st = _abi.lib().atm_residual_norm(ctypes.byref(_abi.problem(prob)), ctypes.byref(_abi.options(opts)),
                                      _ptr(u, _f64(), "u"), _ptr(y, _f64(), "y"), ctypes.byref(out),
                                      _ptr(ws, None, "ws"), ws.numel() * ws.element_size(), _stream(stream))
    _abi.check(st, "atm_residual_norm")
    return out.value


def _norm_of_u(fname, prob, opts, u, ws, stream, source=None):
    out = ctypes.c_double(0.0)
    st = getattr(_abi.lib(), fname)(ctypes.byref(_abi.problem(prob, source)), ctypes.byref(_abi.options(opts)),
                                    _ptr(u, _f64(), "u"), ctypes.byref(out), _ptr(ws, None, "ws"),
                                    ws.numel() * ws.element_size(), _stream(stream))
    _abi.check(st, fname)
    return out.value


def atm_implicit_residual_norm(prob, opts, u, ws, stream=None, source=None) -> float:
    return _norm_of_u("atm_implicit_residual_norm", prob, opts, u, ws, stream, source)


def atm_step_residual_norm(prob, opts, u, ws, stream=None, source=None) -> float:
    return _norm_of_u("atm_step_residual_norm", prob, opts, u, ws, stream, source)


def atm_sequential(prob, u, ws=None, stream=None, source=None) -> None:
    if ws is None:
        ws = workspace(atm_sequential_workspace_bytes(prob), device=u.device)
    st = _abi.lib().atm_sequential(ctypes.byref(_abi.problem(prob, source)), _ptr(u, _f64(), "u"), _ptr(ws, None, "ws"),
                                   ws.numel() * ws.element_size(), _stream(stream))
    _abi.check(st, "atm_sequential")


def atm_solve(prob, opts, u, ws=None, hist_cap: int = 256, stream=None, allow=(ATM_OK, ATM_NOT_CONVERGED),
              source=None):
    """Run AT-MGRIT in place on u; returns (status, residual history list, stats dict).
    source: optional PDE source b(x, t_i), device float64 [nt+1, n] (1D heat)."""
    if ws is None:
        ws = workspace(atm_workspace_bytes(prob, opts), device=u.device)
    hist = (ctypes.c_double * max(hist_cap, 1))()
    stats = _abi.AtmStats()
    st = _abi.lib().atm_solve(ctypes.byref(_abi.problem(prob, source)), ctypes.byref(_abi.options(opts)),
                              _ptr(u, _f64(), "u"), _ptr(ws, None, "ws"), ws.numel() * ws.element_size(),
                              hist, int(hist_cap), ctypes.byref(stats), _stream(stream))
    _abi.check(st, "atm_solve", allow=allow)
    sd = {name: getattr(stats, name) for name, _ in _abi.AtmStats._fields_}
    n = min(sd["iterations"] + 1, hist_cap)
    return st, [hist[i] for i in range(n)], sd


def atm_status_string(status: int) -> str:
    return _abi.lib().atm_status_string(int(status)).decode()


def atm_last_error() -> str:
    return _abi.lib().atm_last_error().decode()


# ---------------------------------------------------------------------------
# learned coarse propagator (CNN): marshalling only
# ---------------------------------------------------------------------------

def _f32():
    return _torch().float32


def _int32_host(a):
    import numpy as np
    arr = np.ascontiguousarray(a, dtype=np.int32)
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def atm_cnn_param_count() -> int:
    return int(_abi.lib().atm_cnn_param_count())


def atm_cnn_workspace_bytes(batch: int, h: int, w: int) -> int:
    return int(_abi.lib().atm_cnn_workspace_bytes(int(batch), int(h), int(w)))


def _nbytes(t):
    return t.numel() * t.element_size()


def atm_cnn_forward(params, x, f_out, ws, stream=None) -> None:
    """f_out[b] = f(x[b]); x, f_out: [batch, h, w] float32 device tensors."""
    b, h, w = x.shape
    st = _abi.lib().atm_cnn_forward(_ptr(params, _f32(), "params"), _ptr(x, _f32(), "x"), b, h, w,
                                    _ptr(f_out, _f32(), "f_out"), _ptr(ws, None, "ws"), _nbytes(ws), _stream(stream))
    _abi.check(st, "atm_cnn_forward")


def atm_cnn_jvp(params, v, e, out, ws, stream=None) -> None:
    b, h, w = v.shape
    st = _abi.lib().atm_cnn_jvp(_ptr(params, _f32(), "params"), _ptr(v, _f32(), "v"), _ptr(e, _f32(), "e"), b, h, w,
                                _ptr(out, _f32(), "out"), _ptr(ws, None, "ws"), _nbytes(ws), _stream(stream))
    _abi.check(st, "atm_cnn_jvp")


def atm_cnn_gradients(params, frames, idx_x, idx_y, grad_out, ws, loss_out=None, stream=None) -> None:
    """frames: [n_frames, h, w] float32 device; idx_x, idx_y: host integer sequences of equal length."""
    n, h, w = frames.shape
    ax, px = _int32_host(idx_x)
    ay, py = _int32_host(idx_y)
    if ax.shape != ay.shape:
        raise ValueError("idx_x and idx_y must have the same length")
    st = _abi.lib().atm_cnn_gradients(_ptr(params, _f32(), "params"), _ptr(frames, _f32(), "frames"), n, px, py,
                                      len(ax), h, w, _ptr(grad_out, _f32(), "grad_out"),
                                      _ptr(loss_out, _f32(), "loss_out"), _ptr(ws, None, "ws"), _nbytes(ws),
                                      _stream(stream))
    _abi.check(st, "atm_cnn_gradients")


def atm_cnn_train_step(params, adam_m, adam_v, step: int, lr: float, frames, idx_x, idx_y, ws, loss_out=None,
                       stream=None) -> None:
    n, h, w = frames.shape
    ax, px = _int32_host(idx_x)
    ay, py = _int32_host(idx_y)
    if ax.shape != ay.shape:
        raise ValueError("idx_x and idx_y must have the same length")
    st = _abi.lib().atm_cnn_train_step(_ptr(params, _f32(), "params"), _ptr(adam_m, _f32(), "adam_m"),
                                       _ptr(adam_v, _f32(), "adam_v"), int(step), float(lr),
                                       _ptr(frames, _f32(), "frames"), n, px, py, len(ax), h, w,
                                       _ptr(loss_out, _f32(), "loss_out"), _ptr(ws, None, "ws"), _nbytes(ws),
                                       _stream(stream))
    _abi.check(st, "atm_cnn_train_step")


# ---------------------------------------------------------------------------
# batched solves: marshalling only
# ---------------------------------------------------------------------------

class Batch:
    """A planned batch (atm_batch_create); run() solves every instance in place."""

    def __init__(self, probs, opts, us, tune_cache=None):
        n = len(probs)
        if not (len(opts) == len(us) == n):
            raise ValueError("probs, opts and us must have the same length")
        self.n = n
        self._P = (_abi.AtmProblem * n)(*[_abi.problem(p) for p in probs])
        self._O = (_abi.AtmOptions * n)(*[_abi.options(o) for o in opts])
        self._us = list(us)  # keep the tensors alive
        ptrs = (ctypes.c_void_p * n)(*[_ptr(u, _f64(), "u").value for u in us])
        nbytes = int(_abi.lib().atm_batch_workspace_bytes(n, self._P, self._O))
        if nbytes == 0:
            raise AtmError(ATM_ERR_INVALID_ARG, "atm_batch_workspace_bytes")
        self.ws = workspace(nbytes, device=us[0].device)
        self._h = ctypes.c_void_p(0)
        cache = tune_cache.encode() if tune_cache else None
        st = _abi.lib().atm_batch_create(ctypes.byref(self._h), n, self._P, self._O, ptrs, _ptr(self.ws, None, "ws"),
                                         nbytes, cache)
        _abi.check(st, "atm_batch_create")

    def run(self, use_graph=True, check_every=4, hist_cap=64, stream=None, allow=(ATM_OK, ATM_NOT_CONVERGED)):
        """Returns (overall status, per-instance statuses, stats dicts, histories, ms_solve, ms_tune)."""
        n = self.n
        status = (ctypes.c_int32 * n)()
        stats = (_abi.AtmStats * n)()
        hist = (ctypes.c_double * (n * hist_cap))()
        ms = ctypes.c_double(0.0)
        mt = ctypes.c_double(0.0)
        st = _abi.lib().atm_batch_run(self._h, int(bool(use_graph)), int(check_every), status, stats, hist,
                                      int(hist_cap), ctypes.byref(ms), ctypes.byref(mt), _stream(stream))
        _abi.check(st, "atm_batch_run", allow=allow)
        sts = [{name: getattr(stats[i], name) for name, _ in _abi.AtmStats._fields_} for i in range(n)]
        hs = [[hist[i * hist_cap + j] for j in range(min(sts[i]["iterations"] + 1, hist_cap))] for i in range(n)]
        return st, [status[i] for i in range(n)], sts, hs, ms.value, mt.value

    def tuning(self):
        o, t = ctypes.c_int32(0), ctypes.c_int32(0)
        tuned = _abi.lib().atm_batch_tuning(self._h, ctypes.byref(o), ctypes.byref(t))
        return bool(tuned), o.value, t.value

    def close(self):
        if self._h:
            _abi.lib().atm_batch_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
