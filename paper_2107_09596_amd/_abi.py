"""ctypes binding of libatmgrit.so (include/atm.h): argument marshalling only.

Every step of the hot path runs in the library's HIP kernels; this module
turns torch tensors into device pointers and the current torch stream into a
hipStream_t.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libatmgrit.so")

ATM_OK = 0
ATM_NOT_CONVERGED = 1
ATM_ERR_INVALID_ARG = -1
ATM_ERR_UNSUPPORTED = -2
ATM_ERR_DEVICE = -3
ATM_ERR_DIVERGED = -4
ATM_ERR_INNER_SOLVE = -5
ATM_ERR_WORKSPACE = -6

ATM_HEAT1D, ATM_HEAT2D, ATM_AC2D = 1, 2, 3


class AtmProblem(ctypes.Structure):
    _fields_ = [
        ("length", ctypes.c_double), ("nu", ctypes.c_double), ("eps", ctypes.c_double),
        ("t0", ctypes.c_double), ("tf", ctypes.c_double), ("cg_rtol", ctypes.c_double),
        ("nt", ctypes.c_int64),
        ("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("cg_max_iter", ctypes.c_int32),
        ("source", ctypes.c_void_p),
    ]


class AtmOptions(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double), ("coarse_cg_rtol", ctypes.c_double), ("mixed_cg_rtol", ctypes.c_double),
        ("fallback_ratio", ctypes.c_double), ("cnn_params", ctypes.c_void_p),
        ("m", ctypes.c_int32), ("k", ctypes.c_int32), ("relax", ctypes.c_int32),
        ("max_iter", ctypes.c_int32), ("coarse_substeps", ctypes.c_int32), ("coarse_form", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("profile", ctypes.c_int32), ("coarse_solver", ctypes.c_int32),
        ("levels", ctypes.c_int32), ("m_coarse", ctypes.c_int32), ("nested", ctypes.c_int32),
    ]


class AtmStats(ctypes.Structure):
    _fields_ = [
        ("final_residual", ctypes.c_double), ("ms_total", ctypes.c_double), ("ms_sweep", ctypes.c_double),
        ("ms_coarse", ctypes.c_double), ("ms_norm", ctypes.c_double),
        ("fine_steps", ctypes.c_int64), ("coarse_steps", ctypes.c_int64), ("cg_fine", ctypes.c_int64),
        ("cg_coarse", ctypes.c_int64), ("fine_steps_skipped", ctypes.c_int64),
        ("iterations", ctypes.c_int32), ("n_sweeps", ctypes.c_int32), ("learned_cycles", ctypes.c_int32),
        ("ms_setup", ctypes.c_double),
    ]


_P = ctypes.POINTER(AtmProblem)
_O = ctypes.POINTER(AtmOptions)
_S = ctypes.POINTER(AtmStats)
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)

# name -> (restype, argtypes); every symbol include/atm.h declares
SIGNATURES = {
    "atm_num_intervals": (ctypes.c_int64, [_P, _O]),
    "atm_window_start": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_int32]),
    "atm_workspace_bytes": (ctypes.c_size_t, [_P, _O]),
    "atm_sweep": (ctypes.c_int32, [_P, _O, ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "atm_coarse_solve": (ctypes.c_int32, [_P, _O, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "atm_coarse_solve_static": (ctypes.c_int32, [_P, _O, _vp, _vp, _vp, _vp]),
    "atm_sweep_kernel": (ctypes.c_char_p, [_P, _O]),
    "atm_coarse_kernel": (ctypes.c_char_p, [_P, _O]),
    "atm_static_scratch_bytes": (ctypes.c_size_t, []),
    "atm_residual_norm": (ctypes.c_int32, [_P, _O, _vp, _vp, _dp, _vp, ctypes.c_size_t, _vp]),
    "atm_implicit_residual_norm": (ctypes.c_int32, [_P, _O, _vp, _dp, _vp, ctypes.c_size_t, _vp]),
    "atm_step_residual_norm": (ctypes.c_int32, [_P, _O, _vp, _dp, _vp, ctypes.c_size_t, _vp]),
    "atm_sequential": (ctypes.c_int32, [_P, _vp, _vp, ctypes.c_size_t, _vp]),
    "atm_sequential_workspace_bytes": (ctypes.c_size_t, [_P]),
    "atm_solve": (ctypes.c_int32, [_P, _O, _vp, _vp, ctypes.c_size_t, _dp, ctypes.c_int32, _S, _vp]),
    "atm_cnn_param_count": (ctypes.c_int32, []),
    "atm_cnn_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "atm_cnn_forward": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                                         ctypes.c_size_t, _vp]),
    "atm_cnn_jvp": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                                     ctypes.c_size_t, _vp]),
    "atm_cnn_gradients": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _ip, _ip, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "atm_cnn_train_step": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_float, _vp, ctypes.c_int32,
                                            _ip, _ip, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                                            ctypes.c_size_t, _vp]),
    "atm_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, _P, _O]),
    "atm_batch_create": (ctypes.c_int32, [ctypes.POINTER(_vp), ctypes.c_int32, _P, _O, ctypes.POINTER(_vp), _vp,
                                          ctypes.c_size_t, ctypes.c_char_p]),
    "atm_batch_run": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32, _ip, _S, _dp, ctypes.c_int32, _dp, _dp,
                                       _vp]),
    "atm_batch_tuning": (ctypes.c_int32, [_vp, _ip, _ip]),
    "atm_batch_destroy": (None, [_vp]),
    "atm_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "atm_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libatmgrit.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2107_09596_amd.build.build() "
                               "(the HIP library is the only implementation of this path)")
        _lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


class AtmError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().atm_last_error().decode()
        name = lib().atm_status_string(status).decode()
        super().__init__(f"{where}: {name} ({status}): {msg}")
        self.status = status


def check(status: int, where: str, allow=(ATM_OK,)) -> int:
    if status not in allow:
        raise AtmError(status, where)
    return status


def problem(p, source=None) -> AtmProblem:
    """AtmProblem from any object with the fields of workloads.Problem; source is an optional device
    tensor holding the PDE source [nt+1, n] FP64 (the caller keeps it alive until the call's work ran)."""
    src = None
    if source is not None:
        import torch
        if not source.is_cuda or source.dtype != torch.float64 or not source.is_contiguous():
            raise ValueError("source must be a contiguous float64 device tensor")
        if tuple(source.shape) != (p.nt + 1, p.nx * p.ny):
            raise ValueError(f"source must have shape {(p.nt + 1, p.nx * p.ny)}, got {tuple(source.shape)}")
        src = source.data_ptr()
    return AtmProblem(length=p.length, nu=p.nu, eps=p.eps, t0=p.t0, tf=p.tf, cg_rtol=p.cg_rtol, nt=p.nt,
                      kind=p.kind, nx=p.nx, ny=p.ny, cg_max_iter=p.cg_max_iter, source=src)


def options(o) -> AtmOptions:
    """AtmOptions from any object with the fields of workloads.Options."""
    cnn = getattr(o, "cnn_params", None)
    if cnn is not None and not isinstance(cnn, int):
        cnn = cnn.data_ptr()  # a device tensor
    return AtmOptions(tol=o.tol, coarse_cg_rtol=float(getattr(o, "coarse_cg_rtol", 0.0)),
                      mixed_cg_rtol=float(getattr(o, "mixed_cg_rtol", 0.0)),
                      fallback_ratio=float(getattr(o, "fallback_ratio", 0.0)), cnn_params=cnn,
                      m=o.m, k=o.k, relax=o.relax,
                      max_iter=o.max_iter, coarse_substeps=o.coarse_substeps, coarse_form=o.coarse_form,
                      precision=getattr(o, "precision", 0), profile=int(getattr(o, "profile", 0)),
                      coarse_solver=int(getattr(o, "coarse_solver", 0)), levels=int(getattr(o, "levels", 2)),
                      m_coarse=int(getattr(o, "m_coarse", 0)), nested=int(getattr(o, "nested", 0)))
