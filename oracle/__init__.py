"""CPU oracle for two-level AT-MGRIT -- TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 implementation (``atm_oracle.c``, plain C loops) of what
the GPU hot path computes, used to check it.  Only ``tests/``, the smoke check
and the CPU-baseline leg of ``bench.py`` may import this package.  It shares
no code with the HIP library and never loads it.

See ``atm_oracle.c`` for the passage of the paper each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "atm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, INVALID, DIVERGED, INNER = 0, 1, -1, -4, -5


class OrProblem(ctypes.Structure):
    _fields_ = [
        ("length", ctypes.c_double), ("nu", ctypes.c_double), ("eps", ctypes.c_double),
        ("t0", ctypes.c_double), ("tf", ctypes.c_double), ("cg_rtol", ctypes.c_double),
        ("nt", ctypes.c_int64),
        ("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("cg_max_iter", ctypes.c_int32),
        ("src", ctypes.POINTER(ctypes.c_double)),
    ]


class OrOptions(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double), ("coarse_cg_rtol", ctypes.c_double),
        ("m", ctypes.c_int32), ("k", ctypes.c_int32), ("relax", ctypes.c_int32),
        ("max_iter", ctypes.c_int32), ("coarse_substeps", ctypes.c_int32), ("coarse_form", ctypes.c_int32),
    ]


OR_MAX_LEVELS = 4


class OrMlOptions(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double), ("coarse_cg_rtol", ctypes.c_double),
        ("levels", ctypes.c_int32), ("m", ctypes.c_int32 * (OR_MAX_LEVELS - 1)),
        ("k", ctypes.c_int32), ("relax", ctypes.c_int32), ("max_iter", ctypes.c_int32),
        ("coarse_substeps", ctypes.c_int32), ("nested", ctypes.c_int32),
    ]


class OrStats(ctypes.Structure):
    _fields_ = [
        ("final_residual", ctypes.c_double),
        ("fine_steps", ctypes.c_int64), ("coarse_steps", ctypes.c_int64), ("cg_iters", ctypes.c_int64),
        ("iterations", ctypes.c_int32), ("status", ctypes.c_int32),
    ]


# Builds of the same source: "default" (the tests' build) and "native" (-O3 for the host it runs on,
# used only to time the oracle as the CPU baseline).  Both keep -ffp-contract=off, so the arithmetic
# is the same.
_BUILDS = {
    "default": (_LIB, ["-O2"]),
    "native": (os.path.join(_HERE, "liboracle_native.so"), ["-O3", "-march=native"]),
}
_variant = "default"


def build(force: bool = False, variant: str = "default") -> str:
    """Compile the oracle with gcc (plain C, OpenMP for the interval/window loops)."""
    path, opt = _BUILDS[variant]
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp"
        subprocess.check_call(["gcc", *opt, "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)
    return path


def select_build(variant: str) -> None:
    """Load the given build for the calls below (the CPU-baseline timing uses "native")."""
    global _lib, _variant
    if variant not in _BUILDS:
        raise KeyError(variant)
    if variant != _variant:
        _variant = variant
        _lib = None


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build(variant=_variant))
        P, O, S = ctypes.POINTER(OrProblem), ctypes.POINTER(OrOptions), ctypes.POINTER(OrStats)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        sig = {
            "or_step": (ctypes.c_int, [P, ctypes.c_double, dp, dp, i64p]),
            "or_coarse_step": (ctypes.c_int, [P, O, dp, dp, i64p]),
            "or_sequential": (ctypes.c_int, [P, dp, i64p]),
            "or_f_relax": (ctypes.c_int, [P, O, dp, i64p]),
            "or_c_relax": (ctypes.c_int, [P, O, dp, i64p]),
            "or_residual": (ctypes.c_int, [P, dp, dp, dp, i64p]),
            "or_norm2": (ctypes.c_double, [ctypes.c_int64, dp]),
            "or_implicit_residual": (ctypes.c_int, [P, dp, dp]),
            "or_step_residual": (ctypes.c_int, [P, dp, dp, i64p]),
            "or_local_solve": (ctypes.c_int, [P, O, ctypes.c_int64, dp, dp, dp, i64p]),
            "or_local_solves": (ctypes.c_int, [P, O, dp, dp, dp, i64p, i64p]),
            "or_correct": (ctypes.c_int, [P, O, dp, dp, i64p]),
            "or_cycle": (ctypes.c_int, [P, O, dp, dp, S]),
            "or_parareal_cycle": (ctypes.c_int, [P, O, dp, dp, S]),
            "or_atmgrit_solve": (ctypes.c_int, [P, O, dp, dp, ctypes.c_int32, S]),
            "or_parareal_solve": (ctypes.c_int, [P, O, dp, dp, ctypes.c_int32, S]),
            "or_num_intervals": (ctypes.c_int64, [P, O]),
            "or_window_start": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_int32]),
            "or_ml_cycle": (ctypes.c_int, [P, ctypes.POINTER(OrMlOptions), dp, dp, i64p]),
            "or_ml_solve": (ctypes.c_int, [P, ctypes.POINTER(OrMlOptions), dp, dp, ctypes.c_int32, S]),
            "or_ml_nested": (ctypes.c_int, [P, ctypes.POINTER(OrMlOptions), dp, i64p]),
            "or_set_threads": (None, [ctypes.c_int]),
            "or_get_max_threads": (ctypes.c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _prob(p, source=None) -> OrProblem:
    """The C problem; source is the PDE forcing b(x, t_i), float64 [nt+1, n] (the caller keeps it alive)."""
    src = None
    if source is not None:
        assert source.shape == (p.nt + 1, p.n)
        src = _ptr(source)
    return OrProblem(length=p.length, nu=p.nu, eps=p.eps, t0=p.t0, tf=p.tf, cg_rtol=p.cg_rtol, nt=p.nt,
                     kind=p.kind, nx=p.nx, ny=p.ny, cg_max_iter=p.cg_max_iter, src=src)


def _src(source):
    return None if source is None else np.ascontiguousarray(source, dtype=np.float64)


def _opts(o) -> OrOptions:
    return OrOptions(tol=o.tol, coarse_cg_rtol=getattr(o, "coarse_cg_rtol", 0.0), m=o.m, k=o.k, relax=o.relax,
                     max_iter=o.max_iter,
                     coarse_substeps=o.coarse_substeps, coarse_form=o.coarse_form)


def _ml_opts(o) -> OrMlOptions:
    """Multilevel options: o.levels levels with factors o.m (level 0 -> 1) and o.m_coarse (between
    the coarser levels), k, relax, tol, max_iter, coarse_substeps and coarse_cg_rtol as for two levels."""
    ms = (ctypes.c_int32 * (OR_MAX_LEVELS - 1))(*([o.m] + [o.m_coarse] * (OR_MAX_LEVELS - 2)))
    return OrMlOptions(tol=o.tol, coarse_cg_rtol=getattr(o, "coarse_cg_rtol", 0.0), levels=o.levels, m=ms, k=o.k,
                       relax=o.relax, max_iter=o.max_iter, coarse_substeps=o.coarse_substeps,
                       nested=int(getattr(o, "nested", 0)))


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"oracle {what} returned status {status}")
        self.status = status


def _check(st, what):
    if st != OK:
        raise OracleError(st, what)


def set_threads(t: int):
    lib().or_set_threads(int(t))


def max_threads() -> int:
    """OpenMP's thread count for this process (OMP_NUM_THREADS, else the host's cores)."""
    return int(lib().or_get_max_threads())


def step(p, dt, x):
    """One integrator step of size dt (Phi at the fine dt)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    cg = ctypes.c_int64(0)
    _check(lib().or_step(ctypes.byref(_prob(p)), dt, _ptr(x), _ptr(out), ctypes.byref(cg)), "step")
    return out


def coarse_step(p, o, x):
    """Psi: coarse_substeps steps of size m dt / coarse_substeps."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    cg = ctypes.c_int64(0)
    _check(lib().or_coarse_step(ctypes.byref(_prob(p)), ctypes.byref(_opts(o)), _ptr(x), _ptr(out),
                                ctypes.byref(cg)), "coarse_step")
    return out


def sequential(p, u0, source=None):
    """Sequential time stepping u_i = Phi(u_{i-1}) + g_i; returns [nt+1, n]."""
    src = _src(source)
    u = np.zeros((p.nt + 1, p.n), dtype=np.float64)
    u[0] = u0
    cg = ctypes.c_int64(0)
    _check(lib().or_sequential(ctypes.byref(_prob(p, src)), _ptr(u), ctypes.byref(cg)), "sequential")
    return u


def f_relax(p, o, u, source=None):
    """F-relaxation of every interval: each F-point is Phi of the point before it."""
    src = _src(source)
    u = np.array(u, dtype=np.float64, order="C")
    _check(lib().or_f_relax(ctypes.byref(_prob(p, src)), ctypes.byref(_opts(o)), _ptr(u), None), "f_relax")
    return u


def c_relax(p, o, u, source=None):
    src = _src(source)
    u = np.array(u, dtype=np.float64, order="C")
    _check(lib().or_c_relax(ctypes.byref(_prob(p, src)), ctypes.byref(_opts(o)), _ptr(u), None), "c_relax")
    return u


def residual(p, u, g0, source=None):
    """Full space-time residual g - A(u), [nt+1, n]."""
    src = _src(source)
    u = np.ascontiguousarray(u, dtype=np.float64)
    g0 = np.ascontiguousarray(g0, dtype=np.float64)
    r = np.empty_like(u)
    _check(lib().or_residual(ctypes.byref(_prob(p, src)), _ptr(u), _ptr(g0), _ptr(r), None), "residual")
    return r


def residual_norm(p, u, g0, source=None):
    return float(np.sqrt(np.sum(residual(p, u, g0, source) ** 2)))


def implicit_residual(p, u, source=None):
    """rho_i = psi(u_{i-1}) + dt b(t_i) - M u_i, [nt+1, n] (row 0 is zero; b only with a source)."""
    src = _src(source)
    u = np.ascontiguousarray(u, dtype=np.float64)
    rho = np.empty_like(u)
    _check(lib().or_implicit_residual(ctypes.byref(_prob(p, src)), _ptr(u), _ptr(rho)), "implicit_residual")
    return rho


def step_residual(p, u, source=None):
    """r_i = M^{-1} rho_i (the residual with the step solved from zero), [nt+1, n]."""
    src = _src(source)
    u = np.ascontiguousarray(u, dtype=np.float64)
    r = np.empty_like(u)
    _check(lib().or_step_residual(ctypes.byref(_prob(p, src)), _ptr(u), _ptr(r), None), "step_residual")
    return r


def local_solve(p, o, pidx, rc, vc):
    rc = np.ascontiguousarray(rc, dtype=np.float64)
    vc = np.ascontiguousarray(vc, dtype=np.float64)
    e = np.empty(p.n, dtype=np.float64)
    _check(lib().or_local_solve(ctypes.byref(_prob(p)), ctypes.byref(_opts(o)), int(pidx), _ptr(rc), _ptr(vc),
                                _ptr(e), None), "local_solve")
    return e


def local_solves(p, o, rc, vc):
    rc = np.ascontiguousarray(rc, dtype=np.float64)
    vc = np.ascontiguousarray(vc, dtype=np.float64)
    e = np.empty_like(rc)
    _check(lib().or_local_solves(ctypes.byref(_prob(p)), ctypes.byref(_opts(o)), _ptr(rc), _ptr(vc), _ptr(e),
                                 None, None), "local_solves")
    return e


def correct(p, o, u, e, source=None):
    src = _src(source)
    u = np.array(u, dtype=np.float64, order="C")
    e = np.ascontiguousarray(e, dtype=np.float64)
    _check(lib().or_correct(ctypes.byref(_prob(p, src)), ctypes.byref(_opts(o)), _ptr(u), _ptr(e), None), "correct")
    return u


def cycle(p, o, u, g0=None, parareal=False, source=None):
    """One AT-MGRIT (or Parareal) cycle of Alg. 1 applied to a copy of u."""
    src = _src(source)
    u = np.array(u, dtype=np.float64, order="C")
    g0 = np.ascontiguousarray(u[0] if g0 is None else g0, dtype=np.float64)
    st = OrStats()
    f = lib().or_parareal_cycle if parareal else lib().or_cycle
    _check(f(ctypes.byref(_prob(p, src)), ctypes.byref(_opts(o)), _ptr(u), _ptr(g0), ctypes.byref(st)), "cycle")
    return u


def solve(p, o, u, parareal=False, hist_cap=1000, allow_status=(OK,), source=None):
    """AT-MGRIT (or Parareal) until tol; returns (u, hist, stats dict)."""
    src = _src(source)
    u = np.array(u, dtype=np.float64, order="C")
    hist = np.zeros(hist_cap, dtype=np.float64)
    st = OrStats()
    f = lib().or_parareal_solve if parareal else lib().or_atmgrit_solve
    status = f(ctypes.byref(_prob(p, src)), ctypes.byref(_opts(o)), _ptr(u), _ptr(hist), hist_cap, ctypes.byref(st))
    if status not in allow_status:
        raise OracleError(status, "solve")
    stats = {name: getattr(st, name) for name, _ in OrStats._fields_}
    return u, hist[: st.iterations + 1].copy(), stats


def num_intervals(p, o) -> int:
    return p.nt // o.m


def window_start(pidx: int, k: int) -> int:
    return int(lib().or_window_start(int(pidx), int(k)))


def ml_cycle(p, o, u, g0=None, source=None):
    """One multilevel FAS V-cycle of Alg. 2 applied to a copy of u."""
    src = _src(source)
    u = np.array(u, dtype=np.float64, order="C")
    g0 = np.ascontiguousarray(u[0] if g0 is None else g0, dtype=np.float64)
    _check(lib().or_ml_cycle(ctypes.byref(_prob(p, src)), ctypes.byref(_ml_opts(o)), _ptr(u), _ptr(g0), None),
           "ml_cycle")
    return u


def ml_solve(p, o, u, hist_cap=1000, allow_status=(OK,), source=None):
    """Multilevel FAS AT-MGRIT (Alg. 2) until tol; returns (u, hist, stats dict)."""
    src = _src(source)
    u = np.array(u, dtype=np.float64, order="C")
    hist = np.zeros(hist_cap, dtype=np.float64)
    st = OrStats()
    status = lib().or_ml_solve(ctypes.byref(_prob(p, src)), ctypes.byref(_ml_opts(o)), _ptr(u), _ptr(hist), hist_cap,
                               ctypes.byref(st))
    if status not in allow_status:
        raise OracleError(status, "ml_solve")
    stats = {name: getattr(st, name) for name, _ in OrStats._fields_}
    return u, hist[: st.iterations + 1].copy(), stats


def ml_nested(p, o, u):
    """The nested-iteration initial guess (o.levels levels) built from a copy of u (u[0] = g_0)."""
    u = np.array(u, dtype=np.float64, order="C")
    _check(lib().or_ml_nested(ctypes.byref(_prob(p)), ctypes.byref(_ml_opts(o)), _ptr(u), None), "ml_nested")
    return u
