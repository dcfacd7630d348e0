"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only draws random numbers and evaluates initial fields; it holds
none of the method's arithmetic (no time stepping, no residuals, no coarse
solves).  Every array is float64, row-major, shaped ``[n]`` for one time
slice (``n = nx * ny``, index ``y * nx + x``) or ``[nt + 1, n]`` for a
space-time iterate.

Problem kinds (the integrator of the one-step form u_i = Phi(u_{i-1}) + g_i of
section 2, eq. (2); g_0 = u0, and g_i = 0 for i >= 1 except in the manufactured
1D heat problem, whose PDE source enters each backward Euler step at its new
time level):

* ``HEAT1D`` -- u_t = nu u_xx on [0, L], zero Dirichlet, nx interior points,
  h = L / (nx + 1), backward Euler.
* ``HEAT2D`` -- u_t = nu (u_xx + u_yy) on [0, L]^2, zero Dirichlet, nx * ny
  interior points, 5-point stencil, backward Euler solved by Jacobi-PCG.
* ``AC2D``   -- u_t = nu Lap(u) + (u - u^3) / eps^2 on the periodic square
  [0, L)^2, h = L / nx, IMEX step (implicit diffusion by CG, explicit cubic).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

HEAT1D = 1
HEAT2D = 2
AC2D = 3

KIND_NAMES = {HEAT1D: "heat1d", HEAT2D: "heat2d", AC2D: "ac2d"}


@dataclasses.dataclass
class Problem:
    """Statement of the discrete initial value problem (section 2)."""

    kind: int
    nx: int
    ny: int = 1
    length: float = 1.0
    nu: float = 1.0
    eps: float = 1.0
    t0: float = 0.0
    tf: float = 1.0
    nt: int = 16
    cg_rtol: float = 1e-12
    cg_max_iter: int = 1000

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @property
    def dt(self) -> float:
        return (self.tf - self.t0) / self.nt


@dataclasses.dataclass
class Options:
    """Two-level AT-MGRIT parameters (section 2.1, Alg. 1)."""

    m: int = 2
    k: int = 2
    relax: int = 1          # 0 = F-relaxation, 1 = FCF-relaxation
    tol: float = 1e-8       # absolute 2-norm of the space-time residual
    max_iter: int = 100
    coarse_substeps: int = 1
    coarse_form: int = 0    # 0 auto (linear for heat, FAS for Allen-Cahn), 1 linear, 2 FAS, 3 learned
    precision: int = 0      # 0 FP64 throughout, 1 FP32 fine sweeps + FP64 residual/correction
    profile: int = 0        # 1: the GPU solve times every kernel launch with HIP events
    coarse_solver: int = 0  # Psi's implicit solve: 0 auto (FP64 eigenbasis where built), 1 CG, 2 BF16 eigenbasis
    levels: int = 2         # 2: two-level AT-MGRIT (Alg. 1); 3: the FAS V-cycle of Alg. 2 over three levels
    m_coarse: int = 0       # levels 3: coarsening factor between level 1 and the coarsest level 2
    nested: int = 0         # 1: start from the nested-iteration guess built from the coarse levels
    coarse_cg_rtol: float = 0.0  # CG tolerance inside Psi; 0 = the problem's cg_rtol
    mixed_cg_rtol: float = 0.0   # precision 1: FP32 CG tolerance of the fine correction solves; 0 = 1e-6
    fallback_ratio: float = 0.0  # coarse_form 3: stagnation ratio that switches to the plain Psi; 0 = 0.95
    cnn_params: object = None    # coarse_form 3: device tensor of the learned propagator's parameters

    def n_intervals(self, nt: int) -> int:
        return nt // self.m


def default_k(n_intervals: int) -> int:
    """k = max(2, ceil(0.1 (N_T + 1))), the 10 % rule of the heat k-study (section 4.3)."""
    return max(2, math.ceil(0.1 * (n_intervals + 1)))


# ---------------------------------------------------------------------------
# initial fields
# ---------------------------------------------------------------------------

def heat1d_u0(nx: int, seed: int, length: float = 1.0, modes=range(2, 9), sigma: float = 0.1):
    """sin(pi x / L) plus seeded N(0, sigma^2) amplitudes on the given sine modes."""
    rng = np.random.default_rng(seed)
    h = length / (nx + 1)
    x = h * np.arange(1, nx + 1)
    u = np.sin(np.pi * x / length)
    amps = rng.normal(0.0, sigma, size=len(list(modes)))
    for a, j in zip(amps, modes):
        u = u + a * np.sin(j * np.pi * x / length)
    return np.ascontiguousarray(u, dtype=np.float64), dict(zip(list(modes), amps))


def heat2d_u0(nx: int, ny: int, seed: int, length: float = 1.0, n_modes: int = 16, max_mode: int = 16):
    """Sum of n_modes sine modes sin(j pi x) sin(l pi y), (j, l) i.i.d. U{1..max_mode}, amplitudes N(0, 1)."""
    rng = np.random.default_rng(seed)
    hx = length / (nx + 1)
    hy = length / (ny + 1)
    x = hx * np.arange(1, nx + 1)
    y = hy * np.arange(1, ny + 1)
    js = rng.integers(1, max_mode + 1, size=n_modes)
    ls = rng.integers(1, max_mode + 1, size=n_modes)
    amps = rng.normal(0.0, 1.0, size=n_modes)
    u = np.zeros((ny, nx))
    for a, j, l in zip(amps, js, ls):
        u += a * np.outer(np.sin(l * np.pi * y / length), np.sin(j * np.pi * x / length))
    return np.ascontiguousarray(u.reshape(-1), dtype=np.float64), list(zip(js.tolist(), ls.tolist(), amps.tolist()))


def ac2d_u0(nx: int, ny: int, seed: int, amp: float = 0.05):
    """i.i.d. U[-amp, amp] field on the periodic grid."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-amp, amp, size=nx * ny), dtype=np.float64)


def initial_guess(prob: Problem, u0: np.ndarray, kind: str = "zero", seed: int = 0):
    """Space-time iterate [nt+1, n] with u[0] = g_0 = u0 and the guess at t > 0.

    kind = "zero": zeros at t > 0.  kind = "random": i.i.d. U[-1, 1] at t > 0
    (the heat study of section 4.3 uses a random guess so that no knowledge of
    the right-hand side enters).
    """
    u = np.zeros((prob.nt + 1, prob.n), dtype=np.float64)
    u[0] = u0
    if kind == "random":
        rng = np.random.default_rng(seed)
        u[1:] = rng.uniform(-1.0, 1.0, size=(prob.nt, prob.n))
    elif kind != "zero":
        raise ValueError(kind)
    return u


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def config(name: str):
    """Return (Problem, Options, u0) for a named workload.

    c1  1D heat, nx=63, Nt=1024 on [0,1], m=16, FCF, FP64.
    c2  2D heat nu=0.1, 128x128 interior, Nt=4096 on [0,1], m=32, CG rtol 1e-12.
    c3  2D Allen-Cahn eps=0.02, periodic 256x256, dt=1e-5, Nt=8192, m=64, 4 coarse substeps.
    c5  2D Allen-Cahn eps=0.03, periodic 128x128, dt=1e-5, Nt=4096, m=32.
    """
    if name == "c1":
        p = Problem(HEAT1D, nx=63, ny=1, length=1.0, nu=1.0, t0=0.0, tf=1.0, nt=1024)
        o = Options(m=16, k=default_k(1024 // 16), relax=1, tol=1e-8)
        u0, _ = heat1d_u0(63, seed=1)
    elif name == "c2":
        p = Problem(HEAT2D, nx=128, ny=128, length=1.0, nu=0.1, t0=0.0, tf=1.0, nt=4096, cg_rtol=1e-12)
        o = Options(m=32, k=default_k(4096 // 32), relax=1, tol=1e-8)
        u0, _ = heat2d_u0(128, 128, seed=2)
    elif name == "c3":
        p = Problem(AC2D, nx=256, ny=256, length=1.0, nu=1.0, eps=0.02, t0=0.0, tf=8192 * 1e-5, nt=8192,
                    cg_rtol=1e-12)
        o = Options(m=64, k=default_k(8192 // 64), relax=1, tol=1e-8, coarse_substeps=4, precision=1)
        u0 = ac2d_u0(256, 256, seed=3)
    elif name == "c5":
        p = Problem(AC2D, nx=128, ny=128, length=1.0, nu=1.0, eps=0.03, t0=0.0, tf=4096 * 1e-5, nt=4096,
                    cg_rtol=1e-12)
        o = Options(m=32, k=default_k(4096 // 32), relax=1, tol=1e-8, coarse_substeps=1, precision=1)
        u0 = ac2d_u0(128, 128, seed=7)
    else:
        raise KeyError(name)
    return p, o, u0


def heat1d_forced(nx: int = 1023, nt: int = 16383, guess_seed: int = 8):
    """The manufactured 1D heat problem of the k-study (section 4.3).

    u_t - u_xx = b on x in [0, 3], t in [0, pi], zero Dirichlet ends,
    u(x, 0) = sin(pi x), b(x, t) = -sin(pi x) (sin t - pi^2 cos t), so that
    u = sin(pi x) cos t solves the PDE.  Defaults: 1025 grid points including
    both ends (nx = 1023 unknowns, h = 3/1024) and 16384 time points
    (nt = 16383 steps).  The guess at t > 0 is i.i.d. U[-1, 1] from
    default_rng(guess_seed).  Returns (Problem, u0, source [nt+1, n], u_guess [nt+1, n]).
    The source is the forcing evaluated at every grid point and time point.
    """
    p = Problem(HEAT1D, nx=nx, ny=1, length=3.0, nu=1.0, t0=0.0, tf=math.pi, nt=nt)
    x = (p.length / (nx + 1)) * np.arange(1, nx + 1)
    t = p.t0 + p.dt * np.arange(nt + 1)
    sx = np.sin(np.pi * x)
    source = np.ascontiguousarray(-np.outer(np.sin(t) - np.pi ** 2 * np.cos(t), sx), dtype=np.float64)
    u0 = np.ascontiguousarray(sx, dtype=np.float64)
    return p, u0, source, initial_guess(p, u0, "random", seed=guess_seed)


def heat1d_forced_exact(p: Problem):
    """The PDE solution sin(pi x) cos t of the manufactured problem at every grid and time point, [nt+1, n]."""
    x = (p.length / (p.nx + 1)) * np.arange(1, p.nx + 1)
    t = p.t0 + p.dt * np.arange(p.nt + 1)
    return np.outer(np.cos(t), np.sin(np.pi * x))


def k_study_options(m: int, k: int, tol: float = 1e-7, max_iter: int = 200):
    """Two-level AT-MGRIT options of the k-study: F-relaxation, linear coarse problem, tol 1e-7."""
    return Options(m=m, k=k, relax=0, tol=tol, max_iter=max_iter, coarse_form=1)


def three_level_config(m_coarse: int, k: int = None, relax: int = 1):
    """The three-level workload: 2D heat as in c2 (128 x 128 interior, nu 0.1, dt 1/4096, CG rtol
    1e-12, seed-2 initial field) over 16384 steps (t in [0, 4]), m = 64 so that level 1 has 256
    points, m_coarse from level 1 to the coarsest level, k = N_2 / 2 by default (half the coarsest
    points, the choice of section 5 for its three-level runs), FCF, tol 1e-8.
    Returns (Problem, Options, u0)."""
    p = Problem(HEAT2D, nx=128, ny=128, length=1.0, nu=0.1, t0=0.0, tf=4.0, nt=16384, cg_rtol=1e-12)
    n2 = (16384 // 64) // m_coarse
    o = Options(m=64, k=max(1, n2 // 2) if k is None else k, relax=relax, tol=1e-8, levels=3, m_coarse=m_coarse)
    u0, _ = heat2d_u0(128, 128, seed=2)
    return p, o, u0


def small_problem(kind: int, seed: int = 0, nt: int = 48, nx: int = 7, ny: int = None, **kw):
    """A tiny problem of the given kind with seeded initial data, for oracle pins and parity."""
    if kind == HEAT1D:
        p = Problem(HEAT1D, nx=nx, ny=1, nu=kw.pop("nu", 1.0), tf=kw.pop("tf", 0.5), nt=nt, **kw)
        u0, _ = heat1d_u0(nx, seed=seed)
    elif kind == HEAT2D:
        ny = nx if ny is None else ny
        p = Problem(HEAT2D, nx=nx, ny=ny, nu=kw.pop("nu", 0.1), tf=kw.pop("tf", 0.5), nt=nt, **kw)
        u0, _ = heat2d_u0(nx, ny, seed=seed, n_modes=4, max_mode=min(nx, ny, 4))
    elif kind == AC2D:
        ny = nx if ny is None else ny
        p = Problem(AC2D, nx=nx, ny=ny, nu=1.0, eps=kw.pop("eps", 0.1), tf=kw.pop("tf", nt * 1e-3), nt=nt, **kw)
        rng = np.random.default_rng(seed)
        u0 = np.ascontiguousarray(rng.uniform(-0.5, 0.5, size=nx * ny))
    else:
        raise KeyError(kind)
    return p, u0


# ---------------------------------------------------------------------------
# learned coarse propagator: seeded initial weights and training-data recipe
# ---------------------------------------------------------------------------

CNN_CHANNELS = 32
# flat parameter layout: W1[9][32] (tap, out), b1[32], W2[9][32][32] (tap, out, in), b2[32],
# W3[9][32][32], b3[32], W4[9][32] (tap, in), b4[1]
CNN_SIZES = [(9 * 32, 9), (32, 0), (9 * 32 * 32, 9 * 32), (32, 0), (9 * 32 * 32, 9 * 32), (32, 0), (9 * 32, 9 * 32),
             (1, 0)]
CNN_N_PARAMS = sum(n for n, _ in CNN_SIZES)


def cnn_init(seed: int, last_scale: float = 0.1) -> np.ndarray:
    """He-normal initial weights (std sqrt(2 / fan_in)), zero biases, as one float32 vector.

    The last layer is scaled by last_scale so that Psi = u + f(u) starts close
    to the identity.
    """
    rng = np.random.default_rng(seed)
    parts = []
    for i, (n, fan_in) in enumerate(CNN_SIZES):
        if fan_in == 0:
            parts.append(np.zeros(n))
        else:
            w = rng.normal(0.0, math.sqrt(2.0 / fan_in), size=n)
            parts.append(w * (last_scale if i == 6 else 1.0))
    return np.concatenate(parts).astype(np.float32)


def cnn_training_recipe():
    """Training trajectories of the learned-Psi workload: 40 fields U[-0.05, 0.05] drawn in turn from
    default_rng(5), pairs (u_n, u_{n+32}) at n = 0, 8, 16, ... of each trajectory, the first 20000 pairs;
    2 validation trajectories from default_rng(6)."""
    return {"n_train_traj": 40, "train_seed": 5, "n_val_traj": 2, "val_seed": 6, "stride": 8, "lag": 32,
            "n_pairs": 20000}


def ac2d_fields(n_fields: int, nx: int, ny: int, seed: int, amp: float = 0.05) -> np.ndarray:
    """n_fields i.i.d. U[-amp, amp] fields drawn in turn from one generator, [n_fields, nx*ny]."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(-amp, amp, size=nx * ny) for _ in range(n_fields)])


def cnn_epoch_orders(seed: int, n_pairs: int, epochs: int):
    """One seeded permutation of the training pairs per epoch."""
    rng = np.random.default_rng(seed)
    return [rng.permutation(n_pairs) for _ in range(epochs)]


def batch_config(count: int = 256, seed: int = 4):
    """The batched workload: `count` independent instances drawn from default_rng(seed).

    kind uniform in {1D heat, 2D heat, 2D Allen-Cahn}; m uniform in {8, 16, 32};
    Nt = m * floor(U{512..8192} / m); 1D: nx in U{63..511} (the 1D heat recipe, nu 1,
    t in [0, 1], FP64); 2D heat: n x n, n in U{32..128} (the 2D heat recipe, nu 0.1,
    t in [0, 1]); 2D Allen-Cahn: periodic n x n, eps 0.02, dt 1e-5, u0 ~ U[-0.05, 0.05],
    coarse substeps s = ceil(m dt / eps^2 / 0.4) so that each coarse step keeps
    dT / (s eps^2) <= 0.4.  2D instances run the FP32-fine / FP64-residual form; the 2D heat
    instances, and the Allen-Cahn instances with one coarse substep (FAS in terms of e = w - v), solve
    Psi in the eigenbasis on the BF16 matrix cores.
    Instance b draws its initial field with seed 1000 + b.  FCF, tol 1e-8,
    k = max(2, ceil(0.1 (N_T + 1))).  Returns a list of (Problem, Options, u0).
    """
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        kind = (HEAT1D, HEAT2D, AC2D)[int(rng.integers(0, 3))]
        m = (8, 16, 32)[int(rng.integers(0, 3))]
        nt = m * (int(rng.integers(512, 8193)) // m)
        k = default_k(nt // m)
        if kind == HEAT1D:
            nx = int(rng.integers(63, 512))
            p = Problem(HEAT1D, nx=nx, ny=1, length=1.0, nu=1.0, t0=0.0, tf=1.0, nt=nt)
            u0, _ = heat1d_u0(nx, seed=1000 + b)
            o = Options(m=m, k=k, relax=1, tol=1e-8)
        elif kind == HEAT2D:
            n = int(rng.integers(32, 129))
            p = Problem(HEAT2D, nx=n, ny=n, length=1.0, nu=0.1, t0=0.0, tf=1.0, nt=nt, cg_rtol=1e-12)
            u0, _ = heat2d_u0(n, n, seed=1000 + b)
            o = Options(m=m, k=k, relax=1, tol=1e-8, precision=1, coarse_solver=2)
        else:
            n = int(rng.integers(32, 129))
            dt, eps = 1e-5, 0.02
            p = Problem(AC2D, nx=n, ny=n, length=1.0, nu=1.0, eps=eps, t0=0.0, tf=nt * dt, nt=nt, cg_rtol=1e-12)
            u0 = ac2d_u0(n, n, seed=1000 + b)
            s = max(1, math.ceil(m * dt / eps ** 2 / 0.4))
            o = Options(m=m, k=k, relax=1, tol=1e-8, precision=1, coarse_substeps=s, coarse_solver=2 if s == 1 else 0)
        out.append((p, o, u0))
    return out
