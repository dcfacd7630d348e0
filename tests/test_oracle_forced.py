"""Pins of the oracle's forced 1D heat problem and of the k-study of section 4.3.

The manufactured problem u_t - u_xx = b on [0, 3] x [0, pi] (section 4.3,
"Size of local coarse grids") adds a PDE source to the backward Euler step:
(I - dt L) u_i = u_{i-1} + dt b(t_i).  The pins below compare the oracle with
routes that share none of its code: the scalar recurrence of a single sine
mode (an exact eigenvector of the discrete Laplacian), dense forward
substitution with the inverse assembled from the operator, and the statements
the paper makes about its k-study (its Figs. of iterations against k and
k / #C-points, and of residual histories and errors).
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "kstudy.json")))


def lap1d(n, h):
    L = np.diag(-2.0 * np.ones(n)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)
    return L / (h * h)


def dense_forced_sequential(p, u0, src):
    """u_i = (I - dt nu L)^-1 (u_{i-1} + dt b_i) by a dense inverse."""
    h = p.length / (p.nx + 1)
    Minv = np.linalg.inv(np.eye(p.n) - p.dt * p.nu * lap1d(p.nx, h))
    u = np.zeros((p.nt + 1, p.n))
    u[0] = u0
    for i in range(1, p.nt + 1):
        u[i] = Minv @ (u[i - 1] + p.dt * src[i])
    return u, Minv


def test_forced_single_mode_recurrence(orc):
    # u0 = sin(pi x) and b = beta(t) sin(pi x) stay on the sine mode sin(pi x) of [0, 3] (the third
    # Dirichlet mode), an exact eigenvector of the three-point Laplacian with eigenvalue
    # -(4/h^2) sin^2(pi h / 2); backward Euler with the source at the new time level reduces to
    # a_i (1 + dt (4/h^2) sin^2(pi h / 2)) = a_{i-1} + dt beta(t_i), a_0 = 1.
    p, u0, src, _ = W.heat1d_forced(nx=63, nt=200)
    h = p.length / (p.nx + 1)
    lam = 4.0 / h ** 2 * math.sin(math.pi * h / 2) ** 2
    a = [1.0]
    for i in range(1, p.nt + 1):
        t = p.t0 + i * p.dt
        beta = -(math.sin(t) - math.pi ** 2 * math.cos(t))
        a.append((a[-1] + p.dt * beta) / (1.0 + p.dt * lam))
    x = h * np.arange(1, p.nx + 1)
    expect = np.outer(np.array(a), np.sin(np.pi * x))
    u = orc.sequential(p, u0, source=src)
    assert np.abs(u - expect).max() <= 1e-13 * np.abs(expect).max()
    # the source taken at the old time level instead would be off by O(dt) per step
    assert np.abs(orc.sequential(p, u0) - expect).max() > 1e-3


def test_forced_sequential_dense_random_source(orc):
    rng = np.random.default_rng(11)
    p = W.Problem(W.HEAT1D, nx=9, length=3.0, nu=0.7, t0=0.2, tf=1.1, nt=23)
    u0 = rng.normal(size=p.n)
    src = rng.normal(size=(p.nt + 1, p.n))
    ref, _ = dense_forced_sequential(p, u0, src)
    u = orc.sequential(p, u0, source=src)
    assert np.abs(u - ref).max() <= 1e-13 * np.abs(ref).max()


def test_forced_residual_forms_dense(orc):
    # r_i = g_i + Phi(u_{i-1}) - u_i with Phi = M^-1 and g_i = M^-1 dt b_i (eq. (2) with the source)
    rng = np.random.default_rng(12)
    p = W.Problem(W.HEAT1D, nx=9, length=3.0, nu=0.7, t0=0.0, tf=1.0, nt=17)
    u0 = rng.normal(size=p.n)
    src = rng.normal(size=(p.nt + 1, p.n))
    u = rng.normal(size=(p.nt + 1, p.n))
    u[0] = u0
    _, Minv = dense_forced_sequential(p, u0, src)
    M = np.linalg.inv(Minv)
    r = np.zeros_like(u)
    rho = np.zeros_like(u)
    for i in range(1, p.nt + 1):
        r[i] = Minv @ (u[i - 1] + p.dt * src[i]) - u[i]
        rho[i] = M @ r[i]
    np.testing.assert_allclose(orc.residual(p, u, u0, source=src), r, rtol=0, atol=1e-12)
    np.testing.assert_allclose(orc.step_residual(p, u, source=src), r, rtol=0, atol=1e-12)
    np.testing.assert_allclose(orc.implicit_residual(p, u, source=src), rho, rtol=0, atol=1e-11)
    # and the residual vanishes at the sequential solution
    seq = orc.sequential(p, u0, source=src)
    assert np.abs(orc.residual(p, seq, u0, source=src)).max() <= 1e-13


@pytest.mark.parametrize("relax", [0, 1])
@pytest.mark.parametrize("k", [2, 3, 100])
def test_forced_atmgrit_reaches_sequential(orc, relax, k):
    p, u0, src, ug = W.heat1d_forced(nx=31, nt=250)  # nt = 250 is not a multiple of m: a ragged tail
    o = W.Options(m=8, k=k, relax=relax, tol=1e-11, max_iter=200, coarse_form=1)
    seq = orc.sequential(p, u0, source=src)
    u, hist, st = orc.solve(p, o, ug, source=src)
    assert st["iterations"] >= 1 and hist[-1] <= o.tol
    assert np.abs(u - seq).max() <= 1e-9


# ---------------------------------------------------------------------------
# the k-study of section 4.3 at the paper's size: 1025 grid points, 16384 time
# points, random initial guess, F-relaxation, two levels, tol 1e-7
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def kstudy(orc):
    orc.set_threads(8)
    p, u0, src, ug = W.heat1d_forced()
    seq = orc.sequential(p, u0, source=src)
    exact = W.heat1d_forced_exact(p)
    runs = {}

    def run(m, k):
        if (m, k) not in runs:
            u, hist, st = orc.solve(p, W.k_study_options(m, k), ug, source=src)
            runs[(m, k)] = dict(its=st["iterations"], hist=hist, err_exact=np.abs(u - exact).max(),
                                err_seq=np.abs(u - seq).max())
        return runs[(m, k)]

    yield run, np.abs(seq - exact).max()
    orc.set_threads(1)


def test_k_study_grid_reading():
    # the grid of the study as read (1025 points with both ends, 16384 time points on [0, pi]) makes
    # k = 128 at m = 128 exactly Parareal: every window reaches back to C-point 0 and the deepest takes
    # 127 coarse steps
    g = GOLDEN["problem"]
    p, _, _, _ = W.heat1d_forced()
    assert p.nx + 2 == g["dof"] and p.nt + 1 == g["time_points"] and p.length == g["length"]
    assert abs(p.tf - math.pi * g["tf_over_pi"]) < 1e-15
    par = GOLDEN["parareal_equivalence"]
    NT = p.nt // par["m"]
    assert NT + 1 == par["k"]                     # k covers every C-point
    assert max(min(q, par["k"] - 1) for q in range(NT + 1)) == par["sequential_coarse_steps"]
    assert all(max(0, q - par["k"] + 1) == 0 for q in range(NT + 1))


@pytest.mark.slow
def test_k_study_k12_matches_parareal(kstudy):
    # m = 128: 128 C-points; k = 128 is Parareal (127 sequential coarse steps), and k = 12 needs
    # the same number of iterations
    run, _ = kstudy
    g = GOLDEN["equal_convergence"]
    assert run(g["m"], g["k_small"])["its"] == run(g["m"], g["k_parareal"])["its"]
    assert run(g["m"], g["k_small"] // 2)["its"] > run(g["m"], g["k_small"])["its"]


@pytest.mark.slow
def test_k_study_saturation_ratio(kstudy):
    # convergence stops improving at about the same k / #C-points (about 0.08) for each m:
    # m = 64 has 256 C-points, so k = 20 (0.078) already converges like Parareal, k = 12 (0.047) not
    run, _ = kstudy
    ratio = GOLDEN["saturation_ratio"]["about"]
    par = run(64, 256)["its"]
    k_sat = 20                                    # the first k of the study at or above ratio * 256
    assert abs(k_sat / 256 - ratio) < 0.01
    assert run(64, k_sat)["its"] == par
    assert run(64, 12)["its"] > par


@pytest.mark.slow
def test_k_study_history_phases_and_error(kstudy):
    # small k: slower than Parareal at first, then the rate of Parareal once the initial condition
    # has crossed all local grids; every variant reaches the time-stepping error against the
    # exact solution sin(pi x) cos t
    run, err_seq = kstudy
    h12, h128 = run(128, 12)["hist"], run(128, 128)["hist"]
    assert all(h12[i] > h128[i] for i in range(1, 6))
    assert len(h12) == len(h128)
    np.testing.assert_allclose(h12[-3:], h128[-3:], rtol=0.15)
    assert 1e-7 < err_seq < 1e-5  # O(dt + h^2) with dt = pi/16383, h = 3/1024
    for key in [(128, 12), (128, 128), (64, 20)]:
        r = run(*key)
        assert abs(r["err_exact"] - err_seq) <= 1e-3 * err_seq
        assert r["err_seq"] <= 1e-8
