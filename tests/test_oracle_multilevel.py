"""Pins of the oracle's multilevel FAS AT-MGRIT V-cycle (section 2.2, Alg. 2).

For a linear problem one V-cycle maps the error e = u - u* by a matrix that can
be assembled from the operators' definitions alone: the level-0 relaxation S_0,
injection R_0, ideal interpolation P_0, the level-1 space-time matrix A_1, and
the two-level AT-MGRIT error propagator E_1 of level 1 (section 3.1: local
matrices with the coarsest propagator, selective ideal interpolation P_S).  The
level-1 FAS problem starts from the injected iterate, i.e. from zero error, so
one level-1 cycle returns x = (I - E_1) A_1^-1 b for its right-hand side b, and

    E = (I - P_0 (I - E_1) A_1^-1 R_0 A_0) S_0.

The oracle's V-cycle is compared column by column with this matrix.  Further
pins: L = 2 reproduces the (pinned) two-level FAS oracle bit for bit, and the
V-cycle converges to sequential stepping for every kind.
"""
import numpy as np
import pytest

import workloads as W


def phi_1d(p, dt):
    h = p.length / (p.nx + 1)
    L = (np.diag(-2.0 * np.ones(p.nx)) + np.diag(np.ones(p.nx - 1), 1) + np.diag(np.ones(p.nx - 1), -1)) / h ** 2
    return np.linalg.inv(np.eye(p.nx) - dt * p.nu * L)


def spacetime(Phi, N, n):
    A = np.eye(N * n)
    for i in range(1, N):
        A[i * n:(i + 1) * n, (i - 1) * n:i * n] = -Phi
    return A


def transfer(Phi, N, m, n):
    """Injection R (to C-points 0..NC) and ideal interpolation P (Phi^i from C-point j to point jm+i)."""
    NC = (N - 1) // m
    R = np.zeros(((NC + 1) * n, N * n))
    P = np.zeros((N * n, (NC + 1) * n))
    for j in range(NC + 1):
        R[j * n:(j + 1) * n, j * m * n:(j * m + 1) * n] = np.eye(n)
        for i in range(m):
            t = j * m + i
            if t < N:
                P[t * n:(t + 1) * n, j * n:(j + 1) * n] = np.linalg.matrix_power(Phi, i)
    return R, P, NC


def relaxation(Phi, N, m, n, relax):
    """Error map of F- (relax 0) or FCF-relaxation (relax 1): F sets e_F = Phi^i e_C, C sets
    e_{jm} = Phi e_{jm-1} for j >= 1."""
    R, P, NC = transfer(Phi, N, m, n)
    F = P @ R
    if relax == 0:
        return F
    C = np.eye(N * n)
    for j in range(1, NC + 1):
        t = j * m
        C[t * n:(t + 1) * n, :] = 0.0
        C[t * n:(t + 1) * n, (t - 1) * n:t * n] = Phi
    return F @ C @ F


def two_level_E(Phi, Psi, N, m, k, n, relax):
    """(I - sum_p P_S^(p) (A~^(p))^-1 R_I^(p) A) S for the grid of N points (section 3.1)."""
    A = spacetime(Phi, N, n)
    R, _, NC = transfer(Phi, N, m, n)
    corr = np.zeros((N * n, N * n))
    for p in range(NC + 1):
        s = max(0, p - k + 1)
        w = p - s + 1
        Ac = spacetime(Psi, w, n)
        PS = np.zeros((N * n, w * n))
        for i in range(m):
            t = p * m + i
            if t < N:
                PS[t * n:(t + 1) * n, (w - 1) * n:w * n] = np.linalg.matrix_power(Phi, i)
        corr += PS @ np.linalg.solve(Ac, R[s * n:(p + 1) * n, :] @ A)
    return (np.eye(N * n) - corr) @ relaxation(Phi, N, m, n, relax)


def three_level_E(p, o):
    n, N0 = p.n, p.nt + 1
    m0, m1 = o.m, o.m_coarse
    Phi0, Phi1, Phi2 = phi_1d(p, p.dt), phi_1d(p, p.dt * m0), phi_1d(p, p.dt * m0 * m1)
    A0 = spacetime(Phi0, N0, n)
    R0, P0, N1 = transfer(Phi0, N0, m0, n)
    A1 = spacetime(Phi1, N1 + 1, n)
    E1 = two_level_E(Phi1, Phi2, N1 + 1, m1, o.k, n, o.relax)
    M1 = (np.eye((N1 + 1) * n) - E1) @ np.linalg.inv(A1)
    return (np.eye(N0 * n) - P0 @ M1 @ R0 @ A0) @ relaxation(Phi0, N0, m0, n, o.relax)


@pytest.mark.parametrize("relax", [0, 1])
@pytest.mark.parametrize("nt,m0,m1,k", [(24, 2, 3, 2), (26, 2, 3, 2), (27, 2, 3, 3), (36, 3, 2, 2), (24, 2, 3, 9)],
                         ids=["exact", "ragged1", "ragged0", "m3x2", "k-global"])
def test_vcycle_equals_assembled_propagator(orc, relax, nt, m0, m1, k):
    p, u0 = W.small_problem(W.HEAT1D, seed=4, nt=nt, nx=2, tf=0.3)
    o = W.Options(m=m0, k=k, relax=relax, levels=3, m_coarse=m1, coarse_form=2)
    E = three_level_E(p, o)
    ref = orc.sequential(p, u0)
    N, n = p.nt + 1, p.n
    Ebf = np.zeros((N * n, N * n))
    for c in range(n, N * n):
        u = ref.copy().reshape(-1)
        u[c] += 1.0
        Ebf[:, c] = (orc.ml_cycle(p, o, u.reshape(N, n), ref[0]) - ref).reshape(-1)
    assert np.max(np.abs(Ebf[:, n:] - E[:, n:])) <= 1e-13


@pytest.mark.parametrize("kind", [W.HEAT1D, W.HEAT2D, W.AC2D])
@pytest.mark.parametrize("relax", [0, 1])
def test_two_levels_reproduce_the_two_level_fas_oracle(orc, kind, relax):
    p, u0 = W.small_problem(kind, seed=3, nt=40, nx=6)
    o = W.Options(m=4, k=3, relax=relax, tol=1e-10, max_iter=50, coarse_form=2, levels=2)
    g = W.initial_guess(p, u0, "random", seed=1) * (0.3 if kind == W.AC2D else 1.0)
    g[0] = u0
    a, ha, sa = orc.solve(p, o, g)
    b, hb, sb = orc.ml_solve(p, o, g)
    assert sa["iterations"] == sb["iterations"]
    assert np.array_equal(a, b) and np.array_equal(ha, hb)


@pytest.mark.parametrize("kind", [W.HEAT1D, W.HEAT2D, W.AC2D])
@pytest.mark.parametrize("relax", [0, 1])
@pytest.mark.parametrize("k", [2, 100])
def test_three_levels_converge_to_sequential(orc, kind, relax, k):
    p, u0 = W.small_problem(kind, seed=3, nt=97, nx=6)  # 97 = 24 * 4 + 1, 24 = 8 * 3: a ragged level 0
    o = W.Options(m=4, k=k, relax=relax, tol=1e-10, max_iter=100, levels=3, m_coarse=3)
    u, hist, st = orc.ml_solve(p, o, W.initial_guess(p, u0))
    assert hist[-1] <= o.tol and st["iterations"] >= 2
    assert np.abs(u - orc.sequential(p, u0)).max() <= 1e-9


def test_three_levels_with_source(orc):
    p, u0, src, ug = W.heat1d_forced(nx=31, nt=255)
    o = W.Options(m=8, k=2, relax=1, tol=1e-9, max_iter=100, levels=3, m_coarse=4)
    u, hist, st = orc.ml_solve(p, o, ug, source=src)
    assert hist[-1] <= o.tol
    assert np.abs(u - orc.sequential(p, u0, source=src)).max() <= 1e-9


# ---------------------------------------------------------------------------
# nested iteration (section 2.2): the initial guess from the coarse levels up
# ---------------------------------------------------------------------------

def nested_windows(Psi, v, k, n):
    """Local problems of the re-discretised coarse system A(w) = g (g = u_0, 0, ..) from the injected
    guess v in FAS form: window p starts at s = max(0, p-k+1) from v_s + r_s, r the coarse residual
    (r_0 = 0, r_s = Psi v_{s-1} - v_s), and steps with Psi; its last value is w_p."""
    N = v.shape[0]
    w = np.zeros_like(v)
    for p in range(N):
        s = max(0, p - k + 1)
        x = v[0] if s == 0 else Psi @ v[s - 1]
        for _ in range(s + 1, p + 1):
            x = Psi @ x
        w[p] = x
    return w


def interpolate(Phi, uc, N, m):
    """Ideal interpolation: C-point j takes uc_j, point jm+i takes Phi^i uc_j."""
    out = np.zeros((N, uc.shape[1]))
    for t in range(N):
        j, i = divmod(t, m)
        out[t] = np.linalg.matrix_power(Phi, i) @ uc[j]
    return out


@pytest.mark.parametrize("k", [2, 3, 50])
def test_nested_two_levels_closed_form(orc, k):
    p, u0 = W.small_problem(W.HEAT1D, seed=4, nt=29, nx=3, tf=0.3)   # ragged: 29 = 9 * 3 + 2
    o = W.Options(m=3, k=k, relax=1, levels=2, coarse_form=2)
    g = W.initial_guess(p, u0, "random", seed=2)
    Phi, Psi = phi_1d(p, p.dt), phi_1d(p, p.dt * o.m)
    v = g[::o.m][: p.nt // o.m + 1]
    ref = interpolate(Phi, nested_windows(Psi, v, k, p.n), p.nt + 1, o.m)
    got = orc.ml_nested(p, o, g)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("relax", [0, 1])
@pytest.mark.parametrize("nt,m0,m1,k", [(24, 2, 3, 2), (27, 2, 3, 3), (36, 3, 2, 9)])
def test_nested_three_levels_assembled(orc, relax, nt, m0, m1, k):
    p, u0 = W.small_problem(W.HEAT1D, seed=4, nt=nt, nx=2, tf=0.3)
    o = W.Options(m=m0, k=k, relax=relax, levels=3, m_coarse=m1, coarse_form=2)
    g = W.initial_guess(p, u0, "random", seed=2)
    n = p.n
    Phi0, Phi1, Phi2 = phi_1d(p, p.dt), phi_1d(p, p.dt * m0), phi_1d(p, p.dt * m0 * m1)
    N1 = p.nt // m0
    N2 = N1 // m1
    v2 = g[::m0][: N1 + 1][::m1][: N2 + 1]
    u1 = interpolate(Phi1, nested_windows(Phi2, v2, k, n), N1 + 1, m1)
    # one level-1 V-cycle for A_1(u) = (u_0, 0, ..): u1 <- u1* + E_1 (u1 - u1*), u1* its sequential solution
    star = np.array([np.linalg.matrix_power(Phi1, i) @ u0 for i in range(N1 + 1)])
    E1 = two_level_E(Phi1, Phi2, N1 + 1, m1, k, n, relax)
    u1 = star + (E1 @ (u1 - star).reshape(-1)).reshape(N1 + 1, n)
    ref = interpolate(Phi0, u1, p.nt + 1, m0)
    got = orc.ml_nested(p, o, g)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("levels", [2, 3])
@pytest.mark.parametrize("kind", [W.HEAT1D, W.HEAT2D, W.AC2D])
def test_nested_solve_reaches_sequential(orc, levels, kind):
    p, u0 = W.small_problem(kind, seed=3, nt=97, nx=6)
    o = W.Options(m=4, k=2, relax=1, tol=1e-10, max_iter=100, levels=levels, m_coarse=3, coarse_form=2, nested=1)
    u, hist, st = orc.ml_solve(p, o, W.initial_guess(p, u0))
    assert hist[-1] <= o.tol
    assert np.abs(u - orc.sequential(p, u0)).max() <= 1e-9
