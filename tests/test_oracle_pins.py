"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formulas: each compares the oracle
with an independent route (closed forms, dense linear algebra assembled from
the paper's operator definitions, the figures' drawn index sets, exactness and
data-flow properties that the paper states).
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# helpers: dense operators assembled independently of the oracle
# ---------------------------------------------------------------------------

def lap1d(n, h):
    L = np.zeros((n, n))
    for i in range(n):
        L[i, i] = -2.0
        if i > 0:
            L[i, i - 1] = 1.0
        if i < n - 1:
            L[i, i + 1] = 1.0
    return L / (h * h)


def lap2d(nx, ny, hx, hy, periodic=False):
    n = nx * ny
    L = np.zeros((n, n))
    for j in range(ny):
        for i in range(nx):
            r = j * nx + i
            L[r, r] = -2.0 / hx ** 2 - 2.0 / hy ** 2
            for di, dj, h in ((-1, 0, hx), (1, 0, hx), (0, -1, hy), (0, 1, hy)):
                ii, jj = i + di, j + dj
                if periodic:
                    ii %= nx
                    jj %= ny
                elif not (0 <= ii < nx and 0 <= jj < ny):
                    continue
                L[r, jj * nx + ii] += 1.0 / h ** 2
    return L


def dense_phi(p, dt):
    """Exact backward-Euler propagator (I - dt nu L)^-1 as a dense matrix."""
    if p.kind == W.HEAT1D:
        L = lap1d(p.nx, p.length / (p.nx + 1))
    else:
        L = lap2d(p.nx, p.ny, p.length / (p.nx + 1), p.length / (p.ny + 1))
    return np.linalg.inv(np.eye(p.n) - dt * p.nu * L)


def c_points(p, o):
    return [j * o.m for j in range(p.nt // o.m + 1)]


# ---------------------------------------------------------------------------
# time grid: the local coarse grids drawn in Figs. 1, 2 and 5
# ---------------------------------------------------------------------------

def test_windows_match_figures(orc):
    g = json.load(open(os.path.join(GOLDEN, "windows.json")))
    f1 = g["fig1"]
    NT = f1["nt"] // f1["m"]
    assert NT == 7
    for p in range(NT + 1):
        s = orc.window_start(p, f1["k"])
        assert list(range(s, p + 1)) == f1["windows"][str(p)]
    f2 = g["fig2"]
    for p, pts in f2["windows_fine_index"].items():
        s = orc.window_start(int(p), f2["k"])
        assert [j * f2["coarse_stride"] for j in range(s, int(p) + 1)] == pts
    f5 = g["fig5"]
    for p, pts in f5["windows_fine_index"].items():
        s = orc.window_start(int(p), f5["k"])
        assert [j * f5["m"] for j in range(s, int(p) + 1)] == pts


# ---------------------------------------------------------------------------
# sequential time stepping: closed-form eigenmode decay and dense solves
# ---------------------------------------------------------------------------

def test_heat1d_closed_form_decay(orc):
    """Backward Euler on a sine mode decays by (1 + nu dt lam_j)^-n, lam_j = 4/h^2 sin^2(j pi h/2)."""
    p, o, u0 = W.config("c1")
    _, amps = W.heat1d_u0(p.nx, seed=1)
    u = orc.sequential(p, u0)
    h = 1.0 / (p.nx + 1)
    x = h * np.arange(1, p.nx + 1)
    coeffs = {1: 1.0, **amps}
    for n in (1, 7, 100, 1024):
        ref = np.zeros(p.nx)
        for j, a in coeffs.items():
            lam = 4.0 / h ** 2 * math.sin(j * math.pi * h / 2) ** 2
            ref += a * (1.0 + p.nu * p.dt * lam) ** (-n) * np.sin(j * math.pi * x)
        assert np.max(np.abs(u[n] - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref))), n


def test_heat2d_closed_form_decay(orc):
    """2D backward Euler with Jacobi-PCG: sum-of-modes decay, lam = lam_j(hx) + lam_l(hy)."""
    nx = ny = 32
    p = W.Problem(W.HEAT2D, nx=nx, ny=ny, nu=0.1, tf=20 / 4096, nt=20, cg_rtol=1e-14)
    u0, modes = W.heat2d_u0(nx, ny, seed=11, n_modes=6, max_mode=8)
    u = orc.sequential(p, u0)
    h = 1.0 / (nx + 1)
    x = h * np.arange(1, nx + 1)
    for n in (1, 5, 20):
        ref = np.zeros((ny, nx))
        for j, l, a in modes:
            lam = 4.0 / h ** 2 * (math.sin(j * math.pi * h / 2) ** 2 + math.sin(l * math.pi * h / 2) ** 2)
            ref += a * (1 + p.nu * p.dt * lam) ** (-n) * np.outer(np.sin(l * math.pi * x), np.sin(j * math.pi * x))
        assert np.max(np.abs(u[n] - ref.reshape(-1))) <= 1e-12 * np.max(np.abs(ref)), n


@pytest.mark.parametrize("kind", [W.HEAT1D, W.HEAT2D])
def test_dense_spacetime_solve(orc, kind):
    """Sequential stepping equals an LU solve of the assembled block-bidiagonal A u = g (section 2)."""
    if kind == W.HEAT1D:
        p, u0 = W.small_problem(W.HEAT1D, seed=3, nt=12, nx=5)
    else:
        p, u0 = W.small_problem(W.HEAT2D, seed=3, nt=10, nx=4, ny=3, cg_rtol=1e-15)
    Phi = dense_phi(p, p.dt)
    n, N = p.n, p.nt + 1
    A = np.eye(N * n)
    for i in range(1, N):
        A[i * n:(i + 1) * n, (i - 1) * n:i * n] = -Phi
    g = np.zeros(N * n)
    g[:n] = u0
    ref = np.linalg.solve(A, g).reshape(N, n)
    u = orc.sequential(p, u0)
    assert np.max(np.abs(u - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_cg_step_matches_dense_solve(orc):
    """One 2D step (Jacobi-PCG) equals the dense solve within its relative residual bound."""
    p, u0 = W.small_problem(W.HEAT2D, seed=5, nt=4, nx=9, ny=7, cg_rtol=1e-12)
    out = orc.step(p, p.dt * 8, u0)
    ref = dense_phi(p, p.dt * 8) @ u0
    # ||x - x*|| <= ||M^-1|| ||r|| <= rtol ||b||   (M = I - dt nu L >= I)
    assert np.linalg.norm(out - ref) <= 1.0001e-12 * np.linalg.norm(u0)


def test_ac_constant_state_recurrence(orc):
    """For a constant field the Laplacian vanishes: Phi(c) = c + dt (c - c^3)/eps^2."""
    p = W.Problem(W.AC2D, nx=8, ny=6, nu=1.0, eps=0.05, tf=1e-4, nt=10, cg_rtol=1e-14)
    for c in (0.3, -0.7, 1.0):
        out = orc.step(p, p.dt, np.full(p.n, c))
        ref = c + p.dt * (c - c ** 3) / p.eps ** 2
        assert np.max(np.abs(out - ref)) <= 4e-16 * max(1.0, abs(ref))


def test_ac_odd_symmetry_bitwise(orc):
    """Phi(-u) = -Phi(u); round-to-nearest is sign-symmetric, so -u0 gives exactly -u."""
    p, u0 = W.small_problem(W.AC2D, seed=9, nt=24, nx=8)
    a = orc.sequential(p, u0)
    b = orc.sequential(p, -u0)
    assert np.array_equal(a, -b)
    o = W.Options(m=4, k=2, relax=1, tol=1e-9)
    ua, _, _ = orc.solve(p, o, W.initial_guess(p, u0))
    ub, _, _ = orc.solve(p, o, W.initial_guess(p, -u0))
    assert np.array_equal(ua, -ub)


# ---------------------------------------------------------------------------
# the iteration: exactness, Parareal equivalence, error propagators
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("relax", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_exact_cpoints_after_i_iterations(orc, relax, k):
    """F: C-points 0..i are exact after i cycles; FCF: 0..2i.  After N_T cycles all of u is exact
    (section 2.1: the method solves for the exact solution in N_T iterations)."""
    p, u0 = W.small_problem(W.HEAT1D, seed=2, nt=40, nx=6)
    o = W.Options(m=4, k=k, relax=relax)
    NT = p.nt // o.m
    ref = orc.sequential(p, u0)
    u = W.initial_guess(p, u0, "random", seed=4)
    scale = np.max(np.abs(ref))
    for i in range(1, NT + 1):
        u = orc.cycle(p, o, u, u0)
        reach = i if relax == 0 else 2 * i
        for j in range(NT + 1):
            err = np.max(np.abs(u[j * o.m] - ref[j * o.m]))
            if j <= reach:
                assert err <= 1e-13 * scale, (i, j, err)
        if reach >= NT:
            assert np.max(np.abs(u - ref)) <= 1e-13 * scale
            break


def test_ragged_tail_exactness(orc):
    """m does not divide nt: the tail after C-point N_T is relaxed from it and still becomes exact."""
    p, u0 = W.small_problem(W.HEAT1D, seed=6, nt=43, nx=5)
    o = W.Options(m=4, k=3, relax=0)
    ref = orc.sequential(p, u0)
    u = W.initial_guess(p, u0, "random", seed=1)
    for _ in range(p.nt // o.m):
        u = orc.cycle(p, o, u, u0)
    assert np.max(np.abs(u - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("kind", [W.HEAT1D, W.HEAT2D, W.AC2D])
def test_f_relaxation_of_relaxed_iterate_is_identity(orc, kind):
    """F-relaxation recomputes every F-point from its C-point alone: a second pass reproduces the first
    bit for bit, and an F-point's value never enters (the property a sweep that leaves unchanged intervals
    alone rests on).  A pass that read a stored F-point (a wrong index) would differ on the scrambled
    iterate."""
    p, u0 = W.small_problem(kind, seed=8, nt=38, nx=9)
    o = W.Options(m=4, k=2)
    u = W.initial_guess(p, u0, "random", seed=2)
    once = orc.f_relax(p, o, u)
    assert np.array_equal(orc.f_relax(p, o, once), once)
    scrambled = once.copy()
    rng = np.random.default_rng(3)
    for t in range(p.nt + 1):
        if t % o.m:
            scrambled[t] = rng.standard_normal(p.n)
    assert np.array_equal(orc.f_relax(p, o, scrambled), once)
    # the F-points are the sequential steps from each C-point
    for j in range(0, p.nt, o.m):
        seq = orc.sequential(W.Problem(**{**p.__dict__, "nt": min(o.m - 1, p.nt - j),
                                          "t0": p.t0 + j * p.dt, "tf": p.t0 + (j + min(o.m - 1, p.nt - j)) * p.dt}),
                             once[j])
        np.testing.assert_allclose(once[j:j + len(seq)], seq, rtol=0, atol=1e-12 * np.max(np.abs(once)))


@pytest.mark.parametrize("kind,form", [(W.HEAT1D, 1), (W.HEAT2D, 1), (W.AC2D, 2)])
@pytest.mark.parametrize("relax", [0, 1])
def test_k_full_equals_parareal_bitwise(orc, kind, form, relax):
    """k = N_T + 1 gives Parareal / two-level MGRIT (section 2.1): iterates agree bit for bit."""
    p, u0 = W.small_problem(kind, seed=8, nt=24, nx=6)
    o = W.Options(m=3, k=p.nt // 3 + 1, relax=relax, coarse_form=form)
    u = W.initial_guess(p, u0, "random", seed=2)
    a, b = u.copy(), u.copy()
    for _ in range(3):
        a = orc.cycle(p, o, a, u0)
        b = orc.cycle(p, o, b, u0, parareal=True)
        assert np.array_equal(a, b)


def ecc_closed_form(Phi, Psi, m, k, NT):
    """E_cc of section 3.2: row p has Psi^x (Phi^m - Psi) at column p-1-x (x = 0..k-2)
    and Psi^{k-1} Phi^m at column p-k."""
    n = Phi.shape[0]
    Phim = np.linalg.matrix_power(Phi, m)
    E = np.zeros(((NT + 1) * n, (NT + 1) * n))
    for pp in range(1, NT + 1):
        for x in range(0, k - 1):
            q = pp - 1 - x
            if q < 0:
                break
            E[pp * n:(pp + 1) * n, q * n:(q + 1) * n] = np.linalg.matrix_power(Psi, x) @ (Phim - Psi)
        q = pp - k
        if q >= 0:
            E[pp * n:(pp + 1) * n, q * n:(q + 1) * n] = np.linalg.matrix_power(Psi, k - 1) @ Phim
    return E


def brute_force_cc(orc, p, o, ref, parareal=False):
    """Matrix of one oracle cycle acting on C-point errors (columns for C-points 1..N_T)."""
    n, NT = p.n, p.nt // o.m
    E = np.zeros(((NT + 1) * n, (NT + 1) * n))
    Ef = []
    for q in range(1, NT + 1):
        for b in range(n):
            u = ref.copy()
            u[q * o.m, b] += 1.0
            un = orc.cycle(p, o, u, ref[0], parareal=parareal)
            err = un - ref
            E[:, q * n + b] = np.concatenate([err[j * o.m] for j in range(NT + 1)])
            Ef.append(err)
    return E, Ef


@pytest.mark.parametrize("k", [1, 2, 3, 4, 8])
def test_ecc_closed_form_F(orc, k):
    """One cycle with F-relaxation maps C-point errors by E_cc (section 3.2, eq. for E_cc)."""
    p, u0 = W.small_problem(W.HEAT1D, seed=1, nt=21, nx=3, tf=0.3)
    o = W.Options(m=3, k=k, relax=0)
    NT = p.nt // o.m
    ref = orc.sequential(p, u0)
    E, Ef = brute_force_cc(orc, p, o, ref)
    Phi = dense_phi(p, p.dt)
    Psi = dense_phi(p, p.dt * o.m)
    Ecl = ecc_closed_form(Phi, Psi, o.m, k, NT)
    assert np.max(np.abs(E[:, p.n:] - Ecl[:, p.n:])) <= 1e-13
    # F rows after the cycle: Phi^i applied to the new error of their C-point (the E_fc block)
    for err in Ef:
        for j in range(NT):
            for i in range(1, o.m):
                assert np.allclose(err[j * o.m + i], np.linalg.matrix_power(Phi, i) @ err[j * o.m],
                                   rtol=0, atol=1e-13)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_ecc_closed_form_FCF(orc, k):
    """FCF: the CF sweep maps C errors by S (S_00 = I, S_{j,j-1} = Phi^m), so one cycle is E_cc S."""
    p, u0 = W.small_problem(W.HEAT1D, seed=1, nt=21, nx=3, tf=0.3)
    o = W.Options(m=3, k=k, relax=1)
    NT = p.nt // o.m
    n = p.n
    ref = orc.sequential(p, u0)
    E, _ = brute_force_cc(orc, p, o, ref)
    Phi = dense_phi(p, p.dt)
    Psi = dense_phi(p, p.dt * o.m)
    S = np.zeros(((NT + 1) * n, (NT + 1) * n))
    S[:n, :n] = np.eye(n)
    Phim = np.linalg.matrix_power(Phi, o.m)
    for j in range(1, NT + 1):
        S[j * n:(j + 1) * n, (j - 1) * n:j * n] = Phim
    Ecl = ecc_closed_form(Phi, Psi, o.m, k, NT) @ S
    assert np.max(np.abs(E[:, n:] - Ecl[:, n:])) <= 1e-13


def test_e0_assembled_from_definitions(orc):
    """Dense E = (I - sum_p P_S^(p) (A~_c^(p))^-1 R_I^(p) A) P R_I (section 3.1, eq. E0 with the
    approximate local matrices of 3.1.2) equals the map of one oracle cycle (F-relaxation)."""
    p, u0 = W.small_problem(W.HEAT1D, seed=4, nt=12, nx=2, tf=0.2)
    o = W.Options(m=3, k=2, relax=0)
    n, m, k, NT, N = p.n, o.m, o.k, p.nt // o.m, p.nt + 1
    Phi = dense_phi(p, p.dt)
    Psi = dense_phi(p, p.dt * m)
    I = np.eye
    A = I(N * n)
    for i in range(1, N):
        A[i * n:(i + 1) * n, (i - 1) * n:i * n] = -Phi
    # ideal interpolation P (columns: C-points) and injection R_I
    P = np.zeros((N * n, (NT + 1) * n))
    R = np.zeros(((NT + 1) * n, N * n))
    for j in range(NT + 1):
        R[j * n:(j + 1) * n, j * m * n:(j * m + 1) * n] = I(n)
        for i in range(m):
            t = j * m + i
            if t < N:
                P[t * n:(t + 1) * n, j * n:(j + 1) * n] = np.linalg.matrix_power(Phi, i)
    corr = np.zeros((N * n, N * n))
    for pp in range(NT + 1):
        s = max(0, pp - k + 1)
        w = pp - s + 1
        Rp = R[s * n:(pp + 1) * n, :]                       # R_I^(p): rows of the local grid
        Ac = I(w * n)
        for a in range(1, w):
            Ac[a * n:(a + 1) * n, (a - 1) * n:a * n] = -Psi
        PS = np.zeros((N * n, w * n))                       # P_S^(p): last local point, interpolated
        for i in range(m):
            t = pp * m + i
            if t < N:
                PS[t * n:(t + 1) * n, (w - 1) * n:w * n] = np.linalg.matrix_power(Phi, i)
        corr += PS @ np.linalg.solve(Ac, Rp @ A)
    E = (I(N * n) - corr) @ P @ R
    ref = orc.sequential(p, u0)
    Ebf = np.zeros((N * n, N * n))
    for c in range(n, N * n):
        u = ref.copy().reshape(-1)
        u[c] += 1.0
        Ebf[:, c] = (orc.cycle(p, o, u.reshape(N, n), ref[0]) - ref).reshape(-1)
    assert np.max(np.abs(Ebf[:, n:] - E[:, n:])) <= 1e-13


def test_selective_interpolation_linear_form(orc):
    """For a linear Phi and an F-relaxed iterate, correct-then-F-relax equals u_{pm+i} += Phi^i e_p."""
    p, u0 = W.small_problem(W.HEAT1D, seed=12, nt=20, nx=7)
    o = W.Options(m=5, k=2, relax=0)
    rng = np.random.default_rng(0)
    u = orc.f_relax(p, o, W.initial_guess(p, u0, "random", seed=5))
    NT = p.nt // o.m
    e = rng.standard_normal((NT + 1, p.n))
    e[0] = 0.0
    a = orc.correct(p, o, u, e)
    b = u.copy()
    for j in range(NT + 1):
        t = e[j].copy()
        for i in range(o.m):
            if j * o.m + i > p.nt:
                break
            b[j * o.m + i] += t
            t = orc.step(p, p.dt, t)
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))


@pytest.mark.parametrize("relax,grow", [(0, 0), (1, 1)])
def test_initial_condition_propagation_bitwise(orc, relax, grow):
    """Perturbing g_0 changes, after i cycles, exactly the C-points p <= k i (F) or (k+1) i (FCF);
    all later C-points are bitwise unchanged (section 4.2, the implicit propagation of the
    initial condition; the paper's count of (k-1) windows per iteration is the lower bound)."""
    p, u0 = W.small_problem(W.HEAT1D, seed=3, nt=60, nx=4)
    o = W.Options(m=2, k=4, relax=relax)
    NT = p.nt // o.m
    guess = W.initial_guess(p, u0, "random", seed=7)
    ga = guess.copy()
    gb = guess.copy()
    gb[0] = u0 * 1.5
    for i in range(1, 5):
        ga = orc.cycle(p, o, ga, ga[0])
        gb = orc.cycle(p, o, gb, gb[0])
        reach = (o.k + grow) * i
        for j in range(1, NT + 1):
            same = np.array_equal(ga[j * o.m], gb[j * o.m])
            assert same == (j > reach), (i, j)
        # the paper's shaded grids (Fig. 5 convention): windows containing C-points <= (k-1)(i-1)
        paper_reach = (o.k - 1) * i
        assert paper_reach <= reach


def test_theorem1_bound(orc):
    """Two-level convergence (Theorem 1): ||E_cc||_2 <= max over modes of
    |lam^m - mu| (1 - |mu|^{k-1}) / (1 - |mu|) + |lam^m mu^{k-1}| for the normal 1D Laplacian."""
    p, u0 = W.small_problem(W.HEAT1D, seed=1, nt=64, nx=7, tf=0.25)
    h = 1.0 / (p.nx + 1)
    ref = orc.sequential(p, u0)
    for k in (2, 3, 5):
        o = W.Options(m=4, k=k, relax=0)
        E, _ = brute_force_cc(orc, p, o, ref)
        norm = np.linalg.norm(E[p.n:, p.n:], 2)
        bound = 0.0
        for j in range(1, p.nx + 1):
            lamL = 4.0 / h ** 2 * math.sin(j * math.pi * h / 2) ** 2
            lam = 1.0 / (1 + p.dt * lamL)
            mu = 1.0 / (1 + o.m * p.dt * lamL)
            b = abs(lam ** o.m - mu) * (1 - abs(mu) ** (k - 1)) / (1 - abs(mu)) + abs(lam ** o.m * mu ** (k - 1))
            bound = max(bound, b)
        assert norm <= bound * (1 + 1e-12), (k, norm, bound)


def test_theorem1_example_value():
    """The worked example after Theorem 1: 0.99^500 = 0.0065..."""
    assert 0.0065 <= 0.99 ** 500 < 0.0066


# ---------------------------------------------------------------------------
# the fixed point
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", [W.HEAT1D, W.HEAT2D, W.AC2D])
def test_converged_solution_is_sequential(orc, kind):
    """Whatever Psi is, the converged iterate solves A(u) = g: it equals sequential stepping."""
    p, u0 = W.small_problem(kind, seed=13, nt=48, nx=6)
    o = W.Options(m=4, k=3, relax=1, tol=1e-11, coarse_substeps=2 if kind == W.AC2D else 1)
    u, hist, st = orc.solve(p, o, W.initial_guess(p, u0))
    assert st["status"] == 0 and hist[-1] <= 1e-11
    ref = orc.sequential(p, u0)
    # ||u - u*|| <= ||A^-1|| ||r||; the forward solve with contractive Phi has ||A^-1|| <= nt + 1
    assert np.linalg.norm(u - ref) <= (p.nt + 1) * 1.0000001e-11 * (10 if kind == W.AC2D else 1)
    assert abs(orc.residual_norm(p, u, u0) - hist[-1]) <= 1e-14 + 1e-9 * hist[-1]


def test_solve_status_codes(orc):
    p, u0 = W.small_problem(W.HEAT2D, seed=1, nt=16, nx=5, cg_max_iter=1)
    o = W.Options(m=4, k=2)
    with pytest.raises(orc.OracleError) as ei:
        orc.solve(p, o, W.initial_guess(p, u0))
    assert ei.value.status == orc.INNER
    p, u0 = W.small_problem(W.HEAT1D, seed=1, nt=64, nx=5)
    o = W.Options(m=4, k=2, max_iter=2, tol=1e-14)
    u, hist, st = orc.solve(p, o, W.initial_guess(p, u0), allow_status=(orc.NOT_CONVERGED,))
    assert st["iterations"] == 2 and st["status"] == orc.NOT_CONVERGED
    g = W.initial_guess(p, u0)
    g[8, 2] = np.nan                     # a C-point (m = 4)
    with pytest.raises(orc.OracleError) as ei:
        orc.solve(p, W.Options(m=4, k=2), g)
    assert ei.value.status == orc.DIVERGED


@pytest.mark.parametrize("relax", [0, 1])
def test_fas_form_equals_linear_form_on_linear_problem(orc, relax):
    """For a linear Psi the FAS local problem A_c(w) = A_c(v) + r_c has w - v = the linear
    solution (Alg. 2's coarsest-level branch reduces to Alg. 1), so the two forms agree to rounding."""
    p, u0 = W.small_problem(W.HEAT1D, seed=21, nt=36, nx=6)
    lin = W.Options(m=3, k=4, relax=relax, coarse_form=1)
    fas = W.Options(m=3, k=4, relax=relax, coarse_form=2)
    a = W.initial_guess(p, u0, "random", seed=3)
    b = a.copy()
    for _ in range(4):
        a = orc.cycle(p, lin, a, u0)
        b = orc.cycle(p, fas, b, u0)
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_fine_and_coarse_steps_share_the_integrator(orc):
    """Psi with s substeps of dT/s equals s integrator steps of size m dt / s."""
    p, u0 = W.small_problem(W.AC2D, seed=2, nt=16, nx=6)
    o = W.Options(m=4, coarse_substeps=3)
    x = u0.copy()
    for _ in range(3):
        x = orc.step(p, p.dt * 4 / 3, x)
    assert np.array_equal(orc.coarse_step(p, o, u0), x)


def test_coarse_tolerance_keeps_fixed_point(orc):
    """A loose CG tolerance inside Psi changes the iteration, not its fixed point (sequential stepping)."""
    p, u0 = W.small_problem(W.HEAT2D, seed=4, nt=48, nx=8, ny=6)
    o = W.Options(m=4, k=3, relax=1, tol=1e-11, coarse_cg_rtol=1e-3)
    u, hist, st = orc.solve(p, o, W.initial_guess(p, u0))
    assert st["status"] == 0 and hist[-1] <= 1e-11
    assert np.linalg.norm(u - orc.sequential(p, u0)) <= (p.nt + 1) * 1.0000001e-11
    tight = W.Options(m=4, k=3, relax=1, tol=1e-11)
    g = W.initial_guess(p, u0, "random", seed=1)
    a = orc.cycle(p, o, g)
    b = orc.cycle(p, tight, g)
    assert not np.array_equal(a, b)      # the option reaches Psi


# ---------------------------------------------------------------------------
# implicit form of the residual (stopping test of the FP32-fine form)
# ---------------------------------------------------------------------------

def dense_M_psi(p):
    """M = I - dt nu L (dense, from the operator definitions) and psi, the explicit part of the step."""
    if p.kind == W.HEAT1D:
        L = lap1d(p.nx, p.length / (p.nx + 1))
    elif p.kind == W.HEAT2D:
        L = lap2d(p.nx, p.ny, p.length / (p.nx + 1), p.length / (p.ny + 1))
    else:
        L = lap2d(p.nx, p.ny, p.length / p.nx, p.length / p.ny, periodic=True)
    M = np.eye(p.n) - p.dt * p.nu * L
    if p.kind == W.AC2D:
        def psi(v):
            return v + p.dt / p.eps ** 2 * (v - v ** 3)
    else:
        def psi(v):
            return v
    return M, psi


def _kind_cases():
    return [
        W.small_problem(W.HEAT1D, seed=2, nt=6, nx=9, cg_rtol=1e-14),
        W.small_problem(W.HEAT2D, seed=3, nt=6, nx=7, ny=5, cg_rtol=1e-14),
        W.small_problem(W.AC2D, seed=4, nt=6, nx=6, ny=5, cg_rtol=1e-14),
    ]


@pytest.mark.parametrize("case", range(3))
def test_implicit_residual_matches_dense_operator(orc, case):
    """rho_i = psi(u_{i-1}) - M u_i with M assembled densely (row 0 is g_0 - u_0 = 0)."""
    p, _ = _kind_cases()[case]
    u = np.random.default_rng(11).uniform(-1, 1, size=(p.nt + 1, p.n))
    M, psi = dense_M_psi(p)
    rho = orc.implicit_residual(p, u)
    assert np.all(rho[0] == 0.0)
    for i in range(1, p.nt + 1):
        ref = psi(u[i - 1]) - M @ u[i]
        assert np.max(np.abs(rho[i] - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("case", range(3))
def test_step_residual_equals_paper_residual(orc, case):
    """M^-1 rho_i (solve from zero) equals Phi(u_{i-1}) - u_i (step, then difference) on a rough iterate."""
    p, u0 = _kind_cases()[case]
    u = np.random.default_rng(12).uniform(-1, 1, size=(p.nt + 1, p.n))
    u[0] = u0
    r_step = orc.step_residual(p, u)
    r_paper = orc.residual(p, u, u0)
    assert np.all(r_step[0] == 0.0)
    assert np.max(np.abs(r_step - r_paper)) <= 1e-12 * np.max(np.abs(r_paper))
    # |M^-1| <= 1: every slice of the residual is no longer than its implicit form
    rho = orc.implicit_residual(p, u)
    for i in range(1, p.nt + 1):
        assert np.linalg.norm(r_step[i]) <= np.linalg.norm(rho[i]) * (1 + 1e-12)


@pytest.mark.parametrize("case", range(3))
def test_implicit_residual_vanishes_on_sequential_solution(orc, case):
    """Sequential stepping solves every step, so rho and M^-1 rho are zero up to the CG tolerance."""
    p, u0 = _kind_cases()[case]
    u = orc.sequential(p, u0)
    scale = np.max(np.abs(u))
    assert np.max(np.abs(orc.implicit_residual(p, u))) <= 1e-13 * scale
    assert np.max(np.abs(orc.step_residual(p, u))) <= 1e-13 * scale
