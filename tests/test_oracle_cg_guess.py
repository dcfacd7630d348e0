"""Pins of the oracle's starting guess for the fine CG solves (cg_guess) and of
its solve loop's handling of an iterate that is already F-relaxed.

The paper leaves the inner linear solve of the 2D steps open (section 4.3 only
names the integrator).  With cg_guess = 1 an F-relaxation pass starts the solve
of F-point t from u_t + (u'_{t-1} - u_{t-1}): the iterate's value there moved by
the change the pass has made at t-1.  The pins below fix that formula without
re-typing it: a CG held to a tolerance it meets from the start returns its guess,
so a pass then moves every F-point of an interval by the change of its C-point
(to rounding) (the plain guess instead copies the C-value forward); the solves still
reach the tolerance, so one pass agrees with the plain guess to the CG error
bound, with fewer iterations once the change is small; and the solve loop,
which no longer repeats the F-relaxation of an F-relaxed iterate, returns bit
for bit what the cycle-by-cycle form returns with the plain guess.
"""
import ctypes
import dataclasses

import numpy as np
import pytest

import workloads as W


def cpoints(p, o, u):
    NT = p.nt // o.m
    return np.ascontiguousarray(u[::o.m][: NT + 1])


def f_relax_count(orc, p, o, u, c_old=None, skip=False):
    """The oracle's F-relaxation with its CG iteration count."""
    u = np.array(u, dtype=np.float64, order="C")
    cg = ctypes.c_int64(0)
    L = orc.lib()
    cptr = orc._ptr(np.ascontiguousarray(c_old)) if c_old is not None else None
    st = L.or_f_relax_from(ctypes.byref(orc._prob(p)), ctypes.byref(orc._opts(o)), orc._ptr(u), cptr, int(skip),
                           ctypes.byref(cg))
    assert st == 0
    return u, cg.value


def relaxed_problem(orc, kind, seed=5, nt=45, nx=9, m=4):
    p, u0 = W.small_problem(kind, seed=seed, nt=nt, nx=nx)   # 45 = 11 * 4 + 1: a ragged tail
    g = W.initial_guess(p, u0, "random", seed=seed) * (0.3 if kind == W.AC2D else 1.0)
    g[0] = u0
    o = W.Options(m=m, k=2, relax=1)
    return p, o, orc.f_relax(p, o, g)


@pytest.mark.parametrize("kind", [W.HEAT2D, W.AC2D])
def test_guess_is_the_shifted_iterate_when_cg_takes_no_step(orc, kind):
    # cg_rtol >= 1: every solve meets its tolerance at the start and returns its guess
    p, o, u = relaxed_problem(orc, kind)
    p = dataclasses.replace(p, cg_rtol=1e3)
    rng = np.random.default_rng(9)
    c_old = cpoints(p, o, u)
    unew = u.copy()
    d = rng.standard_normal(c_old.shape)
    d[0] = 0.0
    d[3] = 0.0                                     # one interval whose C-point does not move
    for j in range(c_old.shape[0]):
        unew[j * o.m] += d[j]
    got1 = orc.f_relax(p, dataclasses.replace(o, cg_guess=1), unew, c_old=c_old)
    got0 = orc.f_relax(p, o, unew, c_old=c_old)
    for t in range(p.nt + 1):
        j, i = divmod(t, o.m)
        if i == 0:
            assert np.array_equal(got1[t], unew[t]) and np.array_equal(got0[t], unew[t])
            continue
        # extrapolated: u_t + d_j (the change telescopes, up to a rounding per step); plain: the C-value
        # copied forward
        np.testing.assert_allclose(got1[t], u[t] + d[j], rtol=0, atol=1e-14 * i * (1 + np.abs(d).max()))
        np.testing.assert_array_equal(got0[t], unew[j * o.m])


@pytest.mark.parametrize("kind", [W.HEAT2D, W.AC2D])
def test_guess_changes_only_the_cg_start(orc, kind):
    p, o, u = relaxed_problem(orc, kind)
    c_old = cpoints(p, o, u)
    rng = np.random.default_rng(10)
    unew = u.copy()
    for j in range(1, c_old.shape[0]):
        unew[j * o.m] += 1e-6 * rng.standard_normal(p.n)
    a, n0 = f_relax_count(orc, p, o, unew, c_old)
    b, n1 = f_relax_count(orc, p, dataclasses.replace(o, cg_guess=1), unew, c_old)
    # both solve every step to cg_rtol: they agree to the CG error bound (kappa rtol |u|, kappa < 10 here)
    assert np.abs(a - b).max() <= 10 * p.cg_rtol * np.abs(a).max()
    # the extrapolated start is within the change's reach of the solution: fewer iterations
    assert n1 < 0.6 * n0, (n0, n1)
    # a wrong sign in the extrapolation starts farther away than the plain guess
    bad = unew.copy()
    for j in range(1, c_old.shape[0]):
        bad[j * o.m] = 2 * c_old[j] - unew[j * o.m]  # mirrors the change: the shift enters with -d
    _, nbad = f_relax_count(orc, p, dataclasses.replace(o, cg_guess=1), unew, bad)
    assert nbad > n1


@pytest.mark.parametrize("kind", [W.HEAT2D, W.AC2D])
def test_unchanged_relaxed_iterate_needs_no_iterations(orc, kind):
    # the stored iterate is the relaxation of its C-points: with nothing moved the extrapolated guess
    # is that relaxation, whose residual is within the tolerance already
    p, o, u = relaxed_problem(orc, kind)
    got, n1 = f_relax_count(orc, p, dataclasses.replace(o, cg_guess=1), u, cpoints(p, o, u))
    _, n0 = f_relax_count(orc, p, o, u, cpoints(p, o, u))
    assert n1 <= n0 // 10
    assert np.abs(got - u).max() <= 10 * p.cg_rtol * np.abs(u).max()
    # and skip keeps such an iterate untouched, with no solve at all
    got, ns = f_relax_count(orc, p, dataclasses.replace(o, cg_guess=1), u, cpoints(p, o, u), skip=True)
    assert ns == 0 and np.array_equal(got, u)


@pytest.mark.parametrize("kind", [W.HEAT2D, W.AC2D])
@pytest.mark.parametrize("relax", [0, 1])
def test_solve_loop_equals_cycles_with_plain_guess(orc, kind, relax):
    # the solve loop skips the F-relaxation of an F-relaxed iterate; with the plain guess that
    # relaxation would recompute the same bits, so the loop equals F-relaxation plus whole cycles
    p, u0 = W.small_problem(kind, seed=3, nt=40, nx=6)
    o = W.Options(m=4, k=3, relax=relax, tol=0.0, max_iter=4)
    g = W.initial_guess(p, u0, "random", seed=1) * (0.3 if kind == W.AC2D else 1.0)
    g[0] = u0
    u, hist, st = orc.solve(p, o, g, allow_status=(orc.OK, orc.NOT_CONVERGED))
    ref = orc.f_relax(p, o, g)
    for _ in range(o.max_iter):
        ref = orc.cycle(p, o, ref, u0)
    assert np.array_equal(u, ref)


@pytest.mark.parametrize("kind", [W.HEAT2D, W.AC2D])
@pytest.mark.parametrize("relax", [0, 1])
def test_extrapolated_guess_solve_reaches_sequential(orc, kind, relax):
    p, u0 = W.small_problem(kind, seed=3, nt=97, nx=8)
    o = W.Options(m=4, k=3, relax=relax, tol=1e-10, max_iter=100)
    g = W.initial_guess(p, u0, "random", seed=2) * (0.3 if kind == W.AC2D else 1.0)
    g[0] = u0
    a, ha, sa = orc.solve(p, o, g)
    b, hb, sb = orc.solve(p, dataclasses.replace(o, cg_guess=1), g)
    assert sb["iterations"] == sa["iterations"]
    # every step carries a CG error of about rtol |u|: over the 97 x 64 points the residual norm has a
    # floor of about 1e-12 sqrt(6208) = 1e-10, below which the histories differ by rounding
    np.testing.assert_allclose(hb, ha, rtol=1e-6, atol=5e-10)
    assert np.abs(b - orc.sequential(p, u0)).max() <= 1e-9
