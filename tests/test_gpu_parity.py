"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

FP64 bar (the benchmark spec): 1e-12 relative, element by element, scaled by the
largest magnitude of the reference (the iterates cross zero, so a pure
pointwise relative bound is undefined there).  Iterate-by-iterate parity of
CG-based integrators uses cg_rtol = 1e-14 on both sides (two CG runs with
different summation orders otherwise differ by up to rtol per step); the
configured-rtol runs are judged at full size by sampled outputs and by the
oracle's own residual of the GPU result.
"""
import numpy as np
import pytest

import workloads as W
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

RTOL = 1e-12


@pytest.fixture(scope="module")
def atm():
    import paper_2107_09596_amd as atm
    return atm


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def assert_close(got, ref, rtol=RTOL, what=""):
    scale = max(float(np.max(np.abs(ref))), 1e-300)
    err = float(np.max(np.abs(got - ref)))
    assert err <= rtol * scale, f"{what}: max|diff| = {err:.3e} > {rtol:.1e} * {scale:.3e}"


def y_of(orc, p, o, u):
    """y_j = Phi(u_{jm-1}) for j = 1..N_T (row 0 zero), from the oracle's integrator."""
    NT = p.nt // o.m
    y = np.zeros((NT + 1, p.n))
    for j in range(1, NT + 1):
        y[j] = orc.step(p, p.dt, u[j * o.m - 1])
    return y


CASES = [
    # (kind, nx, ny, nt, m, k)
    (W.HEAT1D, 7, 1, 40, 4, 3),
    (W.HEAT1D, 63, 1, 64, 16, 2),
    (W.HEAT1D, 100, 1, 45, 4, 5),        # ragged tail: 45 = 11 * 4 + 1
    (W.HEAT2D, 12, 9, 24, 4, 2),
    (W.HEAT2D, 64, 64, 16, 4, 3),        # exactly tiled strips
    (W.HEAT2D, 100, 37, 18, 4, 2),       # masked columns and rows, ragged tail
    (W.HEAT2D, 128, 128, 8, 4, 2),       # the largest grid
    (W.AC2D, 16, 16, 24, 4, 3),
    (W.AC2D, 24, 20, 19, 3, 2),          # ragged tail
    (W.AC2D, 33, 21, 12, 4, 2),          # odd ny: a strip chunk is cut by the periodic halo row
]


def small(kind, nx, ny, nt, seed=5):
    if kind == W.HEAT1D:
        p, u0 = W.small_problem(kind, seed=seed, nt=nt, nx=nx)
    else:
        p, u0 = W.small_problem(kind, seed=seed, nt=nt, nx=nx, ny=ny, cg_rtol=1e-14)
    return p, u0


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}-k{c[5]}")
def test_sweeps_match_oracle(atm, orc, case):
    kind, nx, ny, nt, m, k = case
    p, u0 = small(kind, nx, ny, nt)
    o = W.Options(m=m, k=k, relax=1)
    NT = p.nt // m
    u = W.initial_guess(p, u0, "random", seed=3) * (0.3 if kind == W.AC2D else 1.0)
    u[0] = u0
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    # mode 0: F-relaxation
    ud, yd = dev(u), dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 0, ud, None, yd, ws)
    u_f = orc.f_relax(p, o, u)
    assert_close(host(ud), u_f, what="F-relaxation u")
    y_f = y_of(orc, p, o, u_f)
    assert_close(host(yd)[1:], y_f[1:], what="F-relaxation y")
    # mode 2: C-relaxation from y, then F-relaxation
    y2 = dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 2, ud, yd, y2, ws)
    u_cf = orc.f_relax(p, o, orc.c_relax(p, o, u_f))
    assert_close(host(ud), u_cf, what="CF-relaxation u")
    assert_close(host(y2)[1:], y_of(orc, p, o, u_cf)[1:], what="CF-relaxation y")
    # mode 1: correction by e then F-interpolation
    rng = np.random.default_rng(11)
    e = rng.standard_normal((NT + 1, p.n)) * 0.1
    e[0] = 0.0
    y3 = dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 1, ud, dev(e), y3, ws)
    u_c = orc.correct(p, o, u_cf, e)
    assert_close(host(ud), u_c, what="correction u")
    assert_close(host(y3)[1:], y_of(orc, p, o, u_c)[1:], what="correction y")


@pytest.mark.parametrize("solver", [(0, 0.0), (1, 0.0), (1, 1e-13)], ids=["eigenbasis", "cg", "cg-1e-13"])
@pytest.mark.parametrize("form", [1, 2])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}-k{c[5]}")
def test_coarse_solves_match_oracle(atm, orc, case, form, solver):
    """Psi's implicit solve in the eigenbasis (exact to rounding) or by CG (to the problem's rtol 1e-14, or 1e-13):
    the windows match the oracle's local solves (its Psi by CG to rtol 1e-14)."""
    kind, nx, ny, nt, m, k = case
    p, u0 = small(kind, nx, ny, nt)
    o = W.Options(m=m, k=k, relax=1, coarse_form=form, coarse_substeps=2 if kind == W.AC2D else 1,
                  coarse_solver=solver[0], coarse_cg_rtol=solver[1])
    NT = p.nt // m
    g = W.initial_guess(p, u0, "random", seed=4) * 0.5
    g[0] = u0
    u = orc.f_relax(p, o, g)
    y = y_of(orc, p, o, u)
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    ed = dev(np.zeros((NT + 1, p.n)))
    atm.atm_coarse_solve(p, o, dev(u), dev(y), ed, ws)
    vc = np.stack([u[j * m] for j in range(NT + 1)])
    rc = y - vc
    rc[0] = 0.0
    assert_close(host(ed), orc.local_solves(p, o, rc, vc), what="local coarse solves")


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}-k{c[5]}")
def test_residual_norm_matches_oracle(atm, orc, case):
    kind, nx, ny, nt, m, k = case
    p, u0 = small(kind, nx, ny, nt)
    o = W.Options(m=m, k=k)
    g = W.initial_guess(p, u0, "random", seed=6) * 0.5
    g[0] = u0
    u = orc.f_relax(p, o, g)
    y = y_of(orc, p, o, u)
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    got = atm.atm_residual_norm(p, o, dev(u), dev(y), ws)
    ref = orc.residual_norm(p, u, u0)
    assert abs(got - ref) <= 1e-12 * ref


@pytest.mark.parametrize("relax", [0, 1])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}-k{c[5]}")
def test_solve_iterates_match_oracle(atm, orc, case, relax):
    """After K cycles (K = 1, 3) the GPU iterate and history equal the oracle's."""
    kind, nx, ny, nt, m, k = case
    p, u0 = small(kind, nx, ny, nt)
    for K in (1, 3):
        o = W.Options(m=m, k=k, relax=relax, tol=0.0, max_iter=K, coarse_substeps=2 if kind == W.AC2D else 1)
        g = W.initial_guess(p, u0)
        ref, hist, st = orc.solve(p, o, g, allow_status=(orc.NOT_CONVERGED, orc.OK))
        ud = dev(g)
        status, ghist, gst = atm.atm_solve(p, o, ud)
        assert gst["iterations"] == st["iterations"]
        assert_close(host(ud), ref, what=f"u after {K} cycles")
        # residual norms agree to 1e-11 relative, down to a floor of 1e-13 of the initial residual
        # (small problems converge exactly, after which both sides print rounding noise)
        np.testing.assert_allclose(ghist, hist[: len(ghist)], rtol=1e-11, atol=1e-13 * hist[0])


@pytest.mark.parametrize("kind,nx,ny,nt", [(W.HEAT1D, 63, 1, 50), (W.HEAT2D, 40, 33, 12), (W.AC2D, 20, 20, 15),
                                           (W.HEAT2D, 128, 128, 6)])
def test_sequential_matches_oracle(atm, orc, kind, nx, ny, nt):
    p, u0 = small(kind, nx, ny, nt)
    u = np.zeros((p.nt + 1, p.n))
    u[0] = u0
    ud = dev(u)
    atm.atm_sequential(p, ud)
    assert_close(host(ud), orc.sequential(p, u0), what="sequential stepping")


def test_c1_full_solve_matches_oracle(atm, orc):
    """1D heat 63 x 1024, m = 16, FCF, tol 1e-8: same iterations, iterate within 1e-12."""
    p, o, u0 = W.config("c1")
    g = W.initial_guess(p, u0)
    ref, hist, st = orc.solve(p, o, g)
    ud = dev(g)
    status, ghist, gst = atm.atm_solve(p, o, ud)
    assert status == atm.ATM_OK
    assert gst["iterations"] == st["iterations"]
    assert ghist[-1] <= o.tol
    assert_close(host(ud), ref, what="c1 converged iterate")
    np.testing.assert_allclose(ghist, hist, rtol=1e-10)
    # intervals whose C-point no longer changes are not recomputed (the oracle recomputes them; the
    # F-relaxation of an F-relaxed interval reproduces it bit for bit), and the step accounting adds up
    assert gst["fine_steps_skipped"] > 0
    assert gst["fine_steps"] + gst["fine_steps_skipped"] == gst["n_sweeps"] * p.nt


@pytest.mark.parametrize("k", [1, 2, 65, 200])
def test_c1_k_extremes(atm, orc, k):
    """k = 1 (C-relaxation only), Parareal k = N_T + 1, and k beyond it."""
    p, o, u0 = W.config("c1")
    o.k = k
    o.max_iter = 4
    o.tol = 0.0
    g = W.initial_guess(p, u0)
    ref, hist, st = orc.solve(p, o, g, allow_status=(orc.NOT_CONVERGED,))
    ud = dev(g)
    atm.atm_solve(p, o, ud)
    assert_close(host(ud), ref, what=f"c1 k={k}")


@pytest.mark.parametrize("solver", [1, 2], ids=["psi-cg-1e-3", "psi-bf16-eigenbasis"])
def test_c2_full_size_sampled(atm, orc, solver):
    """2D heat 128^2 x 4096, m = 32, FCF, CG rtol 1e-12, Psi by CG to 1e-3 or in the eigenbasis on the BF16
    matrix cores (the benchmarked launches): converge on the GPU, then check sampled intervals and every
    C-point residual with the oracle's integrator."""
    p, o, u0 = W.config("c2")
    o.coarse_solver, o.coarse_cg_rtol = solver, 1e-3
    ud = dev(W.initial_guess(p, u0))
    status, hist, st = atm.atm_solve(p, o, ud)
    assert status == atm.ATM_OK and hist[-1] <= o.tol
    u = host(ud)
    NT = p.nt // o.m
    # every C-point residual r_j = Phi(u_{jm-1}) - u_{jm}; F-point residuals of sampled intervals
    r2 = 0.0
    for j in range(1, NT + 1):
        r2 += float(np.sum((orc.step(p, p.dt, u[j * o.m - 1]) - u[j * o.m]) ** 2))
    assert abs(np.sqrt(r2) - hist[-1]) <= 1e-3 * hist[-1] + 1e-12
    rng = np.random.default_rng(0)
    for j in sorted(rng.choice(NT, size=4, replace=False)):
        x = u[j * o.m].copy()
        for i in range(1, o.m):
            x = orc.step(p, p.dt, x)
            # each step's CG (either side, from its own starting value) stops at |b - M x| <= rtol |b|
            # with |M^-1| <= 1, so it is within rtol |b| of the exact step, |b| <= |u_{jm}| for heat;
            # the errors of i steps add up (Phi does not amplify them)
            err = float(np.linalg.norm(u[j * o.m + i] - x))
            bound = 2 * i * p.cg_rtol * float(np.linalg.norm(u[j * o.m]))
            assert err <= bound, f"c2 interval {j} step {i}: |diff| = {err:.3e} > {bound:.3e}"
    # the converged iterate is the sequential solution up to the residual tolerance
    q = W.Problem(**{**p.__dict__, "nt": 256, "tf": p.t0 + 256 * p.dt})
    ref = orc.sequential(q, u0)
    assert np.max(np.abs(u[:257] - ref)) <= 1e-7


def test_deterministic_bitwise(atm):
    p, o, u0 = W.config("c1")
    a = dev(W.initial_guess(p, u0))
    b = dev(W.initial_guess(p, u0))
    atm.atm_solve(p, o, a)
    atm.atm_solve(p, o, b)
    assert np.array_equal(host(a), host(b))
    p, u0 = small(W.HEAT2D, 64, 64, 16)
    o = W.Options(m=4, k=2, tol=1e-10)
    a = dev(W.initial_guess(p, u0))
    b = dev(W.initial_guess(p, u0))
    atm.atm_solve(p, o, a)
    atm.atm_solve(p, o, b)
    assert np.array_equal(host(a), host(b))


def test_error_paths(atm):
    p, u0 = small(W.HEAT2D, 16, 16, 16)
    p.cg_max_iter = 1
    o = W.Options(m=4, k=2)
    with pytest.raises(atm.AtmError) as ei:
        atm.atm_solve(p, o, dev(W.initial_guess(p, u0)))
    assert ei.value.status == atm.ATM_ERR_INNER_SOLVE
    p, o, u0 = W.config("c1")
    o.max_iter = 2
    o.tol = 1e-14
    status, hist, st = atm.atm_solve(p, o, dev(W.initial_guess(p, u0)))
    assert status == atm.ATM_NOT_CONVERGED and st["iterations"] == 2 and len(hist) == 3
    g = W.initial_guess(p, u0)
    g[16 * 3, 5] = np.nan
    with pytest.raises(atm.AtmError) as ei:
        atm.atm_solve(p, W.Options(m=16, k=7), dev(g))
    assert ei.value.status == atm.ATM_ERR_DIVERGED


def test_c2_loose_coarse_tolerance_same_fixed_point(atm, orc):
    """Psi by CG to coarse_cg_rtol = 1e-6: same cycle count as the strict solve on the 2D heat workload, and
    the result still has a residual below tol by the oracle's own integrator."""
    p, o, u0 = W.config("c2")
    o.coarse_solver = 1
    strict = dev(W.initial_guess(p, u0))
    _, hs, ss = atm.atm_solve(p, o, strict)
    o.coarse_cg_rtol = 1e-6
    loose = dev(W.initial_guess(p, u0))
    _, hl, sl = atm.atm_solve(p, o, loose)
    assert sl["iterations"] == ss["iterations"] and hl[-1] <= o.tol
    u = host(loose)
    NT = p.nt // o.m
    r2 = sum(float(np.sum((orc.step(p, p.dt, u[j * o.m - 1]) - u[j * o.m]) ** 2)) for j in range(1, NT + 1))
    assert np.sqrt(r2) <= o.tol
    assert np.max(np.abs(u - host(strict))) <= 1e-7


# ---------------------------------------------------------------------------
# Psi in the eigenbasis on the BF16 matrix cores (coarse_solver 2): split operands give about 2^-17
# per product and per rounded stage; four stages with orthonormal bases and mu >= 1 keep one step
# within 10 * 2^-17 < 1e-4 of the exact step, relative in the 2-norm
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny,sub", [(32, 32, 1), (64, 96, 1), (128, 128, 1), (64, 96, 2), (128, 32, 3),
                                       (12, 9, 1), (100, 37, 1), (33, 128, 2), (127, 65, 1)])
def test_bf16_eigenbasis_psi_step(atm, orc, nx, ny, sub):
    """One window step e_p = Psi(r_{p-1}) + r_p (k = 2); with s substeps the errors of s steps add up
    (Psi does not amplify them)."""
    p, u0 = W.small_problem(W.HEAT2D, seed=6, nt=40, nx=nx, ny=ny, cg_rtol=1e-14)
    o = W.Options(m=4, k=2, relax=1, coarse_form=1, coarse_solver=2, coarse_substeps=sub)
    NT = p.nt // o.m
    rng = np.random.default_rng(3)
    u = rng.standard_normal((p.nt + 1, p.n))
    u[0] = u0
    y = rng.standard_normal((NT + 1, p.n))
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    ed = dev(np.zeros((NT + 1, p.n)))
    atm.atm_coarse_solve(p, o, dev(u), dev(y), ed, ws)
    got = host(ed)
    rc = np.zeros((NT + 1, p.n))
    for j in range(1, NT + 1):
        rc[j] = y[j] - u[j * o.m]
    ref = orc.local_solves(p, W.Options(m=4, k=2, coarse_form=1, coarse_substeps=sub), rc, u[:: o.m][: NT + 1])
    for pp in range(2, NT + 1):  # window p: e_p = Psi(r_{p-1}) + r_p
        err = np.linalg.norm(got[pp] - ref[pp])
        assert err <= sub * 1e-4 * np.linalg.norm(rc[pp - 1]), f"window {pp}: {err:.3e}"


def test_bf16_eigenbasis_psi_same_fixed_point(atm, orc):
    """A solve with the BF16 Psi converges to the oracle's fixed point (the fine problem's solution)."""
    p, u0 = W.small_problem(W.HEAT2D, seed=7, nt=64, nx=64, ny=64, cg_rtol=1e-14)
    o = W.Options(m=4, k=3, relax=1, tol=1e-10, max_iter=60, coarse_solver=2)
    g = W.initial_guess(p, u0)
    ref, hist, st = orc.solve(p, W.Options(**{**o.__dict__, "coarse_solver": 1}), g)
    ud = dev(g)
    status, ghist, gst = atm.atm_solve(p, o, ud)
    assert status == atm.ATM_OK and ghist[-1] <= o.tol
    assert gst["iterations"] <= st["iterations"] + 1
    # both iterates have residual <= tol; |u - u*| <= (nt + 1) |r| (|Phi| <= 1)
    assert np.sqrt(np.sum((host(ud) - ref) ** 2)) <= 2 * (p.nt + 1) * o.tol


def test_bf16_eigenbasis_psi_fas_step(atm, orc):
    """FAS windows on the BF16 matrix cores carry e = w - v: with k = 2, window p returns
    e_p = Psi(v_{p-1} + r_{p-1}) - Psi(v_{p-1}) + r_p = M^-1 d + r_p, d = psi(v + r) - psi(v) the explicit
    parts' difference, whose solve is within 1e-4 |d| (as for the linear form)."""
    p, u0 = W.small_problem(W.AC2D, seed=6, nt=40, nx=64, ny=48, cg_rtol=1e-14, eps=0.1)
    o = W.Options(m=4, k=2, relax=1, coarse_form=2, coarse_solver=2)
    NT = p.nt // o.m
    rng = np.random.default_rng(5)
    u = 0.5 * rng.standard_normal((p.nt + 1, p.n))
    u[0] = u0
    y = u[:: o.m][: NT + 1] + 0.1 * rng.standard_normal((NT + 1, p.n))
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    ed = dev(np.zeros((NT + 1, p.n)))
    atm.atm_coarse_solve(p, o, dev(u), dev(y), ed, ws)
    got = host(ed)
    vc = u[:: o.m][: NT + 1]
    rc = np.zeros((NT + 1, p.n))
    for j in range(1, NT + 1):
        rc[j] = y[j] - vc[j]
    ref = orc.local_solves(p, W.Options(m=4, k=2, coarse_form=2), rc, vc)
    react = p.dt * o.m / p.eps ** 2
    for pp in range(2, NT + 1):
        v, r = vc[pp - 1], rc[pp - 1]
        d = (r + react * ((v + r) - (v + r) ** 3)) - react * (v - v ** 3)
        err = np.linalg.norm(got[pp] - ref[pp])
        assert err <= 1e-4 * np.linalg.norm(d), f"window {pp}: {err:.3e} > 1e-4 * {np.linalg.norm(d):.3e}"


def test_bf16_eigenbasis_psi_fas_same_fixed_point(atm, orc):
    p, u0 = W.small_problem(W.AC2D, seed=7, nt=64, nx=32, ny=32, cg_rtol=1e-14)
    o = W.Options(m=4, k=3, relax=1, tol=1e-10, max_iter=60, coarse_form=2, coarse_solver=2)
    g = W.initial_guess(p, u0)
    ref, hist, st = orc.solve(p, W.Options(**{**o.__dict__, "coarse_solver": 1}), g)
    ud = dev(g)
    status, ghist, gst = atm.atm_solve(p, o, ud)
    assert status == atm.ATM_OK and ghist[-1] <= o.tol
    assert gst["iterations"] <= st["iterations"] + 1
    assert np.sqrt(np.sum((host(ud) - ref) ** 2)) <= 2 * (p.nt + 1) * o.tol
