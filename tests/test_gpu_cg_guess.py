"""GPU parity of the sweeps and solves whose fine CG starts from the extrapolated
iterate (atm_options.cg_guess = 1), through the C-ABI, against the CPU oracle
with the same option.

Bars: with a CG held to a tolerance it meets at the start (cg_rtol = 1e3) a sweep
returns its guesses, the same additions on both sides: bit for bit.  With the
solves to cg_rtol 1e-14 (sweeps) or the problem's tolerance (solves), the FP64
bar of the other parity tests: 1e-12 relative to the largest magnitude.
"""
import dataclasses

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


def cpoints(p, o, u):
    return np.ascontiguousarray(u[::o.m][: p.nt // o.m + 1])


def y_of(orc, p, o, u):
    NT = p.nt // o.m
    y = np.zeros((NT + 1, p.n))
    for j in range(1, NT + 1):
        y[j] = orc.step(p, p.dt, u[j * o.m - 1])
    return y


CASES = [
    # (kind, nx, ny, nt, m)
    (W.HEAT2D, 12, 9, 24, 4),
    (W.HEAT2D, 100, 37, 18, 4),      # masked columns and rows, ragged tail
    (W.HEAT2D, 128, 128, 70, 16),    # the largest strips, ragged tail of 6 steps
    (W.HEAT2D, 64, 64, 16, 4),       # exactly tiled, no tail interval (16 = 4 * 4)
    (W.AC2D, 24, 20, 19, 3),         # periodic, ragged tail
    (W.AC2D, 33, 21, 12, 4),
]


def run_sweeps(atm, orc, case, cg_rtol, check):
    kind, nx, ny, nt, m = case
    p, u0 = W.small_problem(kind, seed=5, nt=nt, nx=nx, ny=ny, cg_rtol=cg_rtol)
    o = W.Options(m=m, k=2, relax=1, cg_guess=1)
    NT = p.nt // m
    u = W.initial_guess(p, u0, "random", seed=3) * (0.3 if kind == W.AC2D else 1.0)
    u[0] = u0
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    print(f"cg_guess sweeps kind={kind} {nx}x{ny} nt={nt} m={m} cg_rtol={cg_rtol}", flush=True)
    # mode 0: F-relaxation (the C-points do not move: the start is the stored iterate)
    ud, yd = dev(u), dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 0, ud, None, yd, ws)
    u_f = orc.f_relax(p, o, u)
    check(host(ud), u_f, "F-relaxation u")
    check(host(yd)[1:], y_of(orc, p, o, u_f)[1:], "F-relaxation y")
    # mode 2: C-relaxation from y, then F-relaxation from the moved C-points
    y2 = dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 2, ud, yd, y2, ws)
    u_cf = orc.f_relax(p, o, orc.c_relax(p, o, u_f), c_old=cpoints(p, o, u_f))
    check(host(ud), u_cf, "CF-relaxation u")
    check(host(y2)[1:], y_of(orc, p, o, u_cf)[1:], "CF-relaxation y")
    # mode 1: correction by e (C-point 2 left unchanged), then F-relaxation
    rng = np.random.default_rng(11)
    e = rng.standard_normal((NT + 1, p.n)) * 0.1
    e[0] = 0.0
    if NT >= 2:
        e[2] = 0.0
    y3 = dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 1, ud, dev(e), y3, ws)
    u_c = orc.correct(p, o, u_cf, e)
    check(host(ud), u_c, "correction u")
    check(host(y3)[1:], y_of(orc, p, o, u_c)[1:], "correction y")


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}")
def test_sweeps_return_the_guess_bitwise(atm, orc, case):
    def check(got, ref, what):
        assert np.array_equal(got, ref), f"{what}: max|diff| = {np.abs(got - ref).max():.3e}"
    run_sweeps(atm, orc, case, 1e3, check)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}")
def test_sweeps_match_oracle(atm, orc, case):
    run_sweeps(atm, orc, case, 1e-14, lambda got, ref, what: assert_close(got, ref, what=what))


@pytest.mark.parametrize("relax", [0, 1])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}")
def test_solve_iterates_match_oracle(atm, orc, case, relax):
    """After K cycles (K = 1, 3) the GPU iterate and history equal the oracle's (the solve loop skips
    the intervals whose C-point did not move on both sides)."""
    kind, nx, ny, nt, m = case
    p, u0 = W.small_problem(kind, seed=5, nt=nt, nx=nx, ny=ny, cg_rtol=1e-14)
    for K in (1, 3):
        o = W.Options(m=m, k=2, relax=relax, tol=0.0, max_iter=K, cg_guess=1,
                      coarse_substeps=2 if kind == W.AC2D else 1)
        g = W.initial_guess(p, u0, "random", seed=4) * (0.3 if kind == W.AC2D else 1.0)
        g[0] = u0
        print(f"cg_guess solve kind={kind} {nx}x{ny} nt={nt} m={m} relax={relax} K={K}", flush=True)
        ref, hist, st = orc.solve(p, o, g, allow_status=(orc.NOT_CONVERGED, orc.OK))
        ud = dev(g)
        status, ghist, gst = atm.atm_solve(p, o, ud)
        assert gst["iterations"] == st["iterations"]
        assert_close(host(ud), ref, what=f"u after {K} cycles")
        np.testing.assert_allclose(ghist, hist[: len(ghist)], rtol=1e-11, atol=1e-13 * hist[0])


@pytest.mark.parametrize("kind", [W.HEAT2D, W.AC2D])
def test_converged_solve_fewer_cg_iterations(atm, orc, kind):
    """Both starts converge to the oracle's iterate in the same number of cycles; the extrapolated one
    with fewer fine CG iterations."""
    # CG to 1e-14 as in the other parity tests: at 1e-12 the two sides' different summation orders can
    # end a step's CG one iteration apart, a difference of rtol |u| that 256 nonlinear steps carry along
    p, u0 = W.small_problem(kind, seed=6, nt=256, nx=48, ny=40, cg_rtol=1e-14)
    o0 = W.Options(m=8, k=4, relax=1, tol=1e-9, max_iter=60, coarse_substeps=2 if kind == W.AC2D else 1)
    o1 = dataclasses.replace(o0, cg_guess=1)
    g = W.initial_guess(p, u0)
    print(f"cg_guess converged solve kind={kind}", flush=True)
    ref, hist, st = orc.solve(p, o1, g)
    out = {}
    for name, o in (("plain", o0), ("extrapolated", o1)):
        ud = dev(g)
        status, ghist, gst = atm.atm_solve(p, o, ud)
        assert status == atm.ATM_OK and ghist[-1] <= o.tol
        out[name] = (host(ud), gst)
    u1, s1 = out["extrapolated"]
    assert s1["iterations"] == st["iterations"]
    assert_close(u1, ref, what="converged iterate")
    assert_close(u1, out["plain"][0], rtol=1e-10, what="extrapolated against plain start")
    assert s1["cg_fine"] < out["plain"][1]["cg_fine"]


def test_c2_full_size_extrapolated(atm, orc):
    """2D heat 128^2 x 4096, m = 32, k = 13, FCF, CG rtol 1e-12, Psi in the FP64 eigenbasis: cg_guess 1
    takes the same cycles as the plain start, returns the same iterate to the residual tolerance, needs
    fewer fine CG iterations (about 22% fewer here), and every C-point residual agrees with the oracle's
    integrator."""
    p, o, u0 = W.config("c2")
    o.coarse_solver = 0
    res = {}
    for cg in (0, 1):
        o.cg_guess = cg
        print(f"c2 full size cg_guess={cg}", flush=True)
        ud = dev(W.initial_guess(p, u0))
        status, hist, st = atm.atm_solve(p, o, ud)
        assert status == atm.ATM_OK and hist[-1] <= o.tol
        res[cg] = (host(ud), hist, st)
    (u0_, h0, s0), (u1, h1, s1) = res[0], res[1]
    assert s1["iterations"] == s0["iterations"]
    assert s1["cg_fine"] < 0.85 * s0["cg_fine"]
    # both iterates are within the residual tolerance of the sequential solution: they agree to it
    assert np.abs(u1 - u0_).max() <= 1e-7
    NT = p.nt // o.m
    r2 = 0.0
    for j in range(1, NT + 1):
        r2 += float(np.sum((orc.step(p, p.dt, u1[j * o.m - 1]) - u1[j * o.m]) ** 2))
    assert abs(np.sqrt(r2) - h1[-1]) <= 1e-3 * h1[-1] + 1e-12
