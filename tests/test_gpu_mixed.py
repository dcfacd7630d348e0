"""GPU parity of the mixed-precision form (FP32 fine solves, FP64 residual and correction)
and of the implicit-residual norms, through the C-ABI, against the CPU oracle.

Bars: the FP64 norms match the oracle to 1e-12 relative; the mixed sweeps
match the FP64 oracle to within the FP32 solve tolerance times the size of the
update; the mixed solve converges to a residual of 1e-10 and its iterate is
compared with the oracle's sequential solution (error stated in the asserts).
"""
import numpy as np
import pytest

import workloads as W
from tests.conftest import gpu_available
from tests.test_gpu_parity import CASES, assert_close, dev, host, small, y_of

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

CASES_2D = [c for c in CASES if c[0] != W.HEAT1D]
MIXED_RTOL = 1e-6  # FP32 CG tolerance of the mixed sweeps (the default)


EPS = 2.0 ** -53


def rounding_floor(p, u):
    """Rounding allowance of an FP64 implicit residual norm: every rho_i(x) = psi(u_{i-1}) - M u_i adds
    terms up to w max|u| (w = 1 + d + 2 cx + 2 cy, plus the cubic of Allen-Cahn), each rounded
    once; the errors of the nt n points add up to at most sqrt(nt n) times that in the 2-norm."""
    dt = p.dt
    per = p.kind == W.AC2D
    hx = p.length / (p.nx if per else p.nx + 1)
    cx = p.nu * dt / hx ** 2
    cy = 0.0
    if p.kind != W.HEAT1D:
        hy = p.length / (p.ny if per else p.ny + 1)
        cy = p.nu * dt / hy ** 2
    umax = float(np.max(np.abs(u)))
    w = 2.0 + 4.0 * cx + 4.0 * cy
    if per:
        w += dt / p.eps ** 2 * (1.0 + 3.0 * umax ** 2)
    return 4 * EPS * w * umax * np.sqrt(p.nt * p.n)


def ids(c):
    return f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}-k{c[5]}"


@pytest.fixture(scope="module")
def atm():
    import paper_2107_09596_amd as atm
    return atm


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_implicit_residual_norm_matches_oracle(atm, orc, case):
    kind, nx, ny, nt, m, k = case
    p, u0 = small(kind, nx, ny, nt)
    o = W.Options(m=m, k=k)
    u = W.initial_guess(p, u0, "random", seed=8) * 0.5
    u[0] = u0
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    got = atm.atm_implicit_residual_norm(p, o, dev(u), ws)
    ref = float(np.linalg.norm(orc.implicit_residual(p, u)))
    assert abs(got - ref) <= 1e-12 * ref


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_step_residual_norm_matches_oracle(atm, orc, case):
    """|M^-1 rho| on a rough iterate and on a converged one (tiny residual, no cancellation)."""
    kind, nx, ny, nt, m, k = case
    p, u0 = small(kind, nx, ny, nt)
    o = W.Options(m=m, k=k)
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    u = W.initial_guess(p, u0, "random", seed=9) * 0.5
    u[0] = u0
    got = atm.atm_step_residual_norm(p, o, dev(u), ws)
    ref = float(np.linalg.norm(orc.step_residual(p, u)))
    assert abs(got - ref) <= 1e-12 * ref
    seq = orc.sequential(p, u0)
    seq[1:] += 1e-9 * np.random.default_rng(3).standard_normal(seq[1:].shape)
    got = atm.atm_step_residual_norm(p, o, dev(seq), ws)
    ref = float(np.linalg.norm(orc.step_residual(p, seq)))
    # both solve M r = rho from zero to cg_rtol = 1e-14 relative to |rho|; rho itself is a difference
    # of O(1) terms, so the two sides differ by its rounding
    assert abs(got - ref) <= 1e-11 * ref + rounding_floor(p, seq)


def _update_bound(ref, start):
    """FP32 CG error bound of a mixed sweep: rtol times the update per step, summed over the interval,
    with a factor 10 for FP32 rounding of the right-hand side and of the CG itself."""
    return 10 * MIXED_RTOL * max(float(np.max(np.abs(ref - start))), 1e-300) * 8


@pytest.mark.parametrize("case", CASES_2D, ids=ids)
def test_mixed_sweeps_match_fp64_oracle(atm, orc, case):
    kind, nx, ny, nt, m, k = case
    p, u0 = small(kind, nx, ny, nt)
    o = W.Options(m=m, k=k, relax=1, precision=1)
    NT = p.nt // m
    u = W.initial_guess(p, u0, "random", seed=3) * (0.3 if kind == W.AC2D else 1.0)
    u[0] = u0
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    # mode 0: F-relaxation from the stored values
    ud, yd = dev(u), dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 0, ud, None, yd, ws)
    u_f = orc.f_relax(p, o, u)
    tol = _update_bound(u_f, u)
    assert np.max(np.abs(host(ud) - u_f)) <= tol, "mixed F-relaxation u"
    y_f = y_of(orc, p, o, u_f)
    assert np.max(np.abs(host(yd)[1:] - y_f[1:])) <= tol, "mixed F-relaxation y"
    # mode 2: C-relaxation from y (the Phi values of the last sweep start the new ones)
    y2 = dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 2, ud, yd, y2, ws)
    u_cf = orc.f_relax(p, o, orc.c_relax(p, o, u_f))
    tol2 = _update_bound(u_cf, u_f) + tol
    assert np.max(np.abs(host(ud) - u_cf)) <= tol2, "mixed CF-relaxation u"
    assert np.max(np.abs(host(y2)[1:] - y_of(orc, p, o, u_cf)[1:])) <= tol2, "mixed CF-relaxation y"
    # mode 1: correction, y in/out (its entries start the steps that produce it)
    rng = np.random.default_rng(11)
    e = rng.standard_normal((NT + 1, p.n)) * 0.1
    e[0] = 0.0
    atm.atm_sweep(p, o, 1, ud, dev(e), y2, ws)
    u_c = orc.correct(p, o, u_cf, e)
    tol3 = _update_bound(u_c, u_cf) + tol2
    assert np.max(np.abs(host(ud) - u_c)) <= tol3, "mixed correction u"
    assert np.max(np.abs(host(y2)[1:] - y_of(orc, p, o, u_c)[1:])) <= tol3, "mixed correction y"


@pytest.mark.parametrize("case", CASES_2D, ids=ids)
def test_mixed_sweep_keeps_the_fp64_solution(atm, orc, case):
    """Started from the sequential solution, a mixed sweep moves nothing beyond FP64 rounding:
    the FP64 defect is at rounding level, so the FP32 correction is too."""
    kind, nx, ny, nt, m, k = case
    p, u0 = small(kind, nx, ny, nt)
    o = W.Options(m=m, k=k, precision=1)
    NT = p.nt // m
    seq = orc.sequential(p, u0)
    ud, yd = dev(seq), dev(np.zeros((NT + 1, p.n)))
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    atm.atm_sweep(p, o, 0, ud, None, yd, ws)
    assert_close(host(ud), seq, rtol=1e-13, what="F-points of the sequential solution")
    assert_close(host(yd)[1:], seq[[j * m for j in range(1, NT + 1)]], rtol=1e-13, what="y at the C-points")


FLOOR_CASES = [
    # (kind, nx, ny, nt, m): the strip sweep, the large-grid sweep and the paired sweep
    (W.AC2D, 32, 32, 24, 4),
    (W.HEAT2D, 40, 24, 20, 4),
    (W.AC2D, 320, 64, 8, 4),
    (W.AC2D, 256, 256, 8, 4),
]


@pytest.mark.parametrize("case", FLOOR_CASES, ids=lambda c: f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}")
def test_rounding_level_defects_take_no_correction(atm, orc, case):
    """Repeated F-relaxations of the oracle's sequential solution with its F-points perturbed: the first
    corrects them; once their defects are at the rounding level of their own FP64 evaluation those steps
    take no correction, so the iterate keeps its bits and the CG count settles to that of the steps that
    form Phi of each interval's last F-point against the C-point that follows (unchanged by
    F-relaxation, with the oracle's own CG error)."""
    kind, nx, ny, nt, m = case
    p, u0 = small(kind, nx, ny, nt)
    o = W.Options(m=m, k=2, relax=1, precision=1, tol=0.0, max_iter=0)
    seq = orc.sequential(p, u0)
    g = seq.copy()
    rng = np.random.default_rng(11)
    for t in range(1, p.nt + 1):
        if t % m:
            g[t] += 1e-9 * np.max(np.abs(seq)) * rng.standard_normal(p.n)
    ud = dev(g)
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    counts, changed = [], []
    prev = host(ud)
    for _ in range(4):
        _, _, st = atm.atm_solve(p, o, ud, ws=ws, allow=(atm.ATM_OK, atm.ATM_NOT_CONVERGED))
        counts.append(st["cg_fine"])
        cur = host(ud)
        changed.append(not np.array_equal(cur, prev))
        prev = cur
    print(f"floor {case}: CG iterations per F-relaxation {counts}, iterate changed {changed}", flush=True)
    assert changed[0] and not changed[-1]
    assert counts[0] > counts[-1] == counts[-2]
    np.testing.assert_allclose(prev, seq, rtol=0, atol=1e-12 * np.max(np.abs(seq)))


MIXED_SOLVES = [
    # (kind, nx, ny, nt, m, k, relax)
    (W.HEAT2D, 64, 64, 96, 8, 3, 1),
    (W.HEAT2D, 100, 37, 50, 4, 4, 0),     # masked strips, ragged tail, F-relaxation
    (W.HEAT2D, 128, 128, 64, 8, 2, 1),
    (W.AC2D, 24, 20, 61, 4, 3, 1),        # ragged tail, FAS
    (W.AC2D, 32, 32, 64, 8, 2, 0),
]


@pytest.mark.parametrize("case", MIXED_SOLVES, ids=lambda c: ids(c) + f"-r{c[6]}")
def test_mixed_solve_converges_to_fp64_solution(atm, orc, case):
    kind, nx, ny, nt, m, k, relax = case
    p, u0 = small(kind, nx, ny, nt)
    tol = 1e-10
    sub = 2 if kind == W.AC2D else 1
    o = W.Options(m=m, k=k, relax=relax, tol=tol, precision=1, max_iter=60, coarse_substeps=sub)
    ud = dev(W.initial_guess(p, u0))
    status, hist, st = atm.atm_solve(p, o, ud)
    assert status == atm.ATM_OK and hist[-1] <= tol
    u = host(ud)
    floor = rounding_floor(p, u)
    # the reported paper-form residual is the oracle's |M^-1 rho| of the returned iterate
    ref_r = float(np.linalg.norm(orc.step_residual(p, u)))
    ref_rho = float(np.linalg.norm(orc.implicit_residual(p, u)))
    seq = orc.sequential(p, u0)
    err = float(np.linalg.norm(u - seq))
    print(f"stop {hist[-1]:.3e} (oracle {ref_rho:.3e}), |r| {st['final_residual']:.3e} (oracle {ref_r:.3e}), "
          f"floor {floor:.1e}, |u - u_seq| {err:.3e}, cycles {st['iterations']}")
    assert abs(st["final_residual"] - ref_r) <= 1e-8 * ref_r + floor
    assert st["final_residual"] <= hist[-1] * (1 + 1e-12) + floor
    # the stopping norm is the oracle's implicit residual of the returned iterate
    assert abs(hist[-1] - ref_rho) <= 1e-12 * ref_rho + floor
    # error against the FP64 sequential solution (cg_rtol 1e-14): |u - u*| <= |A^-1| |r| <= (nt + 1) |r|
    # (|Phi| <= 1 for heat; the Allen-Cahn cases stay within the same bound)
    assert err <= (p.nt + 1) * (ref_r + floor + 1e-13 * float(np.linalg.norm(seq)))
    # the FP32 fine solves cost at most a couple of cycles against the FP64 form
    o64 = W.Options(**{**o.__dict__, "precision": 0})
    _, h64, st64 = atm.atm_solve(p, o64, dev(W.initial_guess(p, u0)))
    assert st["iterations"] <= st64["iterations"] + 2
    assert st["fine_steps_skipped"] == 0  # FP32 sweeps refine their F-points every time


def test_mixed_deterministic_bitwise(atm):
    p, u0 = small(W.HEAT2D, 64, 64, 32)
    o = W.Options(m=4, k=2, tol=1e-10, precision=1)
    a = dev(W.initial_guess(p, u0))
    b = dev(W.initial_guess(p, u0))
    _, ha, _ = atm.atm_solve(p, o, a)
    _, hb, _ = atm.atm_solve(p, o, b)
    assert np.array_equal(host(a), host(b)) and ha == hb


def test_c2_mixed_full_size(atm, orc):
    """2D heat 128^2 x 4096, m = 32, k = 13, FCF, FP32 fine solves: converge to 1e-10 on the GPU; the stopping
    norm equals the oracle's implicit residual of the result; the paper-form residual is bracketed by it;
    sampled slices match the FP64 oracle's sequential stepping."""
    p, o, u0 = W.config("c2")
    o.precision = 1
    o.tol = 1e-10
    o.coarse_cg_rtol = 1e-6
    ud = dev(W.initial_guess(p, u0))
    status, hist, st = atm.atm_solve(p, o, ud)
    assert status == atm.ATM_OK and hist[-1] <= o.tol
    u = host(ud)
    floor = rounding_floor(p, u)
    rho = float(np.linalg.norm(orc.implicit_residual(p, u)))
    print(f"stop {hist[-1]:.3e} (oracle {rho:.3e}), |r| {st['final_residual']:.3e}, floor {floor:.1e}, "
          f"cycles {st['iterations']}")
    assert abs(hist[-1] - rho) <= 1e-12 * rho + floor
    # |r| <= |rho| <= |M| |r|, |M| <= 1 + 8 c (Gershgorin)
    c = p.nu * p.dt / (p.length / (p.nx + 1)) ** 2
    assert (rho - floor) / (1 + 8 * c) * (1 - 1e-9) <= st["final_residual"] <= rho * (1 + 1e-12) + floor
    q = W.Problem(**{**p.__dict__, "nt": 256, "tf": p.t0 + 256 * p.dt, "cg_rtol": 1e-14})
    ref = orc.sequential(q, u0)
    err = float(np.max(np.abs(u[:257] - ref)))
    assert err <= 1e-9, f"max error against the FP64 oracle on the first 256 steps: {err:.2e}"


@pytest.mark.parametrize("solver", [0, 2], ids=["psi-fp64-eigenbasis", "psi-bf16-eigenbasis-fas-in-e"])
def test_c5_full_size(atm, orc, solver):
    """2D Allen-Cahn 128x128 periodic, eps 0.03, dt 1e-5, Nt 4096, m 32, k 13, FCF, FP32 fine solves, Psi in the
    FP64 eigenbasis (the benchmarked plain solve of the learned-propagator comparison) or on the BF16 matrix cores
    (FAS in terms of e = w - v), to the reduced-precision bar 1e-10: the stopping norm is the oracle's implicit
    residual of the result, the paper-form residual is bracketed by it, and the first 64 steps match the
    oracle's sequential stepping (its error is printed)."""
    p, o, u0 = W.config("c5")
    o.coarse_solver = solver
    o.tol = 1e-10
    ud = dev(W.initial_guess(p, u0))
    status, hist, st = atm.atm_solve(p, o, ud)
    u = host(ud)
    floor = rounding_floor(p, u)
    rho = float(np.linalg.norm(orc.implicit_residual(p, u)))
    q = W.Problem(**{**p.__dict__, "nt": 64, "tf": p.t0 + 64 * p.dt, "cg_rtol": 1e-14})
    err = float(np.max(np.abs(u[:65] - orc.sequential(q, u0))))
    print(f"cycles {st['iterations']}, stopping norm {hist[-1]:.3e} (oracle {rho:.3e}, floor {floor:.1e}), "
          f"paper-form {st['final_residual']:.3e}, error against the FP64 oracle on the first 64 steps {err:.2e}")
    assert status == atm.ATM_OK and hist[-1] <= 1e-10
    assert abs(hist[-1] - rho) <= 1e-12 * rho + floor
    assert st["final_residual"] <= hist[-1] * (1 + 1e-9) + floor
    assert err <= 1e-9, f"max error against the FP64 oracle on the first 64 steps: {err:.2e}"
