"""The FP32-fine sweeps on two workgroups per interval (sweep_pair_mixed_kernel: 256 x 256, 256 x 128 and
128 x 256 grids) through the C-ABI, against the FP64 CPU oracle: every sweep mode within the FP32 CG's
error bound, the FP64 sequential solution kept to rounding, and solves that converge to the oracle's
fixed point at the 1e-10 bar, with the error against its sequential stepping stated."""
import numpy as np
import pytest

import workloads as W
from tests.conftest import gpu_available
from tests.test_gpu_mixed import MIXED_RTOL, rounding_floor
from tests.test_gpu_parity import assert_close, dev, host, y_of

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

PAIR = [
    # (kind, nx, ny, nt, m, k, dt nu / h^2): step sizes of the order of the workloads', where the step
    # operator's condition number is about 1 + 8 dt nu / h^2 and an FP32 CG can reach its 1e-6
    (W.AC2D, 256, 256, 12, 4, 2, 0.655),   # the 2D Allen-Cahn grid: periodic both ways
    (W.HEAT2D, 256, 128, 9, 4, 3, 1.0),    # Dirichlet, ragged tail
    (W.AC2D, 128, 256, 10, 3, 2, 0.5),     # periodic, ragged tail
    (W.HEAT2D, 256, 256, 8, 4, 2, 0.8),    # Dirichlet on the 256 x 256 grid
]


def ids(c):
    return f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}"


def problem(case, nt=None):
    """The case's problem: 2D heat (nu 0.1, the c2 recipe's field) or 2D Allen-Cahn (eps 0.05, U[-0.5, 0.5]
    field) with the step dt that gives its dt nu / h^2; CG at rtol 1e-14 in the oracle's FP64 steps (the
    iterate-parity setting), so that its sequential solution has a defect at rounding level."""
    kind, nx, ny, nt0, m, k, c = case
    nt = nt0 if nt is None else nt
    if kind == W.AC2D:
        dt = c / nx ** 2
        p, u0 = W.small_problem(W.AC2D, seed=7, nt=nt, nx=nx, ny=ny, eps=0.05, tf=nt * dt, cg_rtol=1e-14)
    else:
        dt = c / (0.1 * (nx + 1) ** 2)
        p, u0 = W.small_problem(W.HEAT2D, seed=8, nt=nt, nx=nx, ny=ny, tf=nt * dt, cg_rtol=1e-14)
    return p, u0


@pytest.fixture(scope="module")
def atm():
    import paper_2107_09596_amd as atm
    return atm


def update_bound(ref, start):
    """The FP32 CG's error in a mixed sweep: its tolerance times the update per step, summed over an
    interval, with a factor 10 for the FP32 rounding of the right-hand side and of the CG itself."""
    return 10 * MIXED_RTOL * max(float(np.max(np.abs(ref - start))), 1e-300) * 8


@pytest.mark.parametrize("case", PAIR, ids=ids)
def test_pair_kernel_is_taken(atm, case):
    kind, nx, ny, nt, m, k, _ = case
    p, _ = problem(case)
    assert atm.atm_sweep_kernel(p, W.Options(m=m, k=k, precision=1)) == "sweep_pair_mixed_kernel"
    assert atm.atm_sweep_kernel(p, W.Options(m=m, k=k, precision=0)) == "sweep_large_kernel"


@pytest.mark.parametrize("case", PAIR, ids=ids)
def test_pair_sweeps_match_fp64_oracle(atm, orc, case):
    kind, nx, ny, nt, m, k, _ = case
    p, u0 = problem(case)
    o = W.Options(m=m, k=k, relax=1, precision=1)
    NT = p.nt // m
    u = W.initial_guess(p, u0, "random", seed=3) * (0.3 if kind == W.AC2D else 1.0)
    u[0] = u0
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    ud, yd = dev(u), dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 0, ud, None, yd, ws)
    u_f = orc.f_relax(p, o, u)
    tol = update_bound(u_f, u)
    assert np.max(np.abs(host(ud) - u_f)) <= tol, "F-relaxation u"
    assert np.max(np.abs(host(yd)[1:] - y_of(orc, p, o, u_f)[1:])) <= tol, "F-relaxation y"
    y2 = dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 2, ud, yd, y2, ws)
    u_cf = orc.f_relax(p, o, orc.c_relax(p, o, u_f))
    tol2 = update_bound(u_cf, u_f) + tol
    assert np.max(np.abs(host(ud) - u_cf)) <= tol2, "CF-relaxation u"
    assert np.max(np.abs(host(y2)[1:] - y_of(orc, p, o, u_cf)[1:])) <= tol2, "CF-relaxation y"
    e = np.random.default_rng(11).standard_normal((NT + 1, p.n)) * 0.1
    e[0] = 0.0
    atm.atm_sweep(p, o, 1, ud, dev(e), y2, ws)
    u_c = orc.correct(p, o, u_cf, e)
    tol3 = update_bound(u_c, u_cf) + tol2
    assert np.max(np.abs(host(ud) - u_c)) <= tol3, "correction u"
    assert np.max(np.abs(host(y2)[1:] - y_of(orc, p, o, u_c)[1:])) <= tol3, "correction y"


@pytest.mark.parametrize("case", PAIR, ids=ids)
def test_pair_sweep_keeps_the_fp64_solution(atm, orc, case):
    """From the sequential solution the FP64 defect is at rounding level, and so is every change."""
    kind, nx, ny, nt, m, k, _ = case
    p, u0 = problem(case)
    o = W.Options(m=m, k=k, precision=1)
    NT = p.nt // m
    seq = orc.sequential(p, u0)
    ud, yd = dev(seq), dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 0, ud, None, yd, atm.workspace(atm.atm_workspace_bytes(p, o)))
    assert_close(host(ud), seq, rtol=1e-13, what="F-points of the sequential solution")
    assert_close(host(yd)[1:], seq[[j * m for j in range(1, NT + 1)]], rtol=1e-13, what="y at the C-points")


@pytest.mark.parametrize("case", PAIR[:3], ids=ids)
def test_pair_solve_converges_to_fp64_solution(atm, orc, case):
    kind, nx, ny, nt, m, k, _ = case
    p, u0 = problem(case, nt * 4)
    o = W.Options(m=m, k=k, relax=1, tol=1e-10, precision=1, max_iter=60, coarse_substeps=2 if kind == W.AC2D else 1)
    ud = dev(W.initial_guess(p, u0))
    status, hist, st = atm.atm_solve(p, o, ud)
    u = host(ud)
    floor = rounding_floor(p, u)
    rho = float(np.linalg.norm(orc.implicit_residual(p, u)))
    seq = orc.sequential(W.Problem(**{**p.__dict__, "cg_rtol": 1e-14}), u0)
    err = float(np.max(np.abs(u - seq)))
    print(f"cycles {st['iterations']}, stop {hist[-1]:.3e} (oracle {rho:.3e}, floor {floor:.1e}), "
          f"paper-form {st['final_residual']:.3e}, max error against the FP64 oracle {err:.2e}")
    assert status == atm.ATM_OK and hist[-1] <= 1e-10
    assert abs(hist[-1] - rho) <= 1e-12 * rho + floor
    assert st["final_residual"] <= hist[-1] * (1 + 1e-9) + floor
    assert err <= (p.nt + 1) * 1e-10
