"""GPU parity of the large-grid kernels (more than 128 points per side: Krylov vectors in a global
scratch) through the C-ABI, against the CPU oracle, and the 2D Allen-Cahn 256x256 workload at full size."""
import numpy as np
import pytest

import workloads as W
from tests.conftest import gpu_available
from tests.test_gpu_mixed import rounding_floor
from tests.test_gpu_parity import assert_close, dev, host, small, y_of

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

LARGE = [
    # (kind, nx, ny, nt, m, k)
    (W.HEAT2D, 160, 136, 16, 4, 2),
    (W.HEAT2D, 130, 257, 9, 4, 3),      # odd rows per pass, ragged tail
    (W.AC2D, 144, 132, 12, 4, 2),
    (W.AC2D, 256, 256, 8, 4, 2),
]


def ids(c):
    return f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}-k{c[5]}"


@pytest.fixture(scope="module")
def atm():
    import paper_2107_09596_amd as atm
    return atm


@pytest.mark.parametrize("case", LARGE, ids=ids)
def test_large_sweeps_match_oracle(atm, orc, case):
    kind, nx, ny, nt, m, k = case
    p, u0 = small(kind, nx, ny, nt)
    o = W.Options(m=m, k=k, relax=1)
    NT = p.nt // m
    u = W.initial_guess(p, u0, "random", seed=3) * (0.3 if kind == W.AC2D else 1.0)
    u[0] = u0
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    ud, yd = dev(u), dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 0, ud, None, yd, ws)
    u_f = orc.f_relax(p, o, u)
    assert_close(host(ud), u_f, what="F-relaxation u")
    assert_close(host(yd)[1:], y_of(orc, p, o, u_f)[1:], what="F-relaxation y")
    y2 = dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 2, ud, yd, y2, ws)
    u_cf = orc.f_relax(p, o, orc.c_relax(p, o, u_f))
    assert_close(host(ud), u_cf, what="CF-relaxation u")
    e = np.random.default_rng(11).standard_normal((NT + 1, p.n)) * 0.1
    e[0] = 0.0
    y3 = dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 1, ud, dev(e), y3, ws)
    u_c = orc.correct(p, o, u_cf, e)
    assert_close(host(ud), u_c, what="correction u")
    assert_close(host(y3)[1:], y_of(orc, p, o, u_c)[1:], what="correction y")


@pytest.mark.parametrize("solver", [0, 1], ids=["eigenbasis", "cg"])
@pytest.mark.parametrize("form", [1, 2])
@pytest.mark.parametrize("case", LARGE, ids=ids)
def test_large_coarse_solves_match_oracle(atm, orc, case, form, solver):
    """Psi's implicit solve by the eigenbasis of the constant-coefficient operator (exact to rounding) or by
    CG (to rtol 1e-14, as the oracle's): both give the oracle's local solves."""
    kind, nx, ny, nt, m, k = case
    p, u0 = small(kind, nx, ny, nt)
    o = W.Options(m=m, k=k, coarse_form=form, coarse_substeps=2 if kind == W.AC2D else 1, coarse_solver=solver)
    NT = p.nt // m
    g = W.initial_guess(p, u0, "random", seed=4) * 0.5
    g[0] = u0
    u = orc.f_relax(p, o, g)
    y = y_of(orc, p, o, u)
    rc = np.zeros((NT + 1, p.n))
    vc = np.stack([u[j * m] for j in range(NT + 1)])
    for j in range(1, NT + 1):
        rc[j] = y[j] - u[j * m]
    ref = orc.local_solves(p, o, rc, vc)
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    e = dev(np.zeros((NT + 1, p.n)))
    atm.atm_coarse_solve(p, o, dev(u), dev(y), e, ws)
    assert_close(host(e), ref, what=f"coarse form {form}")


@pytest.mark.parametrize("case", LARGE[::2], ids=ids)
def test_large_sequential_and_solve(atm, orc, case):
    kind, nx, ny, nt, m, k = case
    p, u0 = small(kind, nx, ny, nt)
    seq = orc.sequential(p, u0)
    us = np.zeros((p.nt + 1, p.n))
    us[0] = u0
    usd = dev(us)
    atm.atm_sequential(p, usd)
    assert_close(host(usd), seq, what="sequential")
    for precision in (0, 1):
        o = W.Options(m=m, k=k, relax=1, tol=1e-11, precision=precision, coarse_substeps=2 if kind == W.AC2D else 1)
        ud = dev(W.initial_guess(p, u0))
        status, hist, st = atm.atm_solve(p, o, ud)
        assert status == atm.ATM_OK and st["final_residual"] <= 1e-11
        assert np.linalg.norm(host(ud) - seq) <= (p.nt + 1) * 1e-11 + 1e-12 * np.linalg.norm(seq)


@pytest.mark.parametrize("solver,mixed_rtol", [(0, 0.0), (2, 0.0), (2, 3e-4)],
                         ids=["fp64-psi", "bf16-psi", "bf16-psi-fp32-cg-3e-4"])
def test_ac256_full_size(atm, orc, solver, mixed_rtol):
    """2D Allen-Cahn 256x256 periodic, eps 0.02, dt 1e-5, Nt 8192, m 64, k 13, FCF, 4 coarse substeps, FP32 fine
    solves, Psi in the eigenbasis on the FP64 or the BF16 matrix cores, to the reduced-precision bar 1e-10: the
    stopping norm equals the oracle's FP64 implicit residual of the result at every one of the 5.4e8
    space-time points, the paper-form residual is at most the stopping norm, and the first 64 steps match the
    oracle's sequential stepping (its error is printed)."""
    p, o, u0 = W.config("c3")
    o.tol = 1e-10
    o.coarse_solver = solver
    o.mixed_cg_rtol = mixed_rtol  # 0: the library's 1e-6; 3e-4: the benchmark's setting
    print(f"c3 full size, coarse_solver {solver}, mixed_cg_rtol {mixed_rtol}", flush=True)
    ud = dev(W.initial_guess(p, u0))
    status, hist, st = atm.atm_solve(p, o, ud)
    u = host(ud)
    floor = rounding_floor(p, u)
    rho = float(np.linalg.norm(orc.implicit_residual(p, u)))
    q = W.Problem(**{**p.__dict__, "nt": 64, "tf": p.t0 + 64 * p.dt, "cg_rtol": 1e-14})
    ref = orc.sequential(q, u0)
    err = float(np.max(np.abs(u[:65] - ref)))
    print(f"cycles {st['iterations']}, stopping norm {hist[-1]:.3e} (oracle {rho:.3e}, rounding floor {floor:.1e}), "
          f"paper-form {st['final_residual']:.3e}, error against the FP64 oracle on the first 64 steps {err:.2e}, "
          f"{st['ms_total']:.0f} ms")
    assert status == atm.ATM_OK and hist[-1] <= 1e-10
    assert abs(hist[-1] - rho) <= 1e-9 * rho + floor
    assert st["final_residual"] <= hist[-1] * (1 + 1e-9) + floor
    assert err <= 1e-9, f"max error against the FP64 oracle on the first 64 steps: {err:.2e}"


@pytest.mark.parametrize("solver", [0, 1], ids=["eigenbasis", "cg"])
def test_max_row_length(atm, orc, solver):
    """The longest supported row (1024 points) with a short side of 40 and a ragged tail: F-relaxation and
    the windows (both Psi solvers) against the oracle."""
    # nu dt / h^2 of order 1 on h = 1/1025 (the default nu would need thousands of CG iterations per step)
    p, u0 = W.small_problem(W.HEAT2D, seed=5, nt=7, nx=1024, ny=40, nu=1e-5, tf=0.7, cg_rtol=1e-14)
    o = W.Options(m=2, k=2, relax=1, coarse_solver=solver)
    NT = p.nt // o.m
    u = W.initial_guess(p, u0, "random", seed=3)
    u[0] = u0
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    ud, yd = dev(u), dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 0, ud, None, yd, ws)
    u_f = orc.f_relax(p, o, u)
    assert_close(host(ud), u_f, what="F-relaxation u")
    y = y_of(orc, p, o, u_f)
    assert_close(host(yd)[1:], y[1:], what="F-relaxation y")
    vc = np.stack([u_f[j * o.m] for j in range(NT + 1)])
    rc = y - vc
    rc[0] = 0.0
    e = dev(np.zeros((NT + 1, p.n)))
    atm.atm_coarse_solve(p, o, dev(u_f), dev(y), e, ws)
    assert_close(host(e), orc.local_solves(p, o, rc, vc), what="windows")


def test_max_1d_grid(atm, orc):
    """1D heat at the largest supported nx (1024 points, one workgroup of 1024 threads): sweep and solve."""
    p, u0 = small(W.HEAT1D, 1024, 1, 40)
    o = W.Options(m=4, k=3, relax=1, tol=1e-12)
    NT = p.nt // o.m
    u = W.initial_guess(p, u0, "random", seed=5)
    u[0] = u0
    ud, yd = dev(u), dev(np.zeros((NT + 1, p.n)))
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    atm.atm_sweep(p, o, 0, ud, None, yd, ws)
    assert_close(host(ud), orc.f_relax(p, o, u), what="1D F-relaxation")
    ud = dev(W.initial_guess(p, u0))
    status, hist, st = atm.atm_solve(p, o, ud)
    assert status == atm.ATM_OK and hist[-1] <= o.tol
    assert_close(host(ud), orc.sequential(p, u0), rtol=1e-10, what="1D solve vs sequential stepping")


@pytest.mark.parametrize("case", [(W.HEAT2D, 256, 256, 12, 4, 2), (W.AC2D, 192, 128, 262, 2, 3),
                                  (W.HEAT2D, 128, 256, 10, 2, 3)], ids=ids)
def test_large_step_residual_norm_in_eigenbasis(atm, orc, case):
    """|M^-1 rho| summed over all fine steps by the whole-chip eigenbasis kernel (the steps split into
    contiguous runs, one workgroup each) equals the oracle's, on a rough iterate and on a converged one."""
    from tests.test_gpu_mixed import rounding_floor
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
    assert abs(got - ref) <= 1e-11 * ref + rounding_floor(p, seq)
