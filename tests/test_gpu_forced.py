"""GPU parity of the forced 1D heat path (a PDE source in every fine step) and of
the k-study of section 4.3 at the paper's size, through the C-ABI, against the
CPU oracle.

FP64 bar: 1e-12 relative to the largest magnitude of the reference for
iterates.  Residual histories: the sides differ only in rounding (PCR on the
GPU, the Thomas algorithm in the oracle), which bounds each C-point residual
entry by about 1e-14 and a norm over the 1.3e5 C-point entries by about 4e-12,
so histories are compared to 1e-9 relative plus 1e-10 absolute.
"""
import os

import numpy as np
import pytest

import workloads as W
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


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


def assert_close(got, ref, rtol=1e-12, what=""):
    scale = max(float(np.max(np.abs(ref))), 1e-300)
    err = float(np.max(np.abs(got - ref)))
    assert err <= rtol * scale, f"{what}: max|diff| = {err:.3e} > {rtol:.1e} * {scale:.3e}"


def step_rtol(p):
    """Two backward-stable solves of the step's tridiagonal system (PCR, Thomas) differ by about
    kappa eps |x| with kappa = 1 + 4 dt/h^2 its condition number: 1e-12, or 10 kappa eps where the
    step is stiffer than the k-study's (kappa about 90 there)."""
    h = p.length / (p.nx + 1)
    kappa = 1.0 + 4.0 * p.nu * p.dt / h ** 2
    return max(1e-12, 10.0 * kappa * np.finfo(np.float64).eps)


@pytest.mark.parametrize("nx,nt", [(63, 200), (1023, 16383), (1023, 300), (5, 7)])
def test_forced_sequential(atm, orc, nx, nt):
    p, u0, src, _ = W.heat1d_forced(nx=nx, nt=nt)
    u = np.zeros((p.nt + 1, p.n))
    u[0] = u0
    ud = dev(u)
    atm.atm_sequential(p, ud, source=dev(src))
    assert_close(host(ud), orc.sequential(p, u0, source=src), rtol=step_rtol(p), what="forced sequential stepping")


@pytest.mark.parametrize("m", [4, 16])
def test_forced_sweeps(atm, orc, m):
    p, u0, src, ug = W.heat1d_forced(nx=100, nt=45 if m == 4 else 70)  # ragged tails
    o = W.Options(m=m, k=3, relax=1, coarse_form=1)
    NT = p.nt // m
    srcd = dev(src)
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))

    def y_ref(u):
        # y_j = Phi(u_{jm-1}) + g_{jm} = r_{jm} + u_{jm}
        r = orc.residual(p, u, u0, source=src)
        y = np.zeros((NT + 1, p.n))
        for j in range(1, NT + 1):
            y[j] = r[j * m] + u[j * m]
        return y

    ud, yd = dev(ug), dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 0, ud, None, yd, ws, source=srcd)
    u_f = orc.f_relax(p, o, ug, source=src)
    assert_close(host(ud), u_f, what="F-relaxation u")
    assert_close(host(yd)[1:], y_ref(u_f)[1:], what="F-relaxation y")
    y2 = dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 2, ud, yd, y2, ws, source=srcd)
    u_cf = orc.f_relax(p, o, orc.c_relax(p, o, u_f, source=src), source=src)
    assert_close(host(ud), u_cf, what="CF-relaxation u")
    assert_close(host(y2)[1:], y_ref(u_cf)[1:], what="CF-relaxation y")
    e = np.random.default_rng(11).standard_normal((NT + 1, p.n)) * 0.1
    e[0] = 0.0
    y3 = dev(np.zeros((NT + 1, p.n)))
    atm.atm_sweep(p, o, 1, ud, dev(e), y3, ws, source=srcd)
    u_c = orc.correct(p, o, u_cf, e, source=src)
    assert_close(host(ud), u_c, what="correction u")
    assert_close(host(y3)[1:], y_ref(u_c)[1:], what="correction y")


def test_forced_residual_norms(atm, orc):
    p, u0, src, ug = W.heat1d_forced(nx=200, nt=90)
    o = W.Options(m=8, k=2, coarse_form=1)
    ws = atm.workspace(atm.atm_workspace_bytes(p, o))
    ud, srcd = dev(ug), dev(src)
    rho = orc.implicit_residual(p, ug, source=src)
    r = orc.step_residual(p, ug, source=src)
    got_rho = atm.atm_implicit_residual_norm(p, o, ud, ws, source=srcd)
    got_r = atm.atm_step_residual_norm(p, o, ud, ws, source=srcd)
    np.testing.assert_allclose(got_rho, np.sqrt(np.sum(rho ** 2)), rtol=1e-12)
    np.testing.assert_allclose(got_r, np.sqrt(np.sum(r ** 2)), rtol=1e-12)


@pytest.mark.parametrize("relax", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3, 100])
def test_forced_solve_small(atm, orc, relax, k):
    p, u0, src, ug = W.heat1d_forced(nx=31, nt=250)
    o = W.Options(m=8, k=k, relax=relax, tol=1e-11, max_iter=300, coarse_form=1)
    ref, hist, st = orc.solve(p, o, ug, source=src)
    ud = dev(ug)
    status, ghist, gst = atm.atm_solve(p, o, ud, source=dev(src), hist_cap=400)
    assert status == atm.ATM_OK
    assert gst["iterations"] == st["iterations"]
    assert_close(host(ud), ref, what="converged forced iterate")
    np.testing.assert_allclose(ghist, hist, rtol=1e-9, atol=1e-12)


@pytest.fixture(scope="module")
def full(orc):
    orc.set_threads(min(16, os.cpu_count() or 1))
    p, u0, src, ug = W.heat1d_forced()
    yield p, u0, src, ug, W.heat1d_forced_exact(p)
    orc.set_threads(1)


@pytest.mark.parametrize("m,k", [(128, 12), (128, 128), (64, 20), (32, 40), (128, 2)])
def test_k_study_full_size(atm, orc, full, m, k):
    """1025 grid points x 16384 time points, random guess, F-relaxation, tol 1e-7: the GPU takes the
    oracle's number of iterations and returns its iterate."""
    p, u0, src, ug, exact = full
    o = W.k_study_options(m, k)
    ref, hist, st = orc.solve(p, o, ug, source=src)
    ud = dev(ug)
    status, ghist, gst = atm.atm_solve(p, o, ud, source=dev(src), hist_cap=256)
    assert status == atm.ATM_OK
    assert gst["iterations"] == st["iterations"]
    got = host(ud)
    assert_close(got, ref, what=f"k-study m={m} k={k} iterate")
    np.testing.assert_allclose(ghist, hist, rtol=1e-9, atol=1e-10)
    err_ref = np.abs(ref - exact).max()
    assert abs(np.abs(got - exact).max() - err_ref) <= 1e-6 * err_ref


def test_source_rejected_elsewhere(atm):
    """A source is taken by the 1D heat kind only."""
    import torch
    p, _ = W.small_problem(W.HEAT2D, nx=8, nt=8)
    o = W.Options(m=2, k=2)
    u = torch.zeros((p.nt + 1, p.n), dtype=torch.float64, device="cuda")
    with pytest.raises(atm.AtmError) as ei:
        atm.atm_solve(p, o, u, ws=atm.workspace(atm.atm_workspace_bytes(p, o)), source=torch.zeros_like(u))
    assert ei.value.status == atm.ATM_ERR_UNSUPPORTED
