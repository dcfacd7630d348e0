"""GPU parity of the windows on two CUs each: the local solves of the truncated coarse problem
(section 2.1, linear and FAS forms) with Psi's implicit solve in the eigenbasis, on large grids of 128,
192 or 256 columns and a multiple of 128 rows, through the C-ABI against the CPU oracle."""
import numpy as np
import pytest

import workloads as W
from tests.conftest import gpu_available
from tests.test_gpu_parity import assert_close, dev, host, small, y_of

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

PAIRED = [
    # (kind, nx, ny, nt, m, k)
    (W.HEAT2D, 256, 256, 12, 4, 3),    # four 64-column tiles per wave, two row blocks per half
    (W.AC2D, 192, 128, 12, 3, 4),      # three tiles, one row block per half
    (W.HEAT2D, 128, 256, 10, 2, 3),    # two tiles
    (W.AC2D, 192, 128, 262, 2, 3),     # 132 windows: with at most 128 pairs resident a pair takes two
]


def ids(c):
    return f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}-k{c[5]}"


@pytest.fixture(scope="module")
def atm():
    import paper_2107_09596_amd as atm
    return atm


def options(kind, m, k, form, solver=0):
    return W.Options(m=m, k=k, coarse_form=form, coarse_substeps=2 if kind == W.AC2D else 1, coarse_solver=solver)


def test_paired_kernel_is_taken(atm):
    for kind, nx, ny, nt, m, k in PAIRED:
        p, _ = small(kind, nx, ny, nt)
        assert atm.atm_coarse_kernel(p, options(kind, m, k, 0)) == "coarse_pair_kernel"
        assert atm.atm_coarse_kernel(p, options(kind, m, k, 0, solver=1)) == "coarse_large_kernel"
    # rows not a multiple of 128, columns beyond 256: one workgroup per window
    for nx, ny in ((256, 192), (320, 256)):
        p, _ = small(W.HEAT2D, nx, ny, 8)
        assert atm.atm_coarse_kernel(p, options(W.HEAT2D, 4, 2, 0)) == "coarse_large_kernel"


@pytest.mark.parametrize("form", [1, 2])
@pytest.mark.parametrize("case", PAIRED, ids=ids)
def test_paired_windows_match_oracle(atm, orc, case, form):
    kind, nx, ny, nt, m, k = case
    p, u0 = small(kind, nx, ny, nt)
    o = options(kind, m, k, form)
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
    assert_close(host(e), ref, what=f"paired windows, coarse form {form}")
    # a second call on the same workspace (meeting counters cleared again) gives the same bits
    e2 = dev(np.zeros((NT + 1, p.n)))
    atm.atm_coarse_solve(p, o, dev(u), dev(y), e2, ws)
    assert np.array_equal(host(e2), host(e))


@pytest.mark.parametrize("precision", [0, 1])
def test_paired_windows_solve(atm, orc, precision):
    kind, nx, ny, nt, m, k = W.HEAT2D, 192, 128, 24, 2, 3
    p, u0 = small(kind, nx, ny, nt)
    seq = orc.sequential(p, u0)
    o = W.Options(m=m, k=k, relax=1, tol=1e-11, precision=precision)
    assert atm.atm_coarse_kernel(p, o) == "coarse_pair_kernel"
    ud = dev(W.initial_guess(p, u0))
    status, hist, st = atm.atm_solve(p, o, ud)
    assert status == atm.ATM_OK and st["final_residual"] <= 1e-11
    assert np.linalg.norm(host(ud) - seq) <= (p.nt + 1) * 1e-11 + 1e-12 * np.linalg.norm(seq)


# ---------------------------------------------------------------------------
# Psi's eigenbasis solve on the BF16 matrix cores (coarse_solver 2): windows in terms of e
# ---------------------------------------------------------------------------

BF_PAIRED = [
    # (kind, nx, ny, nt, m, k, coarse substeps)
    (W.HEAT2D, 256, 256, 12, 4, 2, 1),   # one window step: the tight bound
    (W.AC2D, 256, 256, 16, 4, 2, 4),     # the 256 x 256 periodic grid with four substeps, one step
    (W.HEAT2D, 256, 256, 12, 4, 3, 1),
    (W.AC2D, 192, 128, 12, 3, 4, 2),     # FAS: v through the first of two substeps from the trajectory
    (W.HEAT2D, 128, 256, 10, 2, 3, 1),
    (W.AC2D, 192, 128, 262, 2, 3, 1),    # 132 windows: with at most 128 pairs resident a pair takes two
]


def bf_ids(c):
    return f"k{c[0]}-{c[1]}x{c[2]}-nt{c[3]}-m{c[4]}-k{c[5]}-s{c[6]}"


def bf_options(kind, m, k, form, sub):
    return W.Options(m=m, k=k, coarse_form=form, coarse_substeps=sub, coarse_solver=2)


def test_bf16_paired_kernel_is_taken(atm):
    for kind, nx, ny, nt, m, k, sub in BF_PAIRED:
        p, _ = small(kind, nx, ny, nt)
        assert atm.atm_coarse_kernel(p, bf_options(kind, m, k, 0, sub)) == "coarse_pair_bf_kernel"


@pytest.mark.parametrize("form", [1, 2])
@pytest.mark.parametrize("case", BF_PAIRED, ids=bf_ids)
def test_bf16_paired_windows_match_oracle(atm, orc, case, form):
    """Each product takes BF16 hi + lo parts of its operands (about 2^-17 relative each) with FP32 sums over
    at most 256 terms, so one substep of M^-1 is within about 4e-5 of the FP64 solve relative to the
    correction it acts on; a window of k - 1 steps of s substeps accumulates at most (k - 1) s of them.
    The bound asserted is 5e-5 per substep of the deepest window, relative to max |e|."""
    kind, nx, ny, nt, m, k, sub = case
    p, u0 = small(kind, nx, ny, nt)
    o = bf_options(kind, m, k, form, sub)
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
    got = host(e)
    scale = float(np.max(np.abs(ref)))
    err = float(np.max(np.abs(got - ref)))
    bound = 5e-5 * (k - 1) * sub * scale
    print(f"BF16 paired windows {bf_ids(case)} form {form}: max error {err:.2e} of max |e| {scale:.2e} "
          f"({err / scale:.1e} relative, bound {bound / scale:.1e})", flush=True)
    assert err <= bound
    # the error is that of the products, not of a wrong window: the exact windows' first entries (p < 1)
    # are the residuals themselves
    np.testing.assert_array_equal(got[0], ref[0])
    e2 = dev(np.zeros((NT + 1, p.n)))
    atm.atm_coarse_solve(p, o, dev(u), dev(y), e2, ws)
    assert np.array_equal(host(e2), got)


@pytest.mark.parametrize("kind,sub,precision", [(W.HEAT2D, 1, 0), (W.HEAT2D, 1, 1), (W.AC2D, 2, 1)])
def test_bf16_paired_windows_solve(atm, orc, kind, sub, precision):
    """The BF16 Psi changes the convergence rate only: the solve reaches the FP64 fixed point."""
    nx, ny, nt, m, k = 192, 128, 24, 2, 3
    p, u0 = small(kind, nx, ny, nt)
    seq = orc.sequential(p, u0)
    o = W.Options(m=m, k=k, relax=1, tol=1e-11 if precision == 0 else 1e-10, precision=precision,
                  coarse_substeps=sub, coarse_solver=2, max_iter=60)
    assert atm.atm_coarse_kernel(p, o) == "coarse_pair_bf_kernel"
    ud = dev(W.initial_guess(p, u0))
    status, hist, st = atm.atm_solve(p, o, ud)
    err = float(np.linalg.norm(host(ud) - seq))
    print(f"BF16 paired solve kind {kind} s {sub} precision {precision}: {st['iterations']} cycles, "
          f"final residual {st['final_residual']:.2e}, |u - sequential| {err:.2e}", flush=True)
    assert status == atm.ATM_OK and st["final_residual"] <= o.tol
    assert err <= (p.nt + 1) * 10 * o.tol + 1e-12 * np.linalg.norm(seq)
