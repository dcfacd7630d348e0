"""The window solve without a workspace argument (atm_coarse_solve_static, for callers that cannot allocate):
through the C-ABI its corrections equal those of atm_coarse_solve with a caller's workspace, bit for bit (the
same kernels on the same inputs), on calls in a row that share the one static scratch, the second with a
smaller input; sizes beyond the scratch and unsupported forms are rejected."""
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


def inputs(p, o, seed):
    """A relaxed-looking iterate and Phi values: random data (the window solve's result depends only on them)."""
    rng = np.random.default_rng(seed)
    NT = p.nt // o.m
    u = rng.uniform(-0.5, 0.5, size=(p.nt + 1, p.n))
    y = np.zeros((NT + 1, p.n))
    y[1:] = u[[j * o.m for j in range(1, NT + 1)]] + 1e-2 * rng.standard_normal((NT, p.n))
    return u, y


def both(atm, p, o, seed):
    u, y = inputs(p, o, seed)
    NT = p.nt // o.m
    ud, yd = dev(u), dev(y)
    e_ws = dev(np.full((NT + 1, p.n), np.nan))
    atm.atm_coarse_solve(p, o, ud, yd, e_ws, atm.workspace(atm.atm_workspace_bytes(p, o)))
    e_st = dev(np.full((NT + 1, p.n), np.nan))
    atm.atm_coarse_solve_static(p, o, ud, yd, e_st)
    return host(e_st), host(e_ws)


CASES = [
    # (first, larger call; second, smaller call) sharing the static scratch
    ("heat2d-128x128x4096-bf16-psi", lambda: W.config("c2")[::2], W.Options(m=32, k=13, coarse_solver=2),
     lambda: W.small_problem(W.HEAT2D, seed=2, nt=64, nx=24, ny=20), W.Options(m=4, k=3, coarse_solver=2)),
    ("ac2d-fas-fp64-psi", lambda: W.small_problem(W.AC2D, seed=3, nt=192, nx=64, ny=64),
     W.Options(m=8, k=4, coarse_substeps=2),
     lambda: W.small_problem(W.AC2D, seed=4, nt=40, nx=16, ny=32), W.Options(m=4, k=2, coarse_substeps=2)),
    ("heat1d-then-heat2d", lambda: W.small_problem(W.HEAT1D, seed=5, nt=512, nx=255), W.Options(m=16, k=4),
     lambda: W.small_problem(W.HEAT2D, seed=6, nt=48, nx=16, ny=16), W.Options(m=4, k=2)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_static_window_solve_equals_workspace_call(atm, case):
    _, big, ob, small, osm = case
    pb, _ = big()
    ps, _ = small()
    assert ps.n * (ps.nt // osm.m + 1) < pb.n * (pb.nt // ob.m + 1)
    for p, o, seed in ((pb, ob, 11), (ps, osm, 12)):
        got, ref = both(atm, p, o, seed)
        assert np.all(np.isfinite(ref))
        assert np.array_equal(got, ref), f"max diff {np.max(np.abs(got - ref))}"


def test_static_window_solve_limits(atm):
    assert atm.atm_static_scratch_bytes() == 32 << 20
    p, _ = W.small_problem(W.HEAT2D, seed=1, nt=4096, nx=128, ny=128)
    o = W.Options(m=8, k=5, coarse_solver=2)        # 513 C-points x 16384 x 8 B of residuals: beyond 32 MiB
    NT = p.nt // o.m
    u, y, e = dev(np.zeros((p.nt + 1, p.n))), dev(np.zeros((NT + 1, p.n))), dev(np.zeros((NT + 1, p.n)))
    with pytest.raises(atm.AtmError) as ei:
        atm.atm_coarse_solve_static(p, o, u, y, e)
    assert ei.value.status == atm.ATM_ERR_WORKSPACE
    p, _ = W.small_problem(W.HEAT2D, seed=1, nt=32, nx=16, ny=16)
    o = W.Options(m=4, k=2, coarse_solver=1)         # Psi by CG: not taken
    NT = p.nt // o.m
    u, y, e = dev(np.zeros((p.nt + 1, p.n))), dev(np.zeros((NT + 1, p.n))), dev(np.zeros((NT + 1, p.n)))
    with pytest.raises(atm.AtmError) as ei:
        atm.atm_coarse_solve_static(p, o, u, y, e)
    assert ei.value.status == atm.ATM_ERR_UNSUPPORTED
