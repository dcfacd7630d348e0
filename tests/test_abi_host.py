"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
symbol that include/atm.h declares, and its host logic (window starts, interval
counts, workspace sizing, argument validation) behaves as documented."""
import ctypes
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def abi():
    from paper_2107_09596_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2107_09596_amd import build
        build.build()
    return _abi


def header_functions():
    src = open(os.path.join(ROOT, "include", "atm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(atm_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(abi):
    names = header_functions()
    assert len(names) >= 10
    lib = abi.lib()
    for name in names:
        assert hasattr(lib, name), name
        assert name in abi.SIGNATURES, name


def test_window_start_matches_definition(abi, orc):
    for k in (1, 2, 3, 7, 100):
        for p in range(0, 40):
            assert abi.lib().atm_window_start(p, k) == max(0, p - k + 1) == orc.window_start(p, k)


def test_num_intervals_and_workspace(abi):
    p, o, _ = W.config("c2")
    P, O = abi.problem(p), abi.options(o)
    assert abi.lib().atm_num_intervals(ctypes.byref(P), ctypes.byref(O)) == 128
    ws = abi.lib().atm_workspace_bytes(ctypes.byref(P), ctypes.byref(O))
    slab = 129 * 128 * 128 * 8
    tables = (2 * 128 * 128 * 2 + 2 * 128) * 8  # eigenbasis tables of Psi's solve: Qx, Qx^T, Qy, Qy^T, ex, ey
    assert 3 * slab + tables <= ws <= 3 * slab + tables + 64 * 1024
    o.coarse_solver = 1  # Psi by CG: no tables
    ws_cg = abi.lib().atm_workspace_bytes(ctypes.byref(abi.problem(p)), ctypes.byref(abi.options(o)))
    assert 3 * slab <= ws_cg <= 3 * slab + 64 * 1024 and ws - ws_cg >= tables
    o.coarse_solver = 0
    o.coarse_form = 2
    ws_fas = abi.lib().atm_workspace_bytes(ctypes.byref(abi.problem(p)), ctypes.byref(abi.options(o)))
    assert ws_fas >= ws + slab


@pytest.mark.parametrize("field,value,status", [
    ("m", 1, -1), ("k", 0, -1), ("relax", 2, -1), ("coarse_substeps", 0, -1), ("max_iter", -1, -1),
    ("precision", 3, -1), ("mixed_cg_rtol", -1.0, -1), ("mixed_cg_rtol", 1.0, -1), ("coarse_solver", 3, -1),
    ("precision", 1, -2),  # the FP32 fine form is built for the 2D kinds only
])
def test_invalid_options_rejected_before_launch(abi, field, value, status):
    p, o, _ = W.config("c1")
    setattr(o, field, value)
    P, O = abi.problem(p), abi.options(o)
    assert abi.lib().atm_workspace_bytes(ctypes.byref(P), ctypes.byref(O)) == 0
    st = abi.lib().atm_solve(ctypes.byref(P), ctypes.byref(O), None, None, 0, None, 0, None, None)
    assert st == status
    assert abi.lib().atm_last_error().decode() != ""


@pytest.mark.parametrize("field,value,status", [
    ("nx", 0, -1), ("nt", 0, -1), ("kind", 9, -1), ("nu", 0.0, -1), ("tf", -1.0, -1), ("cg_max_iter", 0, -1),
])
def test_invalid_problem_rejected(abi, field, value, status):
    p, o, _ = W.config("c2")
    setattr(p, field, value)
    st = abi.lib().atm_solve(ctypes.byref(abi.problem(p)), ctypes.byref(abi.options(o)), None, None, 0, None, 0,
                             None, None)
    assert st == status


def test_large_grids_take_the_scratch_layout(abi):
    """Grids beyond 128 points per side are accepted (global-scratch kernels) with five FP64 n-vectors per
    interval or window in the workspace."""
    o = W.Options(m=4, k=2)
    small = W.Problem(W.HEAT2D, nx=128, ny=128, nt=64)
    big = W.Problem(W.HEAT2D, nx=256, ny=256, nt=64)
    ws_small = abi.lib().atm_workspace_bytes(ctypes.byref(abi.problem(small)), ctypes.byref(abi.options(o)))
    ws_big = abi.lib().atm_workspace_bytes(ctypes.byref(abi.problem(big)), ctypes.byref(abi.options(o)))
    assert ws_small > 0 and ws_big >= 4 * (ws_small - 64 * 1024) + 17 * 5 * 256 * 256 * 8


def test_unsupported_sizes(abi):
    p = W.Problem(W.HEAT2D, nx=2000, ny=16, nt=64)
    o = W.Options(m=4, k=2)
    P, O = abi.problem(p), abi.options(o)
    st = abi.lib().atm_solve(ctypes.byref(P), ctypes.byref(O), None, None, 0, None, 0, None, None)
    assert st == abi.ATM_ERR_UNSUPPORTED
    p = W.Problem(W.HEAT1D, nx=2000, ny=1, nt=64)
    st = abi.lib().atm_solve(ctypes.byref(abi.problem(p)), ctypes.byref(O), None, None, 0, None, 0, None, None)
    assert st == abi.ATM_ERR_UNSUPPORTED


def test_workspace_too_small_rejected(abi):
    p, o, _ = W.config("c1")
    P, O = abi.problem(p), abi.options(o)
    need = abi.lib().atm_workspace_bytes(ctypes.byref(P), ctypes.byref(O))
    st = abi.lib().atm_solve(ctypes.byref(P), ctypes.byref(O), ctypes.c_void_p(256), ctypes.c_void_p(256 * 4),
                             need - 8, None, 0, None, None)
    assert st == abi.ATM_ERR_WORKSPACE


def test_status_strings(abi):
    for code, name in [(0, "ATM_OK"), (1, "ATM_NOT_CONVERGED"), (-1, "ATM_ERR_INVALID_ARG"), (-5, "ATM_ERR_INNER_SOLVE")]:
        assert abi.lib().atm_status_string(code).decode() == name


def test_strip_layout_rule_accepts_all_grids_up_to_128(abi):
    """Every 2D grid up to 128 x 128 passes the host's LDS-bounds rule (it is validated, not launched)."""
    for nx in (1, 3, 17, 63, 64, 65, 100, 127, 128):
        for ny in (1, 2, 31, 64, 97, 128):
            for precision in (0, 1):
                p = W.Problem(W.HEAT2D, nx=nx, ny=ny, nt=8)
                o = W.Options(m=2, k=2, precision=precision)
                assert abi.lib().atm_workspace_bytes(ctypes.byref(abi.problem(p)), ctypes.byref(abi.options(o))) > 0


def test_source_accepted_for_1d_only(abi):
    """The PDE source is validated on the host: the 1D heat kind takes it (same workspace), the 2D
    kinds and the batch API reject it before anything is launched (the pointer is never read)."""
    p1, o1 = W.Problem(W.HEAT1D, nx=63, nt=64), W.Options(m=4, k=2)
    P, O = abi.problem(p1), abi.options(o1)
    plain = abi.lib().atm_workspace_bytes(ctypes.byref(P), ctypes.byref(O))
    P.source = 256
    assert abi.lib().atm_workspace_bytes(ctypes.byref(P), ctypes.byref(O)) == plain > 0
    assert abi.lib().atm_batch_workspace_bytes(1, ctypes.byref(P), ctypes.byref(O)) == 0
    assert "source" in abi.lib().atm_last_error().decode()
    P2 = abi.problem(W.Problem(W.HEAT2D, nx=16, ny=16, nt=64))
    P2.source = 256
    assert abi.lib().atm_workspace_bytes(ctypes.byref(P2), ctypes.byref(O)) == 0
    st = abi.lib().atm_solve(ctypes.byref(P2), ctypes.byref(O), None, None, 0, None, 0, None, None)
    assert st == abi.ATM_ERR_UNSUPPORTED


def test_bf16_psi_restrictions(abi):
    """coarse_solver 2 is built for the 2D kinds: grids up to 128 per side (FAS with one substep), and the
    paired large-grid windows (rows of 128, 192 or 256 points, 128 or 256 rows; FAS with any substeps)."""
    ok = W.Problem(W.HEAT2D, nx=64, ny=96, nt=64)
    for p, o, expect in [
            (ok, W.Options(m=4, k=2, coarse_solver=2), True),
            (W.Problem(W.HEAT2D, nx=48, ny=37, nt=64), W.Options(m=4, k=2, coarse_solver=2), True),
            (W.Problem(W.HEAT2D, nx=200, ny=64, nt=64), W.Options(m=4, k=2, coarse_solver=2), False),
            (ok, W.Options(m=4, k=2, coarse_solver=2, coarse_form=2), True),
            (ok, W.Options(m=4, k=2, coarse_solver=2, coarse_form=2, coarse_substeps=2), False),
            (W.Problem(W.HEAT1D, nx=64, nt=64), W.Options(m=4, k=2, coarse_solver=2), False),
            (W.Problem(W.AC2D, nx=64, ny=64, nt=64), W.Options(m=4, k=2, coarse_solver=2), True),
            (W.Problem(W.AC2D, nx=256, ny=256, nt=64), W.Options(m=4, k=2, coarse_solver=2, coarse_substeps=4), True),
            (W.Problem(W.HEAT2D, nx=192, ny=128, nt=64), W.Options(m=4, k=2, coarse_solver=2), True),
            (W.Problem(W.HEAT2D, nx=128, ny=256, nt=64), W.Options(m=4, k=2, coarse_solver=2), True),
            (W.Problem(W.HEAT2D, nx=256, ny=192, nt=64), W.Options(m=4, k=2, coarse_solver=2), False),
            (W.Problem(W.HEAT2D, nx=320, ny=256, nt=64), W.Options(m=4, k=2, coarse_solver=2), False),
            (W.Problem(W.HEAT2D, nx=160, ny=256, nt=64), W.Options(m=4, k=2, coarse_solver=2), False),
            (ok, W.Options(m=4, k=2, coarse_solver=3), False)]:
        n = abi.lib().atm_workspace_bytes(ctypes.byref(abi.problem(p)), ctypes.byref(abi.options(o)))
        assert (n > 0) == expect, (p, o)


def test_three_levels_bf16_coarsest_needs_one_substep(abi):
    p = W.Problem(W.HEAT2D, nx=32, ny=32, nt=64)
    ok = W.Options(m=4, k=2, levels=3, m_coarse=2, coarse_solver=2)
    bad = W.Options(m=4, k=2, levels=3, m_coarse=2, coarse_solver=2, coarse_substeps=2)
    n_ok = abi.lib().atm_workspace_bytes(ctypes.byref(abi.problem(p)), ctypes.byref(abi.options(ok)))
    n_cg = abi.lib().atm_workspace_bytes(ctypes.byref(abi.problem(p)),
                                         ctypes.byref(abi.options(W.Options(**{**ok.__dict__, "coarse_solver": 1}))))
    assert n_ok > n_cg > 0  # the tables and the coarsest level's residual rows
    assert abi.lib().atm_workspace_bytes(ctypes.byref(abi.problem(p)), ctypes.byref(abi.options(bad))) == 0
