"""Batched solves (one captured cycle replayed for many instances) through the C-ABI.

Every instance of a batch must end bit for bit where atm_solve takes it alone (same kernel bodies,
same arithmetic, same buffers) after the same number of cycles.  The stopping norm's pieces are
summed in another grouping than atm_solve's, so the residual histories agree to rounding only.
Graph replays must equal the directly enqueued launches bit for bit; the autotuner's choice is
cached and reused."""
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


def small_batch():
    items = []
    p, u0 = W.small_problem(W.HEAT1D, seed=1, nt=128, nx=63)
    items.append((p, W.Options(m=8, k=3, relax=1, tol=1e-10), u0))
    p, u0 = W.small_problem(W.HEAT1D, seed=2, nt=100, nx=200)          # ragged tail
    items.append((p, W.Options(m=16, k=2, relax=1, tol=1e-10), u0))
    p, u0 = W.small_problem(W.HEAT2D, seed=3, nt=64, nx=24, ny=24, cg_rtol=1e-12)
    items.append((p, W.Options(m=8, k=3, relax=1, tol=1e-9, precision=1), u0))
    p, u0 = W.small_problem(W.HEAT2D, seed=4, nt=48, nx=40, ny=33, cg_rtol=1e-12)
    items.append((p, W.Options(m=4, k=4, relax=1, tol=1e-9), u0))
    p, u0 = W.small_problem(W.AC2D, seed=5, nt=64, nx=32, ny=32, cg_rtol=1e-12)
    items.append((p, W.Options(m=8, k=3, relax=1, tol=1e-9, precision=1, coarse_substeps=2), u0))
    p, u0 = W.small_problem(W.AC2D, seed=6, nt=42, nx=16, ny=20, cg_rtol=1e-12)   # ragged tail, FP64
    items.append((p, W.Options(m=8, k=2, relax=0, tol=1e-9, coarse_substeps=2), u0))
    p, u0 = W.small_problem(W.HEAT2D, seed=7, nt=96, nx=128, ny=128, cg_rtol=1e-12)
    items.append((p, W.Options(m=16, k=3, relax=1, tol=1e-9, precision=1), u0))
    return items


def run_batch(atm, items, use_graph=True, tune_cache=None, check_every=3):
    us = [dev(W.initial_guess(p, u0)) for p, o, u0 in items]
    b = atm.Batch([p for p, _, _ in items], [o for _, o, _ in items], us, tune_cache=tune_cache)
    st, status, stats, hists, ms, mt = b.run(use_graph=use_graph, check_every=check_every)
    res = ([host(u) for u in us], status, stats, hists, ms, mt, b.tuning())
    b.close()
    return res


def test_batch_matches_individual_solves(atm):
    items = small_batch()
    us, status, stats, hists, ms, mt, tuning = run_batch(atm, items)
    assert tuning[0]
    for i, (p, o, u0) in enumerate(items):
        ud = dev(W.initial_guess(p, u0))
        st, hist, s = atm.atm_solve(p, o, ud)
        assert status[i] == st == atm.ATM_OK, i
        assert stats[i]["iterations"] == s["iterations"], i
        assert np.array_equal(us[i], host(ud)), f"instance {i}: max diff {np.max(np.abs(us[i] - host(ud)))}"
        assert len(hists[i]) == len(hist), i
        np.testing.assert_allclose(hists[i], hist, rtol=1e-12, atol=0, err_msg=f"instance {i}")
        # same iterate; the FP64 forms report the stopping norm, the FP32 form the paper's step residual
        np.testing.assert_allclose(stats[i]["final_residual"], s["final_residual"], rtol=1e-12, err_msg=f"{i}")


def test_batch_graph_replays_equal_direct_launches(atm):
    items = small_batch()
    a = run_batch(atm, items, use_graph=True, check_every=2)
    b = run_batch(atm, items, use_graph=False, check_every=5)
    for i in range(len(items)):
        assert np.array_equal(a[0][i], b[0][i]), i
        assert a[3][i] == b[3][i], i     # every cycle's residual norm


def test_batch_autotuner_cache(atm, tmp_path):
    items = small_batch()[:4]
    cache = str(tmp_path / "autotune.txt")
    first = run_batch(atm, items, tune_cache=cache)
    assert os.path.exists(cache) and len(open(cache).read().split()) == 4
    second = run_batch(atm, items, tune_cache=cache)
    assert second[5] == 0.0                      # no tuning work: the cached choice is used
    assert second[6][1:] == first[6][1:]
    for i in range(len(items)):
        assert np.array_equal(first[0][i], second[0][i])


def test_batch_workload_sample(atm):
    """The first 12 instances of the seeded 256-instance batch: all converge; three of them equal atm_solve."""
    items = W.batch_config(count=256)[:12]
    us, status, stats, hists, ms, mt, tuning = run_batch(atm, items, check_every=4)
    assert all(s == atm.ATM_OK for s in status), status
    for i in (0, 5, 11):
        p, o, u0 = items[i]
        ud = dev(W.initial_guess(p, u0))
        st, hist, s = atm.atm_solve(p, o, ud)
        assert st == atm.ATM_OK and s["iterations"] == stats[i]["iterations"]
        assert np.array_equal(us[i], host(ud)), i
    print(f"12 instances: {ms:.1f} ms, tuning {mt:.1f} ms, cycles {[s['iterations'] for s in stats]}")


def parity_batch():
    """small_batch() set up for parity with the oracle: the FP64 2D instances take CG to 1e-14 (iterate
    parity needs the same tight inner tolerance on both sides, whose summation orders differ), the FP32-fine
    instances stop at the reduced-precision bar 1e-10."""
    out = []
    for p, o, u0 in small_batch():
        if o.precision == 0 and p.kind != W.HEAT1D:
            p = W.Problem(**{**p.__dict__, "cg_rtol": 1e-14})
        if o.precision == 1:
            o = W.Options(**{**o.__dict__, "tol": 1e-10})
        out.append((p, o, u0))
    return out


def test_batch_instances_match_oracle(atm, orc):
    """Every instance of a batch against the CPU oracle (not against the GPU's own atm_solve): FP64 instances
    take the oracle's cycle count and match its iterate element by element to 1e-12 relative; FP32-fine
    instances meet 1e-10 in the oracle's FP64 implicit and paper-form residuals of the result, and their
    error against the oracle's sequential stepping is stated."""
    items = parity_batch()
    us, status, stats, hists, ms, mt, tuning = run_batch(atm, items)
    for i, (p, o, u0) in enumerate(items):
        assert status[i] == atm.ATM_OK, i
        g = W.initial_guess(p, u0)
        if o.precision == 0:
            ref, ref_hist, ref_stats = orc.solve(p, o, g)
            err = float(np.max(np.abs(us[i] - ref)) / np.max(np.abs(ref)))
            print(f"instance {i} ({W.KIND_NAMES[p.kind]} {p.nx}x{p.ny} nt {p.nt}, FP64): cycles "
                  f"{stats[i]['iterations']} (oracle {ref_stats['iterations']}), max rel. difference {err:.2e}")
            assert stats[i]["iterations"] == ref_stats["iterations"], i
            assert err <= 1e-12, (i, err)
        else:
            rho = float(np.linalg.norm(orc.implicit_residual(p, us[i])))
            r = float(np.linalg.norm(orc.step_residual(p, us[i])))
            q = W.Problem(**{**p.__dict__, "cg_rtol": 1e-14})
            err = float(np.max(np.abs(us[i] - orc.sequential(q, u0))))
            print(f"instance {i} ({W.KIND_NAMES[p.kind]} {p.nx}x{p.ny} nt {p.nt}, FP32 fine): cycles "
                  f"{stats[i]['iterations']}, oracle implicit residual {rho:.2e}, paper-form {r:.2e}, max error "
                  f"against the FP64 oracle's sequential stepping {err:.2e}")
            assert rho <= 1e-10 * (1 + 1e-6) and r <= rho * (1 + 1e-9), i
            assert err <= 1e-8, (i, err)
