"""Benchmark: space-time point-updates per second to a 1e-8 residual, one GPU.

A step is one complete two-level AT-MGRIT solve (every hot-path row: FCF
relaxation sweeps, the truncated local coarse solves, correction and
interpolation, residual norm and stopping test) of the 2D heat workload
(128x128 interior, nu = 0.1, Nt = 4096, m = 32, k = 13, fine CG rtol 1e-12,
FP64) from the zero initial guess, with all inputs resident in HBM.  The
initial guess is restored by a device copy at the start of each step (inside
the timed region).  The coarse propagator Psi solves its implicit step in the
eigenbasis of the constant-coefficient operator on the BF16 matrix cores with
split operands, about 1e-5 relative (--coarse-solver 2; Psi only approximates
Phi^m, the fixed point does not depend on it, and the cycle count equals the
strict solve's); --coarse-solver 1 takes CG to --coarse-rtol instead, and one
extra solve with Psi's CG at the fine tolerance is reported as
"strict_coarse".  The fine CG of every F-point starts from the previous point's
value; "extrapolated_cg_start" reports the same solve with the library option
cg_guess 1 (the stored iterate moved by the change at the previous point: fewer
CG iterations, but each step first waits for two loads).  The other legs (Allen-Cahn, the batch) take Psi's FP64
eigenbasis solve, the library default.

Prints one JSON line (see the keys below).  --gpus > 1 is refused: this build
runs on a single GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks used for the roofline fraction
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# Algorithmic FP64 flops per grid point of the sweep kernel's CG:
#   per iteration: M p (7), (p, Mp) (2), x += a p (2), r -= a Mp (2), z = r/d (1),
#   (r, z) (2), (r, r) (2), p = z + b p (2)                                    = 20
#   per solve (initial residual r = b - M x, (b,b), (r,r), (r,z), p = z)       = 14
FLOPS_PER_CG_ITER_POINT = 20
FLOPS_PER_SOLVE_POINT = 14
# LDS bytes per grid point per CG iteration of the sweep kernel: the stencil reads the direction at the
# point and at its west and east neighbours (8 B each; north and south come from the same strip), the
# direction update reads it once more and writes it once
LDS_BYTES_PER_CG_ITER_POINT = 40
# LDS bandwidth, assuming 128 B per clock per CU: 256 CUs x 2.4 GHz x 128 B
PEAK_LDS_TBS = 78.6
# HBM bytes per launch of the FP64 sweep kernel on this workload (read, written), from rocprofv3
# FETCH_SIZE and WRITE_SIZE counters scaled by the same counters of a plain 1 GiB copy (x2.0, x1.0)
SWEEP_TRAFFIC_BYTES = (40.8e6, 321.8e6)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--coarse-rtol", type=float, default=1e-3,
                    help="CG tolerance inside the coarse propagator (0 = the fine cg_rtol)")
    ap.add_argument("--coarse-solver", type=int, default=2,
                    help="Psi's implicit solve on the heat workload: 2 the eigenbasis on the BF16 matrix cores "
                         "(28 ms), 1 CG to --coarse-rtol (35 ms), 0 the FP64 eigenbasis (46 ms)")
    ap.add_argument("--cg-guess", type=int, default=0,
                    help="start of the fine CG solves: 0 the previous point's value, 1 the extrapolated iterate "
                         "(fewer CG iterations, a slower sweep here)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-coarse-propagator comparison")
    ap.add_argument("--learned-epochs", type=int, default=15)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-solve leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the c1 and c3 solves")
    ap.add_argument("--no-k-study", action="store_true", help="skip the 1D heat k-study leg")
    ap.add_argument("--no-three-level", action="store_true", help="skip the three-level V-cycle leg")
    ap.add_argument("--no-nested", action="store_true", help="skip the nested-iteration leg")
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline solves only (no context solves, no other legs): for profiling runs")
    ap.add_argument("--batch-count", type=int, default=256,
                    help="instances of the seeded batched workload (the first N of the 256)")
    ap.add_argument("--batch-sample", type=int, default=16,
                    help="instances solved one at a time (every k-th) for the batched-vs-individual comparison")
    ap.add_argument("--cpu-steps", type=int, default=4096,
                    help="time steps of the oracle's sequential stepping timed for cpu_baseline")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB mebibytes 5 times (the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def calibrate_copy(mib):
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_read": n * 8, "calibrate_copy_bytes_written": n * 8, "launches": 5}))


def cpu_baseline(p, u0, steps):
    """The oracle (test infrastructure) timed on the host: sequential time stepping, 1 thread."""
    import oracle
    import workloads as W
    oracle.build()
    oracle.set_threads(1)
    q = W.Problem(**{**p.__dict__, "nt": steps, "tf": p.t0 + steps * p.dt})
    t0 = time.perf_counter()
    oracle.sequential(q, u0)
    dt = time.perf_counter() - t0
    return {
        "value": p.n * steps / dt, "unit": "space-time point-updates/s", "cores": 1, "kind": "oracle",
        "sample": f"oracle sequential time stepping (exact forward solve, residual 0) of the first {steps} "
                  f"of {p.nt} steps of the same workload, 1 thread, {dt:.2f} s",
    }


def learned_leg(epochs):
    """Learned vs plain coarse propagator on 2D Allen-Cahn 128x128 periodic, eps 0.03, Nt 4096, m 32: train the
    CNN on the GPU (pairs of the fine propagator), then time both solves to the same 1e-8 residual."""
    import torch

    import paper_2107_09596_amd as atm
    import workloads as W
    from paper_2107_09596_amd import learned

    p, o, u0 = W.config("c5")
    rc = W.cnn_training_recipe()
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    frames = learned.trajectory_frames(p, W.ac2d_fields(rc["n_train_traj"], p.nx, p.ny, rc["train_seed"]),
                                       stride=rc["stride"], device=dev)
    vframes = learned.trajectory_frames(p, W.ac2d_fields(rc["n_val_traj"], p.nx, p.ny, rc["val_seed"]),
                                        stride=rc["stride"], device=dev)
    gen_s = time.perf_counter() - t0
    per = p.nt // rc["stride"] + 1
    lag = rc["lag"] // rc["stride"]
    ix, iy = learned.pair_indices(rc["n_train_traj"], per, lag, rc["n_pairs"])
    vx, vy = learned.pair_indices(rc["n_val_traj"], per, lag, rc["n_val_traj"] * (per - lag))
    params = torch.from_numpy(W.cnn_init(rc["train_seed"])).to(dev)
    losses, train_s = learned.train(params, frames, ix, iy, W.cnn_epoch_orders(rc["train_seed"], len(ix), epochs))
    val_loss = learned.mean_loss(params, vframes, vx, vy)
    guess = torch.from_numpy(W.initial_guess(p, u0)).to(dev)
    o.profile = 1
    res = {}
    for name, opts in (("plain", o), ("plain_bf16", W.Options(**{**o.__dict__, "coarse_solver": 2})),
                       ("learned", W.Options(**{**o.__dict__, "coarse_form": 3, "cnn_params": params}))):
        ws = atm.workspace(atm.atm_workspace_bytes(p, opts), device=dev)
        runs = []
        for _ in range(2):  # the first run warms up
            u = guess.clone()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            status, hist, st = atm.atm_solve(p, opts, u, ws=ws, allow=(atm.ATM_OK, atm.ATM_NOT_CONVERGED))
            torch.cuda.synchronize()
            runs.append(((time.perf_counter() - ts) * 1e3, status, hist, st))
        ms, status, hist, st = runs[-1]
        res[name] = {"ms": ms, "status": int(status), "cycles": st["iterations"], "final_residual": st["final_residual"],
                     "learned_cycles": st["learned_cycles"], "ms_coarse": st["ms_coarse"], "ms_sweep": st["ms_sweep"],
                     "value": p.n * p.nt / (ms / 1e3)}
        del ws
    res["speedup_learned_over_plain"] = res["plain"]["ms"] / res["learned"]["ms"]
    res["speedup_learned_over_plain_bf16"] = res["plain_bf16"]["ms"] / res["learned"]["ms"]
    res["speedup_with_training_amortised_over_one_solve"] = res["plain"]["ms"] / (res["learned"]["ms"] + train_s * 1e3)
    res["training"] = {"pairs": len(ix), "epochs": epochs, "batch": 64, "lr": 1e-3, "seconds": train_s,
                       "data_generation_seconds": gen_s, "final_train_loss": losses[-1], "validation_loss": val_loss}
    res["workload"] = ("2D Allen-Cahn 128x128 periodic, eps=0.03, dt=1e-5, Nt=4096, m=32, k=%d, FCF, precision %d, "
                       "tol 1e-8; plain = Psi in the FP64 eigenbasis; plain_bf16 = Psi in the eigenbasis on BF16 matrix "
                       "cores (FAS in terms of e = w - v); learned = CNN 1-32-32-32-1 (BF16, FP32 accumulate) as Psi in "
                       "the FAS windows, plain Psi as fallback" %
                       (o.k, o.precision))
    return res


def config_leg(name, runs):
    """One more workload of the suite (c1: 1D heat FP64; c3: 2D Allen-Cahn 256x256, FP32 fine / FP64
    residual, large-grid kernels): `runs` timed solves after one warm-up (c1) or a single solve."""
    import torch

    import paper_2107_09596_amd as atm
    import workloads as W

    p, o, u0 = W.config(name)
    dev = torch.device("cuda:0")
    guess = torch.from_numpy(W.initial_guess(p, u0)).to(dev)
    u = torch.empty_like(guess)
    ws = atm.workspace(atm.atm_workspace_bytes(p, o), device=dev)
    times = []
    # runs > 1: timed without the per-phase events (best of the runs after the first), then one more
    # solve with them for the phase split; a single run is profiled (its events cost nothing against it)
    profiled = [0] * runs + [1] if runs > 1 else [1]
    for r, prof in enumerate(profiled):
        o.profile = prof
        u.copy_(guess)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        status, hist, st = atm.atm_solve(p, o, u, ws=ws, allow=(atm.ATM_OK,))
        torch.cuda.synchronize()
        times.append((time.perf_counter() - ts) * 1e3)
        print(f"# {name} run {r}: {st['iterations']} cycles, {times[-1]:.1f} ms", file=sys.stderr, flush=True)
    ms = times[0] if runs == 1 else min(times[1:runs])
    graph = None
    if name == "c1":
        # the same solve through the batched entry with one instance: one captured cycle per graph replay and
        # the stopping decision on the device (the host reads the state every 4 cycles)
        ug = guess.clone()
        b = atm.Batch([p], [o], [ug])
        gms = []
        for _ in range(4):
            ug.copy_(guess)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            _, gstatus, gstats, _, _, _ = b.run(use_graph=True, check_every=4)
            torch.cuda.synchronize()
            gms.append((time.perf_counter() - ts) * 1e3)
        b.close()
        graph = {"ms": min(gms[1:]), "value": p.n * p.nt / (min(gms[1:]) / 1e3), "cycles": gstats[0]["iterations"],
                 "final_residual": gstats[0]["final_residual"], "status": int(gstatus[0]),
                 "max_abs_diff_to_atm_solve": float((ug - u).abs().max()),
                 "timed": "best of 3 after a run with the autotuner"}
    out = {"value": p.n * p.nt / (ms / 1e3), "unit": "space-time point-updates/s", "ms": ms,
            "iterations": st["iterations"], "final_residual": st["final_residual"], "stopping_norm": hist[-1],
            "phase_ms": {k: st[k] for k in ("ms_sweep", "ms_coarse", "ms_norm")},
            "cg_iters": {"fine": st["cg_fine"], "coarse": st["cg_coarse"]},
            "timed": "single solve" if runs == 1 else "best of %d after a warm-up (phase split from one more, profiled, solve)" % (runs - 1),
            "workload": {"c1": "1D heat nx=63, Nt=1024, m=16, k=7, FCF, FP64, tol 1e-8",
                         "c3": "2D Allen-Cahn 256x256 periodic, eps 0.02, dt 1e-5, Nt=8192, m=64, k=%d, FCF, "
                               "4 coarse substeps, FP32 fine / FP64 residual, tol 1e-8" % o.k}[name]}
    if graph is not None:
        out["graph_captured_cycle"] = graph
    return out


K_STUDY = {128: (2, 4, 6, 8, 10, 12, 16, 128), 64: (4, 8, 12, 16, 20, 24, 32, 256),
           32: (8, 16, 24, 32, 40, 48, 64, 512)}


def k_study_leg(runs=2):
    """The k-study of section 4.3 on the GPU: the manufactured 1D heat problem with 1025 grid points
    (1023 unknowns) and 16384 time points, random initial guess, two-level AT-MGRIT with
    F-relaxation and tol 1e-7, for three coarsening factors and a range of k.  Each entry: cycles,
    best wall time of `runs` solves, and the largest error against the exact solution."""
    import torch
    import paper_2107_09596_amd as atm
    import workloads as W
    dev = torch.device("cuda:0")
    p, u0, src, ug = W.heat1d_forced()
    exact = torch.from_numpy(W.heat1d_forced_exact(p)).to(dev)
    srcd = torch.from_numpy(src).to(dev)
    guess = torch.from_numpy(ug).to(dev)
    u = torch.empty_like(guess)
    table = {}
    for m, ks in K_STUDY.items():
        rows = []
        for k in ks:
            o = W.k_study_options(m, k)
            ws = atm.workspace(atm.atm_workspace_bytes(p, o), device=dev)
            best = None
            for _ in range(runs):
                u.copy_(guess)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                status, hist, st = atm.atm_solve(p, o, u, ws=ws, source=srcd, allow=(atm.ATM_OK,))
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
                best = ms if best is None else min(best, ms)
            err = float((u - exact).abs().max())
            rows.append({"k": k, "k_over_C": k / (p.nt // m + 1), "cycles": st["iterations"], "ms": best,
                         "value": p.n * p.nt / (best / 1e3), "final_residual": hist[-1], "err_exact": err})
            if m == 128:  # the residual histories of the paper's convergence figure (m = 128)
                rows[-1]["history"] = list(hist)
            print(f"# k-study m={m} k={k}: {st['iterations']} cycles, {best:.1f} ms", file=sys.stderr, flush=True)
        par = rows[-1]["cycles"]
        sat = min(r["k"] for r in rows if r["cycles"] <= par)
        table[str(m)] = {"C_points": p.nt // m + 1, "runs": rows, "parareal_cycles": par,
                         "smallest_k_at_parareal_cycles": sat, "saturation_ratio": sat / (p.nt // m + 1)}
    return {"workload": "1D heat u_t - u_xx = b on [0,3] x [0,pi], u = sin(pi x) cos t, 1023 unknowns, "
                        "nt 16383, random guess U[-1,1], F-relaxation, tol 1e-7, FP64",
            "unit": "space-time point-updates/s", "by_m": table}


def three_level_leg(runs=2):
    """Three-level FAS AT-MGRIT (Alg. 2) against three-level MGRIT (the coarsest grid global) as in
    the paper's three-level table: 2D heat 128 x 128, dt 1/4096, 16384 steps, m = 64 (256 level-1
    points), m_coarse in {2, 4, 8, 16}, k = N_2 / 2, FCF, tol 1e-8; plus two-level AT-MGRIT with the
    same m.  Each entry: V-cycles, best wall time of `runs` solves, phase split of one more solve."""
    import torch
    import paper_2107_09596_amd as atm
    import workloads as W
    dev = torch.device("cuda:0")

    def timed(p, o, guess, u):
        ws = atm.workspace(atm.atm_workspace_bytes(p, o), device=dev)
        best = None
        for _ in range(runs):
            u.copy_(guess)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            status, hist, st = atm.atm_solve(p, o, u, ws=ws, allow=(atm.ATM_OK,))
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            best = ms if best is None else min(best, ms)
        o2 = W.Options(**{**o.__dict__, "profile": 1})
        u.copy_(guess)
        _, _, sp = atm.atm_solve(p, o2, u, ws=ws, allow=(atm.ATM_OK,))
        return {"k": o.k, "cycles": st["iterations"], "ms": best, "value": p.n * p.nt / (best / 1e3),
                "final_residual": hist[-1], "phase_ms": {key: sp[key] for key in ("ms_sweep", "ms_coarse", "ms_norm")}}

    rows = []
    p = None
    for mc in (2, 4, 8, 16):
        p, o, u0 = W.three_level_config(mc)
        guess = torch.from_numpy(W.initial_guess(p, u0)).to(dev)
        u = torch.empty_like(guess)
        n2 = (p.nt // o.m) // mc
        at = timed(p, o, guess, u)
        mg = timed(p, W.Options(**{**o.__dict__, "k": n2 + 1}), guess, u)
        # the same with the coarsest windows on the BF16 matrix cores (level 1 by CG)
        atb = timed(p, W.Options(**{**o.__dict__, "coarse_solver": 2}), guess, u)
        mgb = timed(p, W.Options(**{**o.__dict__, "k": n2 + 1, "coarse_solver": 2}), guess, u)
        rows.append({"m_coarse": mc, "coarsest_points": n2 + 1, "at_mgrit": at, "mgrit": mg,
                     "speedup_vs_mgrit": mg["ms"] / at["ms"], "at_mgrit_bf16_coarsest": atb,
                     "mgrit_bf16_coarsest": mgb, "speedup_vs_mgrit_bf16_coarsest": mgb["ms"] / atb["ms"]})
        print(f"# three levels m_coarse={mc}: AT-MGRIT k={o.k} {at['cycles']} cycles {at['ms']:.1f} ms, "
              f"MGRIT {mg['cycles']} cycles {mg['ms']:.1f} ms; coarsest on BF16: AT-MGRIT {atb['cycles']} cycles "
              f"{atb['ms']:.1f} ms, MGRIT {mgb['cycles']} cycles {mgb['ms']:.1f} ms", file=sys.stderr, flush=True)
    p, o, u0 = W.three_level_config(4)
    guess = torch.from_numpy(W.initial_guess(p, u0)).to(dev)
    u = torch.empty_like(guess)
    two = {}
    for k in (W.default_k(p.nt // o.m), (p.nt // o.m) // 2):
        two[str(k)] = timed(p, W.Options(**{**o.__dict__, "levels": 2, "k": k, "coarse_solver": 1}), guess, u)
        two[str(k) + "_bf16"] = timed(p, W.Options(**{**o.__dict__, "levels": 2, "k": k, "coarse_solver": 2}), guess, u)
        print(f"# two levels m=64 k={k}: {two[str(k)]['cycles']} cycles {two[str(k)]['ms']:.1f} ms (Psi by CG), "
              f"{two[str(k) + '_bf16']['cycles']} cycles {two[str(k) + '_bf16']['ms']:.1f} ms (Psi on BF16)",
              file=sys.stderr, flush=True)
    return {"workload": "2D heat 128x128 interior, nu=0.1, dt=1/4096, Nt=16384, m=64, FCF, tol 1e-8, FP64, "
                        "Psi by CG to 1e-12",
            "unit": "space-time point-updates/s", "three_level": rows, "two_level_m64": two}


def nested_leg(runs=2):
    """Nested iteration (section 2.2) against the plain zero guess: the headline 2D heat solve (two
    levels) and the three-level workload with m_coarse 4; setup time, cycles and total time."""
    import torch
    import paper_2107_09596_amd as atm
    import workloads as W
    dev = torch.device("cuda:0")
    out = {}
    p2, o2, u02 = W.config("c2")
    o2.coarse_solver = 2
    p3, o3, u03 = W.three_level_config(4)
    for name, p, o, u0 in (("c2_two_level", p2, o2, u02), ("three_level_m_coarse4", p3, o3, u03)):
        guess = torch.from_numpy(W.initial_guess(p, u0)).to(dev)
        u = torch.empty_like(guess)
        row = {}
        for nested in (0, 1):
            oo = W.Options(**{**o.__dict__, "nested": nested})
            ws = atm.workspace(atm.atm_workspace_bytes(p, oo), device=dev)
            best = None
            for _ in range(runs):
                u.copy_(guess)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                status, hist, st = atm.atm_solve(p, oo, u, ws=ws, allow=(atm.ATM_OK,))
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
                if best is None or ms < best[0]:
                    best = (ms, hist, st)
            ms, hist, st = best
            row["nested" if nested else "zero_guess"] = {
                "cycles": st["iterations"], "ms": ms, "ms_setup": st["ms_setup"], "initial_residual": hist[0],
                "final_residual": hist[-1], "value": p.n * p.nt / (ms / 1e3)}
            print(f"# nested={nested} {name}: {st['iterations']} cycles, setup {st['ms_setup']:.1f} ms, "
                  f"total {ms:.1f} ms, initial residual {hist[0]:.2e}", file=sys.stderr, flush=True)
        out[name] = row
    return out


def batch_leg(count, sample):
    """Batched solves: the first `count` instances of the seeded batch (1D heat, 2D heat and 2D Allen-Cahn of
    uneven sizes; FP32-fine / FP64-residual for 2D), one captured cycle per graph replay.  The first run
    includes the autotuner; the second is timed.  A sample of the instances is also solved one at a time
    with atm_solve and the sum extrapolated to the whole batch."""
    import numpy as np
    import torch

    import paper_2107_09596_amd as atm
    import workloads as W

    items = W.batch_config(256)[:count]
    dev = torch.device("cuda:0")
    guess = []
    for p, _, u0 in items:
        g = torch.zeros((p.nt + 1, p.n), dtype=torch.float64, device=dev)
        g[0].copy_(torch.from_numpy(np.ascontiguousarray(u0, dtype=np.float64).reshape(-1)))
        guess.append(g)
    us = [g.clone() for g in guess]
    b = atm.Batch([p for p, _, _ in items], [o for _, o, _ in items], us)
    runs = []
    for r in range(2):
        for u, g in zip(us, guess):
            u.copy_(g)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        st, status, stats, hists, ms, mt = b.run(use_graph=True, check_every=4)
        torch.cuda.synchronize()
        runs.append(((time.perf_counter() - ts) * 1e3, status, stats, ms, mt))
        print(f"# batch run {r}: {ms:.1f} ms solve, {mt:.1f} ms tuning", file=sys.stderr, flush=True)
    wall, status, stats, ms, _ = runs[-1]
    tuning = b.tuning()
    tune_ms = runs[0][4]
    b.close()
    pts = sum(p.nt * p.n for p, _, _ in items)
    cycles = [s["iterations"] for s in stats]
    # one at a time: every k-th instance, extrapolated by count / sample size
    step = max(1, count // max(sample, 1))
    idx = list(range(0, count, step))[:sample]
    one_ms = 0.0
    for i in idx:
        p, o, u0 = items[i]
        u = guess[i].clone()
        ws = atm.workspace(atm.atm_workspace_bytes(p, o), device=dev)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        atm.atm_solve(p, o, u, ws=ws, allow=(atm.ATM_OK,))
        torch.cuda.synchronize()
        one_ms += (time.perf_counter() - ts) * 1e3
        del ws, u
    one_ms_all = one_ms * count / len(idx)
    kinds = [p.kind for p, _, _ in items]
    return {
        "value": pts / (wall / 1e3), "unit": "space-time point-updates/s", "ms": wall, "ms_solve_reported": ms,
        "instances": count, "space_time_points": pts,
        "mix": {"heat1d": kinds.count(W.HEAT1D), "heat2d": kinds.count(W.HEAT2D), "ac2d": kinds.count(W.AC2D)},
        "all_converged": all(s == atm.ATM_OK for s in status),
        "cycles": {"min": min(cycles), "mean": float(np.mean(cycles)), "max": max(cycles)},
        "max_final_residual": max(s["final_residual"] for s in stats),
        "autotuner": {"order": ["natural", "longest_first"][tuning[1]], "tiles": ["generic32", "per_instance"][tuning[2]],
                      "ms": tune_ms},
        "one_at_a_time": {"sample": len(idx), "every": step, "ms_sample": one_ms, "ms_extrapolated": one_ms_all,
                          "speedup_of_batch": one_ms_all / wall},
        "workload": "seeded batch of %d: 1D heat nx 63..511 (FP64), 2D heat and periodic 2D Allen-Cahn n x n, "
                    "n 32..128 (FP32 fine / FP64 residual; Psi on BF16 matrix cores for 2D heat and one-substep "
                    "Allen-Cahn), Nt 512..8192, "
                    "m in {8,16,32}, k = max(2, ceil(0.1 (N_T+1))), "
                    "FCF, tol 1e-8" % count,
    }


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the time-parallel path is built "
              "for a single GPU, and sharding its intervals over several GPUs is not built", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2107_09596_amd as atm
    import workloads as W

    p, o, u0 = W.config(args.config)
    o.profile = 1
    o.coarse_cg_rtol = args.coarse_rtol
    o.coarse_solver = args.coarse_solver
    o.cg_guess = args.cg_guess
    dev = torch.device("cuda:0")
    guess = torch.from_numpy(W.initial_guess(p, u0)).to(dev)
    u = torch.empty_like(guess)
    ws = atm.workspace(atm.atm_workspace_bytes(p, o), device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        u.copy_(guess)
        return atm.atm_solve(p, o, u, ws=ws, allow=(atm.ATM_OK,))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    agg = {"ms_sweep": 0.0, "ms_coarse": 0.0, "ms_norm": 0.0, "cg_fine": 0, "cg_coarse": 0, "fine_steps": 0,
           "coarse_steps": 0, "n_sweeps": 0, "iterations": 0}
    last = None
    t0 = time.perf_counter()
    for i in range(args.steps):
        status, hist, st = step()
        for key in agg:
            agg[key] += st[key]
        last = (hist, st)
        print(f"# step {i + 1}/{args.steps}: {st['iterations']} cycles, residual {hist[-1]:.3e}, "
              f"{st['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = p.n * p.nt / (ms_per_step / 1e3)

    # roofline of the dominant kernel: the relaxation sweep (FP64 VALU-bound CG)
    sweep_flops = p.n * (FLOPS_PER_CG_ITER_POINT * agg["cg_fine"] + FLOPS_PER_SOLVE_POINT * agg["fine_steps"])
    achieved = sweep_flops / (agg["ms_sweep"] / 1e3) / 1e12 if agg["ms_sweep"] > 0 else 0.0
    roofline = {
        "kernel": ("sweep2d_xg_kernel" if o.cg_guess == 1 else "sweep2d_kernel")
                  + " (FCF/F relaxation + correction sweeps)",
        "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64_VECTOR_TFLOPS, "traffic": sum(SWEEP_TRAFFIC_BYTES),
        "traffic_read_write": list(SWEEP_TRAFFIC_BYTES),
        "avg_launch_ms": agg["ms_sweep"] / max(agg["n_sweeps"], 1),
        "launches": agg["n_sweeps"],
        # the resource a busy workgroup saturates: LDS traffic of its CG iterations (whole chip)
        "lds": {"achieved": (p.n * LDS_BYTES_PER_CG_ITER_POINT * agg["cg_fine"] / (agg["ms_sweep"] / 1e3) / 1e12
                             if agg["ms_sweep"] > 0 else 0.0),
                "peak": PEAK_LDS_TBS, "unit": "TB/s"},
    }
    roofline["lds"]["frac"] = roofline["lds"]["achieved"] / PEAK_LDS_TBS

    out = {
        "metric": "space-time point-updates/s to 1e-8 residual",
        "value": value, "unit": "space-time point-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config}: 2D heat 128x128 interior, nu=0.1, Nt=4096 on [0,1], m=32, "
                               f"k={o.k}, FCF, backward Euler + Jacobi-PCG rtol 1e-12 ("
                               + {0: "Psi solved in the eigenbasis",
                                  2: "Psi solved in the eigenbasis on BF16 matrix cores, split operands"}.get(
                                   args.coarse_solver, f"Psi's CG rtol {args.coarse_rtol:g}") + ")"
                               + (", fine CG started from the extrapolated iterate" if o.cg_guess == 1 else "")
                               + ", tol 1e-8, FP64",
                   "global_batch": 1, "seq_len": p.nt, "parallelism": "time-parallel, 1 GPU"},
        "iterations": last[1]["iterations"], "final_residual": last[0][-1],
        "phase_ms_per_step": {k: agg[k] / args.steps for k in ("ms_sweep", "ms_coarse", "ms_norm")},
        "cg_iters_per_step": {"fine": agg["cg_fine"] / args.steps, "coarse": agg["cg_coarse"] / args.steps},
        "roofline": roofline,
    }
    if args.only_headline:
        print(json.dumps(out), flush=True)
        return

    # context: the same solve with Psi's CG at the fine tolerance
    o_strict = W.Options(**{**o.__dict__, "coarse_cg_rtol": 0.0, "coarse_solver": 1})
    u.copy_(guess)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    _, hist_s, st_s = atm.atm_solve(p, o_strict, u, ws=ws, allow=(atm.ATM_OK,))
    torch.cuda.synchronize()
    strict = {"ms": (time.perf_counter() - ts) * 1e3, "iterations": st_s["iterations"],
              "final_residual": hist_s[-1], "ms_coarse": st_s["ms_coarse"], "cg_coarse": st_s["cg_coarse"]}
    strict["value"] = p.n * p.nt / (strict["ms"] / 1e3)
    u_strict = u.clone()

    # context: the headline solve with the other start of the fine CG solves
    o_other = W.Options(**{**o.__dict__, "cg_guess": 1 - o.cg_guess})
    other_runs = []
    for _ in range(2):  # the first run warms up
        u.copy_(guess)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _, hist_o, st_o = atm.atm_solve(p, o_other, u, ws=ws, allow=(atm.ATM_OK,))
        torch.cuda.synchronize()
        other_runs.append(((time.perf_counter() - ts) * 1e3, hist_o, st_o))
    ms_o, hist_o, st_o = other_runs[-1]
    other_start = {"cg_guess": o_other.cg_guess, "ms": ms_o, "value": p.n * p.nt / (ms_o / 1e3),
                   "iterations": st_o["iterations"], "final_residual": hist_o[-1], "ms_sweep": st_o["ms_sweep"],
                   "cg_fine": st_o["cg_fine"],
                   "avg_sweep_launch_ms": st_o["ms_sweep"] / max(st_o["n_sweeps"], 1)}

    # the FP32-fine / FP64-residual form of the same solve (stops on the FP64 implicit residual, which
    # bounds the paper-form residual; the final paper-form residual is reported)
    o_mixed = W.Options(**{**o.__dict__, "precision": 1, "cg_guess": 0})
    ws_m = atm.workspace(atm.atm_workspace_bytes(p, o_mixed), device=dev)
    mixed_runs = []
    for _ in range(2):  # the first run warms up
        u.copy_(guess)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _, hist_m, st_m = atm.atm_solve(p, o_mixed, u, ws=ws_m, allow=(atm.ATM_OK,))
        torch.cuda.synchronize()
        mixed_runs.append(((time.perf_counter() - ts) * 1e3, hist_m, st_m))
    ms_m, hist_m, st_m = mixed_runs[-1]
    u_mixed = u.clone()
    mixed = {"value": p.n * p.nt / (ms_m / 1e3), "ms": ms_m, "iterations": st_m["iterations"],
             "stopping_norm": hist_m[-1], "final_residual": st_m["final_residual"],
             "phase_ms": {k: st_m[k] for k in ("ms_sweep", "ms_coarse", "ms_norm")},
             "cg_iters": {"fine_fp32": st_m["cg_fine"], "coarse_fp64": st_m["cg_coarse"]}}

    # context: sequential time stepping on the same GPU (one workgroup; the paper's baseline method)
    useq = torch.zeros_like(guess)
    useq[0].copy_(guess[0])
    torch.cuda.synchronize()
    ts = time.perf_counter()
    atm.atm_sequential(p, useq)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - ts
    max_diff = float((useq - u_strict).abs().max())
    mixed["max_abs_diff_to_gpu_sequential"] = float((useq - u_mixed).abs().max())

    out["strict_coarse"] = strict
    out["plain_cg_start" if o.cg_guess == 1 else "extrapolated_cg_start"] = other_start
    out["mixed_precision"] = mixed
    out["gpu_sequential"] = {"value": p.n * p.nt / seq_s, "ms": seq_s * 1e3,
                             "speedup_of_atmgrit": seq_s * 1e3 / ms_per_step, "max_abs_diff_to_atmgrit": max_diff}
    if not args.no_learned:
        out["learned_coarse"] = learned_leg(args.learned_epochs)
    if not args.no_batch:
        out["batched"] = batch_leg(args.batch_count, args.batch_sample)
    if not args.no_configs:
        out["other_configs"] = {"c1": config_leg("c1", 4), "c3": config_leg("c3", 1)}
    if not args.no_k_study:
        out["k_study"] = k_study_leg()
    if not args.no_three_level:
        out["three_level"] = three_level_leg()
    if not args.no_nested:
        out["nested_iteration"] = nested_leg()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, u0, min(args.cpu_steps, p.nt))
        out["cpu_baseline"]["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
