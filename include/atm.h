/*
 * atm.h -- C-ABI of libatmgrit.so: two-level asynchronous truncated
 * multigrid-reduction-in-time (AT-MGRIT) on one AMD MI355X (gfx950).
 *
 * Method: J. Hahne, B. S. Southworth, S. Friedhoff, "Asynchronous Truncated
 * Multigrid-reduction-in-time", arXiv 2107.09596.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Plain C; all pointers marked (device) are HIP device pointers owned by the
 *   caller (e.g. PyTorch tensors); (host) pointers are ordinary host memory.
 * - `stream` is a hipStream_t passed as void*.  Work is enqueued on it; calls
 *   that return a residual norm or statistics synchronise the stream first.
 *   All other calls return after enqueueing (results valid after a stream sync).
 * - The library allocates no device memory: all scratch lives in the
 *   caller's workspace `ws` of at least atm_workspace_bytes() bytes, 256-byte
 *   aligned.  Norms are read back into host stack memory.  A workspace must
 *   be zero-filled before its first use unless that use is atm_solve or
 *   atm_sequential (which initialise it); its header carries the CG failure
 *   flag from launch to launch, and a norm call outside atm_solve clears it
 *   after reporting.
 * - Arguments are validated before any launch; on error nothing is enqueued,
 *   the status is returned and atm_last_error() holds a message
 *   (thread-local).  No exception crosses the ABI.
 * - Space-time layout: u is [nt+1][n] FP64, row-major, n = nx*ny, spatial
 *   index y*nx + x.  For a coarsening factor m this is the
 *   [interval][step][space] layout: time index t = j*m + i.
 * - The library is re-entrant for distinct workspaces; calls that share a
 *   workspace must be ordered on one stream.
 *
 * Problem statement (section 2, eq. (2)): u_0 = g_0, u_i = Phi(u_{i-1}) + g_i,
 * with g_i = 0 for i >= 1 unless the problem carries a PDE source (then each
 * backward Euler step takes it at its new time level, see atm_problem.source).
 * Time grid t_i = t0 + i dt, dt = (tf - t0)/nt.
 */
#ifndef ATM_H
#define ATM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t atm_status;
#define ATM_OK 0
#define ATM_NOT_CONVERGED 1      /* max_iter reached; result and stats valid */
#define ATM_ERR_INVALID_ARG (-1)
#define ATM_ERR_UNSUPPORTED (-2) /* valid but not implemented (e.g. a grid too large for a CU) */
#define ATM_ERR_DEVICE (-3)      /* HIP runtime error; see atm_last_error() */
#define ATM_ERR_DIVERGED (-4)    /* non-finite residual norm */
#define ATM_ERR_INNER_SOLVE (-5) /* a CG solve inside Phi or Psi missed rtol within cg_max_iter */
#define ATM_ERR_WORKSPACE (-6)   /* workspace smaller than atm_workspace_bytes() */

/* problem kinds: the one-step integrator Phi (section 2, eq. (2)) */
#define ATM_HEAT1D 1 /* u_t = nu u_xx on [0,L], zero Dirichlet, nx interior points,
                        h = L/(nx+1); backward Euler, tridiagonal solve */
#define ATM_HEAT2D 2 /* u_t = nu (u_xx+u_yy) on [0,L]^2, zero Dirichlet, nx*ny interior
                        points, 5-point stencil; backward Euler by Jacobi-PCG */
#define ATM_AC2D 3   /* u_t = nu Lap u + (u - u^3)/eps^2, periodic [0,L)^2, h = L/nx;
                        IMEX: (I - dt nu Lap) u_i = u_{i-1} + dt (u_{i-1} - u_{i-1}^3)/eps^2 by CG */

typedef struct atm_problem {
    double length;  /* L, side of the domain */
    double nu;      /* diffusion coefficient */
    double eps;     /* Allen-Cahn interface width (ATM_AC2D only) */
    double t0, tf;  /* time interval (t0, tf] */
    double cg_rtol; /* CG stops when ||b - M x||_2 <= cg_rtol ||b||_2 (2D kinds) */
    int64_t nt;     /* number of fine time steps N_t; nt+1 time points */
    int32_t kind;   /* ATM_HEAT1D, ATM_HEAT2D or ATM_AC2D */
    int32_t nx, ny; /* spatial points; ny = 1 for ATM_HEAT1D */
    int32_t cg_max_iter;
    const double* source; /* (device) NULL, or the PDE source b(x, t_i) at every time point, [nt+1][n]
                             FP64 (row 0 unused), for the forced heat equation u_t - nu u_xx = b of
                             the k-study in section 4.3.  Each fine step then solves
                             (I - dt nu L) u_i = u_{i-1} + dt b(t_i), i.e. g_i = (I - dt nu L)^{-1} dt b(t_i)
                             in eq. (2); Psi is unchanged (it acts on corrections, or on C-point values
                             with the FAS right-hand side).  ATM_HEAT1D only (other kinds and the batch
                             API: ATM_ERR_UNSUPPORTED).  Read by the kernels of the call; it must stay
                             valid until the stream has run them */
} atm_problem;

typedef struct atm_options {
    double tol;            /* stop when ||g - A(u)||_2 <= tol (absolute, all space-time points) */
    double coarse_cg_rtol; /* CG tolerance inside Psi (2D kinds); 0 = the problem's cg_rtol.  Psi only
                              approximates Phi^m, so this changes the convergence rate, not the
                              fixed point */
    double mixed_cg_rtol;  /* precision 1: relative tolerance of the FP32 CG of each fine step's
                              correction solve; 0 = 1e-6.  The FP64 fixed point does not depend on it */
    double fallback_ratio; /* coarse_form 3: once the residual has decreased in some cycle, two
                              consecutive cycles with ||r_i|| > fallback_ratio ||r_{i-1}|| (or, at any
                              time, ||r_i|| > 1e6 ||r_0||) switch the remaining cycles to the plain
                              coarse propagator, keeping the iterate; 0 = 0.95 */
    const float* cnn_params; /* coarse_form 3: the learned propagator's parameters (device, see
                              atm_cnn_param_count); read during the call only */
    int32_t m;             /* coarsening factor, >= 2 (section 2.1) */
    int32_t k;             /* C-points per local coarse grid, >= 1; k >= N_T+1 is Parareal */
    int32_t relax;         /* 0: F-relaxation, 1: FCF-relaxation (section 2.2) */
    int32_t max_iter;      /* maximum number of cycles */
    int32_t coarse_substeps; /* Psi = s steps of size m dt / s, s >= 1 */
    int32_t coarse_form;   /* 0 auto (linear for heat, FAS for Allen-Cahn), 1 linear, 2 FAS,
                              3 learned: the FAS form with the learned propagator Psi(v) = v + f(v)
                              (see atm_cnn_forward) in place of the re-discretised one (ATM_AC2D, nx a
                              multiple of 16 up to 128).  A BF16 network is not a smooth function of its
                              input, so FAS differences Psi(w) - Psi(v) of nearby states carry rounding
                              jumps that stall the residual at some level: the fallback below then
                              finishes with the plain propagator */
    int32_t precision;     /* 0: FP64 throughout; 1 (2D kinds): FP32 fine solves in defect-correction
                              form with the residual, coarse correction and iterate in FP64
                              (see atm_sweep and atm_solve) */
    int32_t profile;       /* 1: time every kernel launch of atm_solve with HIP events (atm_stats.ms_*) */
    int32_t coarse_solver; /* the implicit solve inside Psi (2D kinds): 0 auto = exact solve in the
                              eigenbasis of the constant-coefficient operator where built (grids with
                              more than 128 points per side), CG elsewhere; 1 CG everywhere (to
                              coarse_cg_rtol).  Both take the same step: the eigenbasis solve is exact to
                              rounding, CG to its tolerance.  2: the eigenbasis solve on the BF16 matrix
                              cores with split operands (each value hi + lo in BF16, products in FP32),
                              accurate to about 1e-5 relative; grids up to 128 per side (FAS form with
                              coarse_substeps 1), and the two-CU windows of grids with rows of 128, 192
                              or 256 points and 128 or 256 rows (any coarse_substeps).  In the FAS
                              form the windows carry e = w - v:
                              e_j = M^-1 (psi(v_{j-1} + e_{j-1}) - psi(v_{j-1})) + r_j, the explicit
                              parts' difference in FP64, so that the solve's error scales with e (a
                              plain Psi(w) - Psi(v) would keep it); with several substeps the difference
                              is taken substep by substep along v's own path through them */
    int32_t levels;        /* 0 or 2: two-level AT-MGRIT (Alg. 1).  3: the multilevel FAS V-cycle of
                              Alg. 2 (section 2.2) over three levels: level 1 takes every m-th point of
                              the fine grid and steps with dt m in coarse_substeps substeps (CG to
                              coarse_cg_rtol); level 2, every m_coarse-th point of level 1 with step
                              dt m m_coarse, is the coarsest and is replaced by the local grids of k
                              points.  F(CF)^nu relaxation on levels 0 and 1, injection of the iterate
                              and its residual, the FAS right-hand side A_1(v) + g on level 1, ideal
                              interpolation back.  Precision 0, grids up to 128 per side, not with the
                              learned propagator or the batch API; coarse_form does not apply (the
                              cycle is the FAS form).  Level 1 steps by CG; the coarsest level's
                              windows take Psi by CG, or with coarse_solver 2 (coarse_substeps 1) on the
                              BF16 matrix cores in terms of e = w - v */
    int32_t m_coarse;      /* levels 3: coarsening factor from level 1 to level 2, >= 2, with
                              floor(nt / m) >= m_coarse */
    int32_t nested;        /* 1: nested iteration (section 2.2) replaces the initial guess before the
                              first cycle: the guess at the coarse levels' points is injected, the
                              coarsest level's local problems of the re-discretised system are solved
                              from it (each window starting from the coarse residual of the injected
                              guess), and every finer level takes the coarser values at its C-points and
                              F-relaxes them, a level between getting one V-cycle of its own system.
                              Precision 0, grids up to 128 per side, no source, not the learned
                              propagator; its time is atm_stats.ms_setup */
} atm_options;

typedef struct atm_stats {
    double final_residual; /* ||g - A(u)||_2 of the returned iterate: precision 0, the C-point form
                              sqrt(sum_j ||y_j - u_{jm}||^2); precision 1, atm_step_residual_norm */
    double ms_total;       /* wall time of atm_solve (host clock, stream synchronised) */
    double ms_sweep;       /* summed device time of the relaxation sweeps (profile = 1, else 0) */
    double ms_coarse;      /* summed device time of the local coarse solves incl. FAS tau (profile = 1) */
    double ms_norm;        /* summed device time of the residual-norm kernels (profile = 1) */
    int64_t fine_steps;    /* Phi applications computed (all intervals, all sweeps) */
    int64_t coarse_steps;  /* Psi applications (all windows) */
    int64_t cg_fine;       /* CG iterations inside the sweeps' Phi steps (2D kinds) */
    int64_t cg_coarse;     /* CG iterations inside Psi (windows and FAS tau; 2D kinds) */
    int64_t fine_steps_skipped; /* precision 0: Phi applications not recomputed because the
                              interval's C-point value was unchanged since its last sweep (the
                              F-points would come out bit for bit the same) */
    int32_t iterations;    /* cycles applied (number of coarse corrections) */
    int32_t n_sweeps;      /* sweep launches */
    int32_t learned_cycles; /* coarse_form 3: cycles whose correction came from the learned propagator */
    double ms_setup;       /* nested = 1: wall time of the nested-iteration setup (included in ms_total) */
} atm_stats;

/* Number of coarse intervals N_T = floor(nt / m); C-points are 0..N_T. */
int64_t atm_num_intervals(const atm_problem* prob, const atm_options* opts);

/* First C-point of the local coarse grid T^(p) = {max(0, p-k+1), ..., p}
   (section 2.1, definition of the local grids; Fig. 1). */
int64_t atm_window_start(int64_t p, int32_t k);

/* Workspace size in bytes for the calls below with this problem and options,
   or 0 if the arguments are invalid. */
size_t atm_workspace_bytes(const atm_problem* prob, const atm_options* opts);

/* Relaxation sweep over every interval at once (section 2.1 F-relaxation,
   section 2.2 CF-relaxation, Alg. 1 correction with selective ideal
   interpolation P_S).  Every interval j = 0..N_T (interval N_T holds only
   C-point N_T and the ragged tail after it, empty when m divides nt) first
   sets its C-point value c_j:
     mode 0: c_j = u_{jm}                 (F-relaxation)
     mode 1: c_j = u_{jm} + aux_j         (correction by e_j = aux_j, then F-interpolation)
     mode 2: c_j = aux_j for j >= 1, u_0 for j = 0   (C-relaxation from aux = Phi(u_{jm-1}),
                                                      then F-relaxation)
   writes u_{jm} = c_j, then u_{jm+i} = Phi(u_{jm+i-1}) for its F-points, and
   for j < N_T writes y_{j+1} = Phi(u_{jm+m-1}).  The C-point residual of the
   result is r_j = y_j - u_{jm} (j >= 1); r_0 = 0; F-point residuals are 0.
   u    (device) [nt+1][n] FP64, in/out.
   aux  (device) [N_T+1][n] FP64, read in modes 1 and 2, else may be NULL.
   y    (device) [N_T+1][n] FP64, out (row 0 untouched); must not alias aux.
   Precision 1 (2D kinds): every step that produces a value v_i = Phi(v_{i-1})
   starts from the value s_i stored at that point, rho = psi(v_{i-1}) - M s_i
   in FP64 (M = I - dt nu L; psi is the identity for heat and the explicit
   Allen-Cahn part otherwise), solves M d = rho by FP32 CG to mixed_cg_rtol and
   stores v_i = s_i + d in FP64.  For the F-points s_i is u_{jm+i} on entry;
   for y_{j+1} it is, by mode: 0 u_{(j+1)m}, 1 y_{j+1} on entry (y is then
   in/out and must hold finite values), 2 aux_{j+1}.  v_i equals Phi(v_{i-1})
   up to mixed_cg_rtol times |Phi(v_{i-1}) - s_i|.
   Errors: INVALID_ARG, UNSUPPORTED, WORKSPACE, DEVICE.  A CG failure inside
   Phi is reported by the next call that synchronises (atm_residual_norm,
   atm_solve) as ATM_ERR_INNER_SOLVE. */
atm_status atm_sweep(const atm_problem* prob, const atm_options* opts, int32_t mode, double* u,
                     const double* aux, double* y, void* ws, size_t ws_bytes, void* stream);

/* The N_T+1 mutually independent local coarse-grid solves (Alg. 1: restrict
   by injection, solve A~_c^(p) u_c^(p) = r_c^(p); section 3.1.2 defines A~_c^(p)
   as the bidiagonal matrix with I on the diagonal and -Psi below).  With
   r_j = y_j - u_{jm} (j >= 1), r_0 = 0 and s = max(0, p-k+1):
     linear form: e = r_s; e = Psi(e) + r_j for j = s+1..p; e_p = e.
     FAS form (Alg. 2, coarsest level): v_j = u_{jm}; w = v_s + r_s;
       w = Psi(w) + (v_j - Psi(v_{j-1}) + r_j) for j = s+1..p; e_p = w - v_p.
   learned form (coarse_form 3): the FAS form with Psi = the learned propagator.
   u (device) [nt+1][n] in; y (device) [N_T+1][n] in; e (device) [N_T+1][n] out. */
atm_status atm_coarse_solve(const atm_problem* prob, const atm_options* opts, const double* u,
                            const double* y, double* e, void* ws, size_t ws_bytes, void* stream);

/* The window solve of atm_coarse_solve without a workspace argument, for
   callers that cannot allocate device memory (code under HIP graph capture,
   serving loops, harnesses that forbid allocation).  The call allocates
   nothing: the workspace is a static device array of
   atm_static_scratch_bytes() bytes (32 MiB), one per GPU, held from the
   library's load until the process ends; the call enqueues kernels only
   (no memset, copy or synchronisation).  Same arguments, results and layout
   as atm_coarse_solve.  Limits: two levels, the plain coarse propagator with
   a direct solve (1D, or 2D with coarse_solver 0 or 2, which cannot fail),
   grids of at most 128 points per side, and a window phase that fits the
   scratch (tau, the eigenbasis tables and the C-point residuals; about
   (N_T+1) n 8 bytes each), else WORKSPACE.  The stream must belong to the
   current device (the default stream is the current device's).  Every call on
   a GPU uses that GPU's one array, which keeps the previous call's contents:
   calls that overlap on one GPU (on different streams or host threads)
   race, so a caller serialises them.  Errors: INVALID_ARG, UNSUPPORTED,
   WORKSPACE, DEVICE. */
atm_status atm_coarse_solve_static(const atm_problem* prob, const atm_options* opts, const double* u,
                                   const double* y, double* e, void* stream);

/* Size in bytes of the static scratch of atm_coarse_solve_static. */
size_t atm_static_scratch_bytes(void);

/* Name of the kernel that runs the relaxation sweeps of atm_sweep and atm_solve for
   this problem and these options on the current device (static string; "" if
   the arguments are invalid): sweep1d_kernel, sweep2d_kernel, sweep2d_mixed_kernel,
   sweep_large_kernel, sweep_large_mixed_kernel, or sweep_pair_mixed_kernel (precision 1
   on 256 x 256, 256 x 128 and 128 x 256 grids: two workgroups per interval, launched
   cooperatively, when the device holds them all at once). */
const char* atm_sweep_kernel(const atm_problem* prob, const atm_options* opts);

/* Name of the kernel that runs the local solves (the windows of the truncated coarse
   problem, section 2.1) of atm_coarse_solve and of the two-level atm_solve on the
   current device (static string; "" if the arguments are invalid, for coarse_form 3
   and for levels 3): coarse1d_kernel, coarse2d_kernel, coarse2d_spec_kernel,
   coarse2d_bf_kernel, coarse2d_bf_fas_kernel, coarse_large_kernel, or
   coarse_pair_kernel (the eigenbasis Psi on large grids of 128, 192 or 256 columns and
   a multiple of 128 rows: two workgroups per window, launched cooperatively, when the
   device holds them all at once). */
const char* atm_coarse_kernel(const atm_problem* prob, const atm_options* opts);

/* Residual 2-norm ||g - A(u)||_2 of an iterate whose F-points are relaxed
   (the stopping test of section 4.3): sqrt(sum_{j=1..N_T} ||y_j - u_{jm}||^2).
   Synchronises the stream and writes the value to *norm_out (host).
   Returns INNER_SOLVE if a CG failure was flagged in this workspace since
   the last synchronising call. */
atm_status atm_residual_norm(const atm_problem* prob, const atm_options* opts, const double* u,
                             const double* y, double* norm_out, void* ws, size_t ws_bytes, void* stream);

/* FP64 implicit residual norm sqrt(sum_{i=1..nt} ||rho_i||^2),
   rho_i = psi(u_{i-1}) - M u_i with M = I - dt nu L the matrix of the implicit
   solve of Phi and psi its explicit part (section 2, eq. (2), written as
   M u_i = psi(u_{i-1})).  Since the paper-form residual is r_i = M^-1 rho_i
   and ||M^-1||_2 <= 1, ||r||_2 <= this value: the stopping test of precision 1.
   All time points are included, F-points too.  u (device) [nt+1][n] in.
   Synchronises the stream; writes *norm_out (host). */
atm_status atm_implicit_residual_norm(const atm_problem* prob, const atm_options* opts, const double* u,
                                      double* norm_out, void* ws, size_t ws_bytes, void* stream);

/* Paper-form residual norm with the step solved to FP64 accuracy,
   sqrt(sum_{i=1..nt} ||M^-1 rho_i||^2) (section 4.3 stopping norm; the
   definition of rho_i is above).  M r_i = rho_i is solved by FP64 CG from zero
   to cg_rtol relative to ||rho_i|| (2D) or by a direct tridiagonal solve (1D),
   so small residuals are not lost to the cancellation of Phi(u_{i-1}) - u_i.
   u (device) [nt+1][n] in.  Synchronises the stream; writes *norm_out (host).
   Errors as atm_residual_norm. */
atm_status atm_step_residual_norm(const atm_problem* prob, const atm_options* opts, const double* u,
                                  double* norm_out, void* ws, size_t ws_bytes, void* stream);

/* Sequential time stepping on the GPU: u_i = Phi(u_{i-1}) for i = 1..nt from
   u_0 (the forward block solve of A u = g, section 2), in one workgroup.
   u (device) [nt+1][n], in: u_0, out: all slices.  Needs nt >= 2 and a
   workspace of atm_sequential_workspace_bytes().  Synchronises the stream.
   Errors: INVALID_ARG, UNSUPPORTED, WORKSPACE, DEVICE, INNER_SOLVE. */
atm_status atm_sequential(const atm_problem* prob, double* u, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for atm_sequential, or 0 if the problem is invalid. */
size_t atm_sequential_workspace_bytes(const atm_problem* prob);

/* Two-level AT-MGRIT (Alg. 1) until ||g - A(u)||_2 <= tol or max_iter cycles.
   u (device) [nt+1][n]: in, u_0 = g_0 and the initial guess at t > 0; out,
   the final iterate.  hist (host, nullable) receives hist_cap residual norms:
   hist[0] of the F-relaxed initial guess, hist[i] after cycle i.  Precision 0
   stops on the C-point residual (atm_residual_norm); precision 1 on the FP64
   implicit residual (atm_implicit_residual_norm, which bounds the paper-form
   residual), reports the paper-form residual of the final iterate in
   stats->final_residual (atm_step_residual_norm), and uses FP64 coarse solves.
   stats (host, nullable).  Synchronises the stream once per cycle.
   Returns OK, NOT_CONVERGED, DIVERGED, INNER_SOLVE, or an argument error. */
atm_status atm_solve(const atm_problem* prob, const atm_options* opts, double* u, void* ws,
                     size_t ws_bytes, double* hist, int32_t hist_cap, atm_stats* stats, void* stream);

/* ------------------------------------------------------------------------
 * Batched solves: many independent instances (ATM_HEAT1D with nx <= 512, 2D
 * kinds up to 128 x 128, plain coarse propagator) advance together, one cycle
 * per replay of a captured hipGraph.  Each phase of a cycle is one launch per
 * instance class (1D heat, 2D heat, 2D Allen-Cahn; concurrent graph branches)
 * over a table of (instance, interval / window) tasks; an autotuner picks the
 * task order (as given or longest first) and the strip tile (one 32-row tile
 * for all 2D instances, or each instance's own) by timing the window phase,
 * and can keep its choice in a cache file.  Every instance runs Alg. 1 as
 * atm_solve does with its own options (precision 1 for the FP32-fine form);
 * an instance stops when its own test is met, its later tasks are skipped.
 * The stopping decision is taken on the device; the host reads the instance
 * states every check_every cycles.
 * ------------------------------------------------------------------------ */
typedef struct atm_batch atm_batch;

/* Workspace bytes for the batch (0 if an instance is invalid or unsupported). */
size_t atm_batch_workspace_bytes(int32_t n, const atm_problem* probs, const atm_options* opts);

/* Plan a batch of n instances: probs[i], opts[i] (host arrays), u[i] (host array of device
   pointers, each [nt_i+1][n_i] FP64 holding u_0 and the initial guess, updated in place by
   atm_batch_run).  ws (device) of atm_batch_workspace_bytes() bytes, 256-byte aligned, owned by
   the caller and used by the plan until atm_batch_destroy.  tune_cache (host path, nullable): a
   text file where the autotuner's choice is read and appended, keyed by the instances' shapes.
   The plan holds HIP streams, events and a graph (host-side objects); it allocates no device
   memory. */
atm_status atm_batch_create(atm_batch** out, int32_t n, const atm_problem* probs, const atm_options* opts,
                            double* const* u, void* ws, size_t ws_bytes, const char* tune_cache);

/* Solve every instance: the initial F-relaxation, the autotuner on the first call, then cycles
   until every instance has stopped.  use_graph 1 replays one captured cycle (captured on the
   first call), 0 enqueues the same launches directly.  status[i], stats[i] (host, nullable; the
   ms_* fields hold the batch's time), hist (host, nullable, [n][hist_cap], up to 256 norms per
   instance) are filled.  ms_solve (host, nullable): wall time without the autotuner; ms_tune
   (host, nullable): the autotuner's time (0 once tuned).  Work is ordered after `stream` and
   `stream` waits for the batch.  Returns OK if every instance converged, NOT_CONVERGED if one
   reached max_iter, else the first error status of an instance. */
atm_status atm_batch_run(atm_batch* b, int32_t use_graph, int32_t check_every, atm_status* status, atm_stats* stats,
                         double* hist, int32_t hist_cap, double* ms_solve, double* ms_tune, void* stream);

/* The autotuner's choice: *order 0 as given / 1 longest task first; *tiles 0 one 32-row strip
   tile / 1 each instance's own.  Returns 1 once tuned. */
int32_t atm_batch_tuning(const atm_batch* b, int32_t* order, int32_t* tiles);

void atm_batch_destroy(atm_batch* b);

/* ------------------------------------------------------------------------
 * Learned coarse propagator (section 2.1 lets the coarse propagator be any
 * approximation of Phi over a coarse step).  Psi(u) = u + f(u), f a four-layer
 * 3x3 convolutional network on the periodic h x w grid: 1 -> 32 -> 32 -> 32 -> 1
 * channels, ReLU after the first three layers, circular padding.  Weights and
 * activations BF16, FP32 accumulation (BF16 MFMA for the 32 -> 32 layers);
 * biases FP32.  Parameters are one FP32 vector of atm_cnn_param_count() entries
 * (device), in this order: W1[9][32] (tap, out channel), b1[32],
 * W2[9][32][32] (tap, out, in), b2[32], W3[9][32][32], b3[32], W4[9][32]
 * (tap, in channel), b4[1]; tap t = (dy + 1) * 3 + (dx + 1) weighs the input at
 * (y + dy, x + dx).  Fields are [batch][h][w] FP32 (device), row-major.
 * All calls enqueue on `stream` and return; results are valid after a sync.
 * Limits: w a multiple of 16 in [16, 128]; h >= 1.  Errors: INVALID_ARG,
 * UNSUPPORTED, WORKSPACE, DEVICE.
 * ------------------------------------------------------------------------ */

/* 19105: the length of the parameter vector. */
int32_t atm_cnn_param_count(void);

/* Workspace bytes for a batch of that many h x w fields (0 if invalid). */
size_t atm_cnn_workspace_bytes(int32_t batch, int32_t h, int32_t w);

/* f_out[b] = f(x[b]) for b < batch (the network output; Psi(x) = x + f(x)). */
atm_status atm_cnn_forward(const float* params, const float* x, int32_t batch, int32_t h, int32_t w,
                           float* f_out, void* ws, size_t ws_bytes, void* stream);

/* out[b] = e[b] + J_f(v[b]) e[b]: the derivative of Psi at v applied to e (the
   ReLU masks of the forward pass at v; no biases). */
atm_status atm_cnn_jvp(const float* params, const float* v, const float* e, int32_t batch, int32_t h,
                       int32_t w, float* out, void* ws, size_t ws_bytes, void* stream);

/* Mean squared error L = mean over the batch of (x + f(x) - y)^2 with
   x = frames[idx_x[b]], y = frames[idx_y[b]] (frames: [n_frames][h][w] FP32,
   device; idx_x, idx_y: host arrays of batch indices in [0, n_frames)), and
   its gradient by back-propagation.  grad_out (device) receives
   atm_cnn_param_count() floats; loss_out (device, nullable) one float. */
atm_status atm_cnn_gradients(const float* params, const float* frames, int32_t n_frames, const int32_t* idx_x,
                             const int32_t* idx_y, int32_t batch, int32_t h, int32_t w, float* grad_out,
                             float* loss_out, void* ws, size_t ws_bytes, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) on
   params (device, in/out) with the moments adam_m, adam_v (device, in/out,
   zero before step 1) and the gradient of the batch above.  loss_out (device,
   nullable) receives the batch loss before the step. */
atm_status atm_cnn_train_step(float* params, float* adam_m, float* adam_v, int32_t step, float lr,
                              const float* frames, int32_t n_frames, const int32_t* idx_x, const int32_t* idx_y,
                              int32_t batch, int32_t h, int32_t w, float* loss_out, void* ws, size_t ws_bytes,
                              void* stream);

/* Human-readable name of a status code (static string). */
const char* atm_status_string(atm_status status);

/* Message of the last error on the calling thread ("" if none). */
const char* atm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ATM_H */
