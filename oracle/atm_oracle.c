/*
 * CPU oracle for two-level AT-MGRIT (Hahne, Southworth, Friedhoff,
 * "Asynchronous Truncated Multigrid-reduction-in-time", arXiv 2107.09596).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 reference that
 * the GPU library is checked against.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark load it.  It shares no code,
 * header, table or helper with the HIP library, and it never calls it.
 *
 * Everything follows the paper's statement in its own order:
 *   - the one-step form u_i = Phi(u_{i-1}) + g_i and the space-time system
 *     A(u) = g (section 2, eq. (2) and the block bidiagonal matrix A);
 *   - the CF-splitting with every m-th point a C-point and the local
 *     truncated coarse grids T^(p) = {i dT : max(0, p-k+1) <= i <= p}
 *     (section 2.1, definition of T^(p); Fig. 1);
 *   - Alg. 1: F-relaxation, residual, restriction by injection to every local
 *     grid, independent local solves with the bidiagonal coarse matrix in Psi
 *     (section 3.1.2, definition of the approximate local matrix), correction
 *     by selective ideal interpolation P_S^(p) (section 3.1, P_S);
 *   - F(CF)^nu relaxation with nu = 1 (section 2.2 and Alg. 2);
 *   - the FAS form of the local problems for a nonlinear Psi (Alg. 2, the
 *     coarsest-level branch);
 *   - stopping on the discrete 2-norm of the absolute space-time residual
 *     (section 4.3);
 *   - the multilevel FAS V-cycle of Alg. 2 (section 2.2): F(CF)^nu relaxation,
 *     injection of the approximation and its residual, the next level's FAS
 *     system, local grids on the coarsest level, ideal interpolation back.
 *
 * Readings taken where the paper is silent:
 *   - g_0 = u_0.  Without a forcing term g_i = 0 for i >= 1.  With a PDE source
 *     b(x, t) (the manufactured 1D heat problem of section 4.3) the backward
 *     Euler step takes it at the new time level, M u_i = psi(u_{i-1}) + dt b(t_i),
 *     so Phi(u_{i-1}) + g_i is that solve and g_i = M^{-1} dt b(t_i); the coarse
 *     propagator Psi acts on corrections (linear form) or on C-point values with
 *     the FAS right-hand side, and takes no source.
 *   - Selective ideal interpolation is applied as "add e_p to C-point p, then
 *     F-relax interval p from it".  For a linear Phi this equals adding
 *     Phi^i e_p to the F-points of an F-relaxed iterate; for a nonlinear Phi
 *     it is the usual FAS interpolation.
 *   - Phi for the 2D problems is one backward-Euler (heat) or IMEX
 *     (Allen-Cahn) step whose linear system (I - dt nu L_h) is solved by
 *     Jacobi-preconditioned CG started from the input state, stopped when the
 *     recursively updated residual satisfies ||r|| <= rtol ||b||.
 *   - Every cycle runs its whole F(CF)^nu relaxation, the leading F-relaxation
 *     included, and every F-relaxation steps every interval from its C-point.
 *   - Psi is coarse_substeps steps of size m dt / coarse_substeps of the same
 *     integrator (a re-discretisation with step dT, section 2.1 end); its CG
 *     tolerance is coarse_cg_rtol when set (Psi only approximates Phi^m, so its
 *     solve accuracy changes the convergence rate, never the fixed point).
 *
 * Status codes: 0 ok, 1 not converged (result valid), -1 invalid argument,
 * -4 diverged (non-finite residual), -5 inner CG did not reach rtol.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_HEAT1D = 1, OR_HEAT2D = 2, OR_AC2D = 3 };
enum { OR_OK = 0, OR_NOT_CONVERGED = 1, OR_INVALID = -1, OR_DIVERGED = -4, OR_INNER = -5 };

typedef struct {
    double length, nu, eps, t0, tf, cg_rtol;
    int64_t nt;
    int32_t kind, nx, ny, cg_max_iter;
    const double* src; /* nullable [nt+1][n]: PDE source b(x, t_i) at every time point (row 0 unused) */
} or_problem;

typedef struct {
    double tol;
    double coarse_cg_rtol; /* CG tolerance inside Psi; 0 means the fine cg_rtol */
    int32_t m, k, relax, max_iter, coarse_substeps, coarse_form;
} or_options;

typedef struct {
    double final_residual;
    int64_t fine_steps, coarse_steps, cg_iters;
    int32_t iterations, status;
} or_stats;

static int g_threads = 1;

void or_set_threads(int t) { g_threads = t < 1 ? 1 : t; }

int or_get_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int64_t nspace(const or_problem* P) { return (int64_t)P->nx * (int64_t)P->ny; }
static double step_size(const or_problem* P) { return (P->tf - P->t0) / (double)P->nt; }

/* grid spacing: Dirichlet problems have nx interior points, h = L/(nx+1);
   the periodic problem has nx points per period, h = L/nx. */
static double spacing(const or_problem* P, int32_t npts)
{
    return P->kind == OR_AC2D ? P->length / (double)npts : P->length / (double)(npts + 1);
}

/* ------------------------------------------------------------------------ */
/* the spatial operator M = I - dt nu L_h (five-point Laplacian in 2D)       */
/* ------------------------------------------------------------------------ */

static void apply_M2d(const or_problem* P, double cx, double cy, const double* x, double* y)
{
    const int nx = P->nx, ny = P->ny;
    const int periodic = (P->kind == OR_AC2D);
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            double w, e, s, n;
            if (periodic) {
                w = x[j * nx + (i + nx - 1) % nx];
                e = x[j * nx + (i + 1) % nx];
                s = x[((j + ny - 1) % ny) * nx + i];
                n = x[((j + 1) % ny) * nx + i];
            } else {
                w = i > 0 ? x[j * nx + i - 1] : 0.0;
                e = i < nx - 1 ? x[j * nx + i + 1] : 0.0;
                s = j > 0 ? x[(j - 1) * nx + i] : 0.0;
                n = j < ny - 1 ? x[(j + 1) * nx + i] : 0.0;
            }
            y[j * nx + i] = (1.0 + 2.0 * cx + 2.0 * cy) * x[j * nx + i] - cx * (w + e) - cy * (s + n);
        }
    }
}

static double dot(int64_t n, const double* a, const double* b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Jacobi-preconditioned conjugate gradients for M x = b, started from x.
   work holds 4n doubles.  Returns 0, or OR_INNER when rtol is not reached
   within cg_max_iter iterations. */
static int pcg2d(const or_problem* P, double cx, double cy, double rtol, const double* b, double* x,
                 double* work, int64_t* its)
{
    const int64_t n = nspace(P);
    double* r = work;
    double* z = work + n;
    double* p = work + 2 * n;
    double* q = work + 3 * n;
    const double diag = 1.0 + 2.0 * cx + 2.0 * cy;
    const double bb = dot(n, b, b);
    if (bb == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        return OR_OK;
    }
    apply_M2d(P, cx, cy, x, q);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    for (int64_t i = 0; i < n; ++i) z[i] = r[i] / diag;
    for (int64_t i = 0; i < n; ++i) p[i] = z[i];
    double rz = dot(n, r, z);
    double rr = dot(n, r, r);
    const double thresh = rtol * rtol * bb;
    int it = 0;
    while (rr > thresh) {
        if (it >= P->cg_max_iter) return OR_INNER;
        apply_M2d(P, cx, cy, p, q);
        const double alpha = rz / dot(n, p, q);
        for (int64_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int64_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        for (int64_t i = 0; i < n; ++i) z[i] = r[i] / diag;
        const double rz_new = dot(n, r, z);
        const double beta = rz_new / rz;
        rz = rz_new;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rr = dot(n, r, r);
        ++it;
    }
    if (its) *its += it;
    return OR_OK;
}

/* Thomas algorithm for the constant tridiagonal system (1+2c) x_i - c x_{i-1} - c x_{i+1} = b_i
   with zero Dirichlet ends.  work holds 2n doubles. */
static void thomas(int n, double c, const double* b, double* x, double* work)
{
    double* cp = work;
    double* dp = work + n;
    const double diag = 1.0 + 2.0 * c;
    const double off = -c;
    cp[0] = off / diag;
    dp[0] = b[0] / diag;
    for (int i = 1; i < n; ++i) {
        const double den = diag - off * cp[i - 1];
        cp[i] = off / den;
        dp[i] = (b[i] - off * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
}

/* The right-hand side of the step's linear system M u_i = psi(u_{i-1}):
   psi is the identity for heat; for Allen-Cahn the reaction term is taken
   explicitly, psi(v) = v + dt (v - v^3) / eps^2 (IMEX). */
static void explicit_part(const or_problem* P, double dt, const double* in, double* b)
{
    const int64_t n = nspace(P);
    if (P->kind != OR_AC2D) {
        for (int64_t i = 0; i < n; ++i) b[i] = in[i];
    } else {
        const double s = dt / (P->eps * P->eps);
        for (int64_t i = 0; i < n; ++i) b[i] = in[i] + s * (in[i] - in[i] * in[i] * in[i]);
    }
}

/* y = M x for the fine step, M = I - dt nu L_h (1D: the tridiagonal matrix of thomas()) */
static void apply_M_fine(const or_problem* P, const double* x, double* y)
{
    const double dt = step_size(P);
    const double hx = spacing(P, P->nx);
    const double cx = P->nu * dt / (hx * hx);
    if (P->kind == OR_HEAT1D) {
        const int nx = P->nx;
        for (int i = 0; i < nx; ++i) {
            const double w = i > 0 ? x[i - 1] : 0.0;
            const double e = i < nx - 1 ? x[i + 1] : 0.0;
            y[i] = (1.0 + 2.0 * cx) * x[i] - cx * (w + e);
        }
        return;
    }
    const double hy = spacing(P, P->ny);
    apply_M2d(P, cx, P->nu * dt / (hy * hy), x, y);
}

/* One step of the integrator with step size dt: out solves
   M out = psi(in) + dt f, with f the source at the step's new time level
   (NULL: no source), the linear systems of the 2D kinds solved to relative
   tolerance rtol.  work must hold 6n doubles.  out may not alias in. */
static int step_dt_tol(const or_problem* P, double dt, double rtol, const double* in, const double* f,
                       double* out, double* work, int64_t* cg_its);

static int step_dt(const or_problem* P, double dt, const double* in, const double* f, double* out,
                   double* work, int64_t* cg_its)
{
    return step_dt_tol(P, dt, P->cg_rtol, in, f, out, work, cg_its);
}

static int step_dt_tol(const or_problem* P, double dt, double rtol, const double* in, const double* f,
                       double* out, double* work, int64_t* cg_its)
{
    const int64_t n = nspace(P);
    double* b = work + 4 * n;
    explicit_part(P, dt, in, b);
    if (f)
        for (int64_t i = 0; i < n; ++i) b[i] += dt * f[i];
    if (P->kind == OR_HEAT1D) {
        const double h = spacing(P, P->nx);
        thomas(P->nx, P->nu * dt / (h * h), b, out, work);
        return OR_OK;
    }
    const double hx = spacing(P, P->nx), hy = spacing(P, P->ny);
    const double cx = P->nu * dt / (hx * hx), cy = P->nu * dt / (hy * hy);
    for (int64_t i = 0; i < n; ++i) out[i] = in[i];
    return pcg2d(P, cx, cy, rtol, b, out, work, cg_its);
}

static int64_t work_len(const or_problem* P) { return 6 * nspace(P); }

/* Phi(in) + g_i: the fine step of size dt that produces time point i (eq. (2)),
   with the source at t_i when the problem has one. */
static int fine_step(const or_problem* P, int64_t i, const double* in, double* out, double* work,
                     int64_t* cg)
{
    return step_dt(P, step_size(P), in, P->src ? P->src + i * nspace(P) : NULL, out, work, cg);
}

/* Psi: the coarse propagator, a re-discretisation with dT = m dt taken in s substeps. */
static int coarse_step(const or_problem* P, const or_options* O, const double* in, double* out,
                       double* work, int64_t* cg)
{
    const int64_t n = nspace(P);
    const int s = O->coarse_substeps < 1 ? 1 : O->coarse_substeps;
    const double dts = step_size(P) * (double)O->m / (double)s;
    const double rtol = O->coarse_cg_rtol > 0.0 ? O->coarse_cg_rtol : P->cg_rtol;
    double* tmp = work + work_len(P);
    const double* src = in;
    for (int i = 0; i < s; ++i) {
        double* dst = (i == s - 1) ? out : tmp + (i & 1) * n;
        int st = step_dt_tol(P, dts, rtol, src, NULL, dst, work, cg);
        if (st) return st;
        src = dst;
    }
    return OR_OK;
}

static int64_t coarse_work_len(const or_problem* P) { return work_len(P) + 2 * nspace(P); }

/* ------------------------------------------------------------------------ */
/* exported single steps                                                     */
/* ------------------------------------------------------------------------ */

/* one step of size dt without source */
int or_step(const or_problem* P, double dt, const double* in, double* out, int64_t* cg_its)
{
    double* work = malloc(sizeof(double) * work_len(P));
    int st = step_dt(P, dt, in, NULL, out, work, cg_its);
    free(work);
    return st;
}

int or_coarse_step(const or_problem* P, const or_options* O, const double* in, double* out, int64_t* cg)
{
    double* work = malloc(sizeof(double) * coarse_work_len(P));
    int st = coarse_step(P, O, in, out, work, cg);
    free(work);
    return st;
}

/* Sequential time stepping: the forward block solve of A u = g (section 2). */
int or_sequential(const or_problem* P, double* u, int64_t* cg_its)
{
    const int64_t n = nspace(P);
    double* work = malloc(sizeof(double) * work_len(P));
    int st = OR_OK;
    for (int64_t i = 1; i <= P->nt && st == OR_OK; ++i)
        st = fine_step(P, i, u + (i - 1) * n, u + i * n, work, cg_its);
    free(work);
    return st;
}

/* ------------------------------------------------------------------------ */
/* the time grid (section 2.1)                                               */
/* ------------------------------------------------------------------------ */

/* number of coarse intervals N_T; C-points are 0..N_T (C-point j is time index j m). */
int64_t or_num_intervals(const or_problem* P, const or_options* O) { return P->nt / O->m; }

/* first C-point index of the local coarse grid T^(p): max(0, p - k + 1) */
int64_t or_window_start(int64_t p, int32_t k) { return p - k + 1 > 0 ? p - k + 1 : 0; }

/* last time index of the F-points following C-point j (an interval may be a ragged tail) */
static int64_t interval_end(const or_problem* P, const or_options* O, int64_t j)
{
    const int64_t e = (j + 1) * O->m - 1;
    return e < P->nt ? e : P->nt;
}

/* ------------------------------------------------------------------------ */
/* relaxation (section 2.1; F(CF)^nu, section 2.2)                           */
/* ------------------------------------------------------------------------ */

/* F-relaxation of one interval: u_{jm+i} = Phi(u_{jm+i-1}) for its F-points, in
   order.  work: work_len doubles. */
static int f_relax_interval(const or_problem* P, const or_options* O, double* u, int64_t j, double* work,
                            int64_t* cg)
{
    const int64_t n = nspace(P);
    int st = OR_OK;
    for (int64_t i = j * O->m + 1; i <= interval_end(P, O, j) && st == OR_OK; ++i)
        st = fine_step(P, i, u + (i - 1) * n, u + i * n, work, cg);
    return st;
}

static int64_t n_relax_intervals(const or_problem* P, const or_options* O)
{
    /* full intervals 0..N_T-1, plus the tail after C-point N_T when m does not divide nt */
    const int64_t NT = or_num_intervals(P, O);
    return (NT * O->m < P->nt) ? NT + 1 : NT;
}

/* F-relaxation of every interval (the intervals are independent) */
int or_f_relax(const or_problem* P, const or_options* O, double* u, int64_t* cg)
{
    const int64_t NI = n_relax_intervals(P, O);
    int status = OR_OK;
    int64_t cg_total = 0;
#pragma omp parallel num_threads(g_threads) reduction(+ : cg_total)
    {
        double* work = malloc(sizeof(double) * work_len(P));
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < NI; ++j) {
            int64_t c = 0;
            int st = f_relax_interval(P, O, u, j, work, &c);
            cg_total += c;
            if (st) {
#pragma omp critical
                status = st;
            }
        }
        free(work);
    }
    if (cg) *cg += cg_total;
    return status;
}

/* C-relaxation: u_{jm} = Phi(u_{jm-1}) for every C-point j >= 1. */
int or_c_relax(const or_problem* P, const or_options* O, double* u, int64_t* cg)
{
    const int64_t n = nspace(P);
    const int64_t NT = or_num_intervals(P, O);
    int status = OR_OK;
    int64_t cg_total = 0;
#pragma omp parallel num_threads(g_threads) reduction(+ : cg_total)
    {
        double* work = malloc(sizeof(double) * work_len(P));
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 1; j <= NT; ++j) {
            int64_t c = 0;
            int st = fine_step(P, j * O->m, u + (j * O->m - 1) * n, u + j * O->m * n, work, &c);
            cg_total += c;
            if (st) {
#pragma omp critical
                status = st;
            }
        }
        free(work);
    }
    if (cg) *cg += cg_total;
    return status;
}

/* ------------------------------------------------------------------------ */
/* residual r = g - A(u) (Alg. 1, "compute residual")                        */
/* ------------------------------------------------------------------------ */

/* Full space-time residual at all nt+1 time points: r_0 = g_0 - u_0,
   r_i = g_i + Phi(u_{i-1}) - u_i (g_i = 0 for i >= 1 without a source). */
int or_residual(const or_problem* P, const double* u, const double* g0, double* r, int64_t* cg)
{
    const int64_t n = nspace(P);
    for (int64_t x = 0; x < n; ++x) r[x] = g0[x] - u[x];
    int status = OR_OK;
    int64_t cg_total = 0;
#pragma omp parallel num_threads(g_threads) reduction(+ : cg_total)
    {
        double* work = malloc(sizeof(double) * work_len(P));
        double* phi = malloc(sizeof(double) * n);
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 1; i <= P->nt; ++i) {
            int64_t c = 0;
            int st = fine_step(P, i, u + (i - 1) * n, phi, work, &c);
            cg_total += c;
            if (st) {
#pragma omp critical
                status = st;
            }
            for (int64_t x = 0; x < n; ++x) r[i * n + x] = phi[x] - u[i * n + x];
        }
        free(phi);
        free(work);
    }
    if (cg) *cg += cg_total;
    return status;
}

double or_norm2(int64_t len, const double* v) { return sqrt(dot(len, v, v)); }

/* The implicit form of the residual.  Every fine step solves M u_i = psi(u_{i-1})
   (eq. (2) for the integrators above), so the paper's residual at a point,
   r_i = Phi(u_{i-1}) + g_i - u_i, equals M^{-1} rho_i with
       rho_i = psi(u_{i-1}) + dt b(t_i) - M u_i   (i = 1..nt; rho_0 = 0 as g_0 - u_0 = 0),
   the source term present only when the problem has one.
   rho needs no solve.  M = I - dt nu L_h has eigenvalues >= 1, so |r_i| <= |rho_i|. */
int or_implicit_residual(const or_problem* P, const double* u, double* rho)
{
    const int64_t n = nspace(P);
    const double dt = step_size(P);
    for (int64_t x = 0; x < n; ++x) rho[x] = 0.0;
#pragma omp parallel num_threads(g_threads)
    {
        double* mu = malloc(sizeof(double) * n);
        double* ps = malloc(sizeof(double) * n);
#pragma omp for schedule(static)
        for (int64_t i = 1; i <= P->nt; ++i) {
            explicit_part(P, dt, u + (i - 1) * n, ps);
            if (P->src)
                for (int64_t x = 0; x < n; ++x) ps[x] += dt * P->src[i * n + x];
            apply_M_fine(P, u + i * n, mu);
            for (int64_t x = 0; x < n; ++x) rho[i * n + x] = ps[x] - mu[x];
        }
        free(ps);
        free(mu);
    }
    return OR_OK;
}

/* r_i = M^{-1} rho_i for i = 1..nt (r_0 = 0): the paper's residual with the
   step's linear system solved by CG from zero to cg_rtol relative to |rho_i|
   (2D) or exactly by the Thomas algorithm (1D).  Unlike Phi(u_{i-1}) - u_i it
   keeps its relative accuracy when the residual is tiny. */
int or_step_residual(const or_problem* P, const double* u, double* r, int64_t* cg)
{
    const int64_t n = nspace(P);
    int st = or_implicit_residual(P, u, r);
    if (st) return st;
    const double dt = step_size(P);
    int status = OR_OK;
    int64_t cg_total = 0;
#pragma omp parallel num_threads(g_threads) reduction(+ : cg_total)
    {
        double* work = malloc(sizeof(double) * work_len(P));
        double* z = malloc(sizeof(double) * n);
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 1; i <= P->nt; ++i) {
            double* ri = r + i * n;
            if (P->kind == OR_HEAT1D) {
                const double h = spacing(P, P->nx);
                thomas(P->nx, P->nu * dt / (h * h), ri, z, work);
            } else {
                const double hx = spacing(P, P->nx), hy = spacing(P, P->ny);
                int64_t c = 0;
                for (int64_t x = 0; x < n; ++x) z[x] = 0.0;
                int s2 = pcg2d(P, P->nu * dt / (hx * hx), P->nu * dt / (hy * hy), P->cg_rtol, ri, z, work, &c);
                cg_total += c;
                if (s2) {
#pragma omp critical
                    status = s2;
                }
            }
            for (int64_t x = 0; x < n; ++x) ri[x] = z[x];
        }
        free(z);
        free(work);
    }
    if (cg) *cg += cg_total;
    return status;
}

/* ------------------------------------------------------------------------ */
/* local coarse-grid solves (Alg. 1; approximate local matrix of 3.1.2)      */
/* ------------------------------------------------------------------------ */

static int use_fas(const or_problem* P, const or_options* O)
{
    if (O->coarse_form == 1) return 0;
    if (O->coarse_form == 2) return 1;
    return P->kind == OR_AC2D;
}

/* Solve the local problem on T^(p) and return its last point e_p.
   rc: C-point residuals r_c = R_I r, [N_T+1][n].  vc: C-point values of the
   current iterate, [N_T+1][n] (read by the FAS form only).
   Linear form: the bidiagonal system with I on the diagonal and -Psi below,
   solved forward: e_s = r_s, e_j = Psi(e_{j-1}) + r_j.
   FAS form: A_c(w) = A_c(v) + r_c, i.e. w_s = v_s + r_s,
   w_j = Psi(w_{j-1}) + (v_j - Psi(v_{j-1}) + r_j); e_p = w_p - v_p. */
static int local_solve(const or_problem* P, const or_options* O, int64_t p, const double* rc,
                       const double* vc, double* e, double* work, int64_t* cg, int64_t* nsteps)
{
    const int64_t n = nspace(P);
    const int64_t s = or_window_start(p, O->k);
    double* w = work + coarse_work_len(P);
    double* psi = w + n;
    double* psiv = psi + n;
    int st;
    if (!use_fas(P, O)) {
        for (int64_t x = 0; x < n; ++x) w[x] = rc[s * n + x];
        for (int64_t j = s + 1; j <= p; ++j) {
            if ((st = coarse_step(P, O, w, psi, work, cg))) return st;
            ++*nsteps;
            for (int64_t x = 0; x < n; ++x) w[x] = psi[x] + rc[j * n + x];
        }
        for (int64_t x = 0; x < n; ++x) e[x] = w[x];
    } else {
        for (int64_t x = 0; x < n; ++x) w[x] = vc[s * n + x] + rc[s * n + x];
        for (int64_t j = s + 1; j <= p; ++j) {
            if ((st = coarse_step(P, O, vc + (j - 1) * n, psiv, work, cg))) return st;
            if ((st = coarse_step(P, O, w, psi, work, cg))) return st;
            *nsteps += 2;
            for (int64_t x = 0; x < n; ++x) {
                const double tau = (vc[j * n + x] - psiv[x]) + rc[j * n + x];
                w[x] = psi[x] + tau;
            }
        }
        for (int64_t x = 0; x < n; ++x) e[x] = w[x] - vc[p * n + x];
    }
    return OR_OK;
}

static int64_t local_work_len(const or_problem* P) { return coarse_work_len(P) + 3 * nspace(P); }

int or_local_solve(const or_problem* P, const or_options* O, int64_t p, const double* rc,
                   const double* vc, double* e, int64_t* cg)
{
    double* work = malloc(sizeof(double) * local_work_len(P));
    int64_t ns = 0;
    int st = local_solve(P, O, p, rc, vc, e, work, cg, &ns);
    free(work);
    return st;
}

/* all windows p = 0..N_T, each from the same (pre-correction) residual */
int or_local_solves(const or_problem* P, const or_options* O, const double* rc, const double* vc,
                    double* e, int64_t* cg, int64_t* coarse_steps)
{
    const int64_t n = nspace(P);
    const int64_t NT = or_num_intervals(P, O);
    int status = OR_OK;
    int64_t cg_total = 0, ns_total = 0;
#pragma omp parallel num_threads(g_threads) reduction(+ : cg_total, ns_total)
    {
        double* work = malloc(sizeof(double) * local_work_len(P));
#pragma omp for schedule(dynamic, 1)
        for (int64_t p = 0; p <= NT; ++p) {
            int64_t c = 0, ns = 0;
            int st = local_solve(P, O, p, rc, vc, e + p * n, work, &c, &ns);
            cg_total += c;
            ns_total += ns;
            if (st) {
#pragma omp critical
                status = st;
            }
        }
        free(work);
    }
    if (cg) *cg += cg_total;
    if (coarse_steps) *coarse_steps += ns_total;
    return status;
}

/* Correction u = u + P_S^(p) e_p for every p: add e_p to C-point p, then
   F-relax the interval that follows it (selective ideal interpolation). */
int or_correct(const or_problem* P, const or_options* O, double* u, const double* e, int64_t* cg)
{
    const int64_t n = nspace(P);
    const int64_t NT = or_num_intervals(P, O);
    for (int64_t p = 0; p <= NT; ++p)
        for (int64_t x = 0; x < n; ++x) u[p * O->m * n + x] += e[p * n + x];
    return or_f_relax(P, O, u, cg);
}

/* C-point injection R_I of a space-time vector: out_j = v_{jm}. */
static void inject(const or_problem* P, const or_options* O, const double* v, double* out)
{
    const int64_t n = nspace(P);
    const int64_t NT = or_num_intervals(P, O);
    for (int64_t j = 0; j <= NT; ++j) memcpy(out + j * n, v + j * O->m * n, sizeof(double) * n);
}

/* ------------------------------------------------------------------------ */
/* one cycle and the solve loop (Alg. 1)                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *r, *rc, *vc, *e;
} buffers;

static int alloc_buffers(const or_problem* P, const or_options* O, buffers* B)
{
    const int64_t n = nspace(P);
    const int64_t NT = or_num_intervals(P, O);
    B->r = malloc(sizeof(double) * (P->nt + 1) * n);
    B->rc = malloc(sizeof(double) * (NT + 1) * n);
    B->vc = malloc(sizeof(double) * (NT + 1) * n);
    B->e = malloc(sizeof(double) * (NT + 1) * n);
    return (B->r && B->rc && B->vc && B->e) ? OR_OK : OR_INVALID;
}

static void free_buffers(buffers* B)
{
    free(B->r);
    free(B->rc);
    free(B->vc);
    free(B->e);
}

/* F(CF)^nu relaxation (nu = relax: 0 or 1) */
static int relax(const or_problem* P, const or_options* O, double* u, or_stats* S)
{
    const int64_t NT = or_num_intervals(P, O);
    int st = or_f_relax(P, O, u, &S->cg_iters);
    S->fine_steps += P->nt - NT;
    if (st || O->relax == 0) return st;
    st = or_c_relax(P, O, u, &S->cg_iters);
    S->fine_steps += NT;
    if (st) return st;
    st = or_f_relax(P, O, u, &S->cg_iters);
    S->fine_steps += P->nt - NT;
    return st;
}

/* One AT-MGRIT cycle in Alg. 1's order, with a coarse solve that is either the
   local windows (global = 0) or one global sequential coarse grid (global = 1,
   the Parareal / two-level MGRIT cycle, written separately below). */
static int global_coarse_solve(const or_problem* P, const or_options* O, const double* rc,
                               const double* vc, double* e, or_stats* S);

static int cycle(const or_problem* P, const or_options* O, double* u, const double* g0, buffers* B,
                 or_stats* S, int global)
{
    int st = relax(P, O, u, S);
    if (st) return st;
    if ((st = or_residual(P, u, g0, B->r, &S->cg_iters))) return st;
    S->fine_steps += P->nt;
    inject(P, O, B->r, B->rc);
    inject(P, O, u, B->vc);
    if (global)
        st = global_coarse_solve(P, O, B->rc, B->vc, B->e, S);
    else
        st = or_local_solves(P, O, B->rc, B->vc, B->e, &S->cg_iters, &S->coarse_steps);
    if (st) return st;
    st = or_correct(P, O, u, B->e, &S->cg_iters);
    S->fine_steps += P->nt - or_num_intervals(P, O);
    return st;
}

int or_cycle(const or_problem* P, const or_options* O, double* u, const double* g0, or_stats* S)
{
    buffers B;
    if (alloc_buffers(P, O, &B)) return OR_INVALID;
    int st = cycle(P, O, u, g0, &B, S, 0);
    free_buffers(&B);
    return st;
}

/* Residual norm of the current iterate after F-relaxation, as Alg. 1 checks it. */
static int residual_norm(const or_problem* P, const or_options* O, double* u, const double* g0,
                         buffers* B, or_stats* S, double* out)
{
    int st = or_residual(P, u, g0, B->r, &S->cg_iters);
    S->fine_steps += P->nt;
    if (st) return st;
    *out = or_norm2((P->nt + 1) * nspace(P), B->r);
    (void)O;
    return OR_OK;
}

static int solve(const or_problem* P, const or_options* O, double* u, double* hist, int32_t hist_cap,
                 or_stats* S, int global)
{
    const int64_t n = nspace(P);
    memset(S, 0, sizeof(*S));
    if (P->nt < 1 || O->m < 2 || O->k < 1 || P->nx < 1 || P->ny < 1) return S->status = OR_INVALID;
    double* g0 = malloc(sizeof(double) * n);
    memcpy(g0, u, sizeof(double) * n);
    buffers B;
    if (alloc_buffers(P, O, &B)) {
        free(g0);
        return S->status = OR_INVALID;
    }
    /* the initial guess is F-relaxed first (the start of every cycle), so the
       history starts from the residual of the F-relaxed guess */
    int st = or_f_relax(P, O, u, &S->cg_iters);
    S->fine_steps += P->nt - or_num_intervals(P, O);
    double res = 0.0;
    if (!st) st = residual_norm(P, O, u, g0, &B, S, &res);
    if (!st && hist && hist_cap > 0) hist[0] = res;
    int it = 0;
    while (!st && !(res <= O->tol)) {
        if (!isfinite(res)) {
            st = OR_DIVERGED;
            break;
        }
        if (it >= O->max_iter) {
            st = OR_NOT_CONVERGED;
            break;
        }
        st = cycle(P, O, u, g0, &B, S, global);
        if (st) break;
        ++it;
        st = residual_norm(P, O, u, g0, &B, S, &res);
        if (!st && hist && it < hist_cap) hist[it] = res;
    }
    if (!st && !isfinite(res)) st = OR_DIVERGED;
    S->iterations = it;
    S->final_residual = res;
    S->status = st;
    free_buffers(&B);
    free(g0);
    return st;
}

/* Two-level AT-MGRIT (Alg. 1) until ||g - A(u)||_2 <= tol. u[0] holds g_0 and
   u[1..nt] the initial guess; on return u holds the final iterate and
   hist[0..iterations] the residual norms (hist[0]: F-relaxed initial guess). */
int or_atmgrit_solve(const or_problem* P, const or_options* O, double* u, double* hist,
                     int32_t hist_cap, or_stats* S)
{
    return solve(P, O, u, hist, hist_cap, S, 0);
}

/* ------------------------------------------------------------------------ */
/* plain two-level MGRIT / Parareal: one global sequential coarse grid       */
/* (section 1 and 2.1; AT-MGRIT with k = N_T + 1 is the same method)         */
/* ------------------------------------------------------------------------ */

static int global_coarse_solve(const or_problem* P, const or_options* O, const double* rc,
                               const double* vc, double* e, or_stats* S)
{
    const int64_t n = nspace(P);
    const int64_t NT = or_num_intervals(P, O);
    double* work = malloc(sizeof(double) * (coarse_work_len(P) + 3 * n));
    double* psi = work + coarse_work_len(P);
    double* psiv = psi + n;
    double* w = psiv + n;
    int st = OR_OK;
    if (!use_fas(P, O)) {
        /* forward substitution with the global coarse matrix (I on the diagonal, -Psi below) */
        memcpy(e, rc, sizeof(double) * n);
        for (int64_t j = 1; j <= NT && !st; ++j) {
            st = coarse_step(P, O, e + (j - 1) * n, psi, work, &S->cg_iters);
            S->coarse_steps += 1;
            for (int64_t x = 0; x < n; ++x) e[j * n + x] = psi[x] + rc[j * n + x];
        }
    } else {
        /* FAS coarse problem A_c(w) = A_c(v) + r_c, solved forward; e = w - v */
        for (int64_t x = 0; x < n; ++x) w[x] = vc[x] + rc[x];
        for (int64_t x = 0; x < n; ++x) e[x] = w[x] - vc[x];
        for (int64_t j = 1; j <= NT && !st; ++j) {
            st = coarse_step(P, O, vc + (j - 1) * n, psiv, work, &S->cg_iters);
            if (!st) st = coarse_step(P, O, w, psi, work, &S->cg_iters);
            S->coarse_steps += 2;
            for (int64_t x = 0; x < n; ++x) {
                const double tau = (vc[j * n + x] - psiv[x]) + rc[j * n + x];
                w[x] = psi[x] + tau;
                e[j * n + x] = w[x] - vc[j * n + x];
            }
        }
    }
    free(work);
    return st;
}

int or_parareal_solve(const or_problem* P, const or_options* O, double* u, double* hist,
                      int32_t hist_cap, or_stats* S)
{
    return solve(P, O, u, hist, hist_cap, S, 1);
}

int or_parareal_cycle(const or_problem* P, const or_options* O, double* u, const double* g0, or_stats* S)
{
    buffers B;
    if (alloc_buffers(P, O, &B)) return OR_INVALID;
    int st = cycle(P, O, u, g0, &B, S, 1);
    free_buffers(&B);
    return st;
}

/* ------------------------------------------------------------------------ */
/* multilevel FAS AT-MGRIT V-cycle (section 2.2, Alg. 2)                     */
/* ------------------------------------------------------------------------ */

#define OR_MAX_LEVELS 4

/* Levels l = 0..L-1: level 0 is the fine grid; level l+1 takes every m[l]-th point of level l
   (restriction by injection); the coarsest level L-1 is replaced by the local grids of size k.
   Level l >= 1 steps with a re-discretisation of step dt m[0]..m[l-1], taken in coarse_substeps
   substeps whose linear systems are solved to coarse_cg_rtol (0: the problem's cg_rtol). */
typedef struct {
    double tol;
    double coarse_cg_rtol;
    int32_t levels;
    int32_t m[OR_MAX_LEVELS - 1];
    int32_t k, relax, max_iter, coarse_substeps;
    int32_t nested; /* 1: start from the nested-iteration guess (or_ml_nested) */
} or_ml_options;

typedef struct {
    int64_t nt; /* steps of this level: time points 0..nt */
    double dt;
    int32_t m;  /* coarsening factor to the next level (unused on the coarsest) */
    int32_t substeps;
    double rtol;
    int32_t fine; /* level 0: the fine integrator (with the problem's source, if any) */
} ml_level;

static int ml_levels(const or_problem* P, const or_ml_options* O, ml_level* lv)
{
    if (O->levels < 2 || O->levels > OR_MAX_LEVELS || O->k < 1) return OR_INVALID;
    int64_t nt = P->nt;
    double dt = step_size(P);
    for (int l = 0; l < O->levels; ++l) {
        lv[l].nt = nt;
        lv[l].dt = dt;
        lv[l].fine = (l == 0);
        lv[l].substeps = (l == 0) ? 1 : (O->coarse_substeps < 1 ? 1 : O->coarse_substeps);
        lv[l].rtol = (l == 0 || O->coarse_cg_rtol <= 0.0) ? P->cg_rtol : O->coarse_cg_rtol;
        lv[l].m = (l < O->levels - 1) ? O->m[l] : 0;
        if (l < O->levels - 1) {
            if (lv[l].m < 2 || nt < lv[l].m) return OR_INVALID;
            nt /= lv[l].m;
            dt *= lv[l].m;
        }
    }
    return OR_OK;
}

/* the integrator of level l producing point i from in (work: coarse_work_len doubles) */
static int ml_step(const or_problem* P, const ml_level* L, int64_t i, const double* in, double* out, double* work,
                   int64_t* cg)
{
    if (L->fine) return fine_step(P, i, in, out, work, cg);
    const int64_t n = nspace(P);
    double* tmp = work + work_len(P);
    const double* src = in;
    for (int q = 0; q < L->substeps; ++q) {
        double* dst = (q == L->substeps - 1) ? out : tmp + (q & 1) * n;
        int st = step_dt_tol(P, L->dt / L->substeps, L->rtol, src, NULL, dst, work, cg);
        if (st) return st;
        src = dst;
    }
    return OR_OK;
}

/* right-hand side of point i >= 1 of the level's system u_i - Phi_l(u_{i-1}) = G_i (0 without G) */
static double ml_rhs(const double* G, int64_t n, int64_t i, int64_t x) { return G ? G[i * n + x] : 0.0; }

/* u_i = Phi_l(u_{i-1}) + G_i for the F-points of every interval (F-relaxation of level l) */
static int ml_f_relax(const or_problem* P, const ml_level* L, double* u, const double* G, int64_t* cg)
{
    const int64_t n = nspace(P);
    const int64_t NC = L->nt / L->m;
    const int64_t NI = (NC * L->m < L->nt) ? NC + 1 : NC;
    int status = OR_OK;
    int64_t cg_total = 0;
#pragma omp parallel num_threads(g_threads) reduction(+ : cg_total)
    {
        double* work = malloc(sizeof(double) * coarse_work_len(P));
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < NI; ++j) {
            int64_t end = (j + 1) * L->m - 1;
            if (end > L->nt) end = L->nt;
            int st = OR_OK;
            int64_t c = 0;
            for (int64_t i = j * L->m + 1; i <= end && st == OR_OK; ++i) {
                st = ml_step(P, L, i, u + (i - 1) * n, u + i * n, work, &c);
                for (int64_t x = 0; x < n; ++x) u[i * n + x] += ml_rhs(G, n, i, x);
            }
            cg_total += c;
            if (st) {
#pragma omp critical
                status = st;
            }
        }
        free(work);
    }
    if (cg) *cg += cg_total;
    return status;
}

/* u_{jm} = Phi_l(u_{jm-1}) + G_{jm} for every C-point j >= 1 (C-relaxation of level l) */
static int ml_c_relax(const or_problem* P, const ml_level* L, double* u, const double* G, int64_t* cg)
{
    const int64_t n = nspace(P);
    const int64_t NC = L->nt / L->m;
    int status = OR_OK;
    int64_t cg_total = 0;
#pragma omp parallel num_threads(g_threads) reduction(+ : cg_total)
    {
        double* work = malloc(sizeof(double) * coarse_work_len(P));
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 1; j <= NC; ++j) {
            const int64_t i = j * L->m;
            int64_t c = 0;
            int st = ml_step(P, L, i, u + (i - 1) * n, u + i * n, work, &c);
            for (int64_t x = 0; x < n; ++x) u[i * n + x] += ml_rhs(G, n, i, x);
            cg_total += c;
            if (st) {
#pragma omp critical
                status = st;
            }
        }
        free(work);
    }
    if (cg) *cg += cg_total;
    return status;
}

/* residual of level l's system injected to its C-points: rc_j = G_{jm} + Phi_l(u_{jm-1}) - u_{jm}
   (j >= 1), rc_0 = G_0 - u_0 with G_0 = g0 on level 0 */
static int ml_c_residual(const or_problem* P, const ml_level* L, const double* u, const double* G,
                         const double* g0, double* rc, int64_t* cg)
{
    const int64_t n = nspace(P);
    const int64_t NC = L->nt / L->m;
    for (int64_t x = 0; x < n; ++x) rc[x] = (G ? G[x] : g0[x]) - u[x];
    int status = OR_OK;
    int64_t cg_total = 0;
#pragma omp parallel num_threads(g_threads) reduction(+ : cg_total)
    {
        double* work = malloc(sizeof(double) * coarse_work_len(P));
        double* phi = malloc(sizeof(double) * n);
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 1; j <= NC; ++j) {
            const int64_t i = j * L->m;
            int64_t c = 0;
            int st = ml_step(P, L, i, u + (i - 1) * n, phi, work, &c);
            for (int64_t x = 0; x < n; ++x) rc[j * n + x] = (ml_rhs(G, n, i, x) + phi[x]) - u[i * n + x];
            cg_total += c;
            if (st) {
#pragma omp critical
                status = st;
            }
        }
        free(phi);
        free(work);
    }
    if (cg) *cg += cg_total;
    return status;
}

/* The coarsest level: for every point p its local grid T^(l,p) = {max(0, p-k+1)..p} gets
   v^(l,p) = R_I^(l,p) v and g^(l,p) = R_I^(l,p) g; the local problem
   A^(l,p)(w) = A^(l,p)(v^(l,p)) + g^(l,p), with the identity on the grid's first point and
   -Phi_l below the diagonal, is solved forward, and u_p = w_p (injection P_I^(l,p)). */
static int ml_local_solves(const or_problem* P, const ml_level* L, int32_t k, const double* v, const double* g,
                           double* u, int64_t* cg)
{
    const int64_t n = nspace(P);
    const int64_t N = L->nt;
    int status = OR_OK;
    int64_t cg_total = 0;
#pragma omp parallel num_threads(g_threads) reduction(+ : cg_total)
    {
        double* work = malloc(sizeof(double) * (coarse_work_len(P) + 3 * n));
        double* w = work + coarse_work_len(P);
        double* pw = w + n;
        double* pv = pw + n;
#pragma omp for schedule(dynamic, 1)
        for (int64_t p = 0; p <= N; ++p) {
            const int64_t s = or_window_start(p, k);
            int st = OR_OK;
            int64_t c = 0;
            for (int64_t x = 0; x < n; ++x) w[x] = v[s * n + x] + g[s * n + x];
            for (int64_t j = s + 1; j <= p && st == OR_OK; ++j) {
                st = ml_step(P, L, j, v + (j - 1) * n, pv, work, &c);
                if (st == OR_OK) st = ml_step(P, L, j, w, pw, work, &c);
                for (int64_t x = 0; x < n; ++x) w[x] = pw[x] + ((v[j * n + x] - pv[x]) + g[j * n + x]);
            }
            for (int64_t x = 0; x < n; ++x) u[p * n + x] = w[x];
            cg_total += c;
            if (st) {
#pragma omp critical
                status = st;
            }
        }
        free(work);
    }
    if (cg) *cg += cg_total;
    return status;
}

/* One FAS V-cycle on level l (l < L-1) for A_l(u) = G (G = NULL on level 0: g_0 = g0, g_i = 0):
   F(CF)^nu relaxation, injection of the approximation and of its residual, the next level
   (recursively; local grids on the coarsest), e = u^(l+1) - v^(l+1), and the correction by ideal
   interpolation (add e at the C-points, then F-relax). */
static int ml_vcycle(const or_problem* P, const or_ml_options* O, const ml_level* lv, int l, double* u,
                     const double* G, const double* g0, int64_t* cg)
{
    const ml_level* L = &lv[l];
    const ml_level* Lc = &lv[l + 1];
    const int64_t n = nspace(P);
    const int64_t NC = Lc->nt; /* C-points 0..NC */
    int st = ml_f_relax(P, L, u, G, cg);
    if (!st && O->relax == 1) st = ml_c_relax(P, L, u, G, cg);
    if (!st && O->relax == 1) st = ml_f_relax(P, L, u, G, cg);
    if (st) return st;
    double* v = malloc(sizeof(double) * (NC + 1) * n);
    double* g = malloc(sizeof(double) * (NC + 1) * n);
    double* uc = malloc(sizeof(double) * (NC + 1) * n);
    st = ml_c_residual(P, L, u, G, g0, g, cg);
    for (int64_t j = 0; j <= NC; ++j)
        memcpy(v + j * n, u + j * L->m * n, sizeof(double) * n);
    memcpy(uc, v, sizeof(double) * (NC + 1) * n);
    if (!st) {
        if (l + 1 == O->levels - 1) {
            st = ml_local_solves(P, Lc, O->k, v, g, uc, cg);
        } else {
            /* the next level's FAS right-hand side G^(l+1) = A_{l+1}(v) + g */
            double* Gc = malloc(sizeof(double) * (NC + 1) * n);
            double* work = malloc(sizeof(double) * coarse_work_len(P));
            for (int64_t x = 0; x < n; ++x) Gc[x] = v[x] + g[x];
            for (int64_t j = 1; j <= NC && !st; ++j) {
                st = ml_step(P, Lc, j, v + (j - 1) * n, Gc + j * n, work, cg);
                for (int64_t x = 0; x < n; ++x) Gc[j * n + x] = (v[j * n + x] - Gc[j * n + x]) + g[j * n + x];
            }
            free(work);
            if (!st) st = ml_vcycle(P, O, lv, l + 1, uc, Gc, NULL, cg);
            free(Gc);
        }
    }
    if (!st) {
        for (int64_t j = 0; j <= NC; ++j)
            for (int64_t x = 0; x < n; ++x) u[j * L->m * n + x] += uc[j * n + x] - v[j * n + x];
        st = ml_f_relax(P, L, u, G, cg);
    }
    free(uc);
    free(g);
    free(v);
    return st;
}

/* Nested iteration (section 2.2; the setup phase of section 5): an improved initial guess built
   from the coarsest level up.  The guess u (u_0 = g_0) is injected to every level; on the coarsest
   level the local problems of the re-discretised system A_{L-1}(w) = g_{L-1} (g: u_0 at the first
   point, zero elsewhere) are solved from the injected guess v in FAS form, i.e. with the coarse
   residual g - A_{L-1}(v) as right-hand side; then each finer level takes the coarser level's
   values at its C-points and F-relaxes them (ideal interpolation), and every level between gets one
   V-cycle for its own re-discretised system.  The fine iterate returned is F-relaxed.  No source:
   the coarse levels would need it re-discretised too. */
int or_ml_nested(const or_problem* P, const or_ml_options* O, double* u, int64_t* cg)
{
    if (P->src) return OR_INVALID;
    ml_level lv[OR_MAX_LEVELS];
    int st = ml_levels(P, O, lv);
    if (st) return st;
    const int64_t n = nspace(P);
    const int Lc = O->levels - 1;
    double* lu[OR_MAX_LEVELS];
    lu[0] = u;
    for (int l = 1; l <= Lc; ++l) {
        lu[l] = malloc(sizeof(double) * (lv[l].nt + 1) * n);
        for (int64_t j = 0; j <= lv[l].nt; ++j)
            memcpy(lu[l] + j * n, lu[l - 1] + j * lv[l - 1].m * n, sizeof(double) * n);
    }
    /* coarsest level: residual of the injected guess, then the local problems */
    {
        const ml_level* L = &lv[Lc];
        double* g = malloc(sizeof(double) * (L->nt + 1) * n);
        double* w = malloc(sizeof(double) * (L->nt + 1) * n);
        double* work = malloc(sizeof(double) * coarse_work_len(P));
        const double* v = lu[Lc];
        for (int64_t x = 0; x < n; ++x) g[x] = u[x] - v[x];
        for (int64_t j = 1; j <= L->nt && !st; ++j) {
            st = ml_step(P, L, j, v + (j - 1) * n, g + j * n, work, cg);
            for (int64_t x = 0; x < n; ++x) g[j * n + x] = g[j * n + x] - v[j * n + x];
        }
        free(work);
        if (!st) st = ml_local_solves(P, L, O->k, v, g, w, cg);
        if (!st) memcpy(lu[Lc], w, sizeof(double) * (L->nt + 1) * n);
        free(w);
        free(g);
    }
    /* up the hierarchy: ideal interpolation, and one V-cycle on every level between */
    for (int l = Lc - 1; l >= 0 && !st; --l) {
        for (int64_t j = 0; j <= lv[l + 1].nt; ++j)
            memcpy(lu[l] + j * lv[l].m * n, lu[l + 1] + j * n, sizeof(double) * n);
        st = ml_f_relax(P, &lv[l], lu[l], NULL, cg);
        if (!st && l > 0) st = ml_vcycle(P, O, lv, l, lu[l], NULL, u, cg);
    }
    for (int l = 1; l <= Lc; ++l) free(lu[l]);
    return st;
}

int or_ml_cycle(const or_problem* P, const or_ml_options* O, double* u, const double* g0, int64_t* cg)
{
    ml_level lv[OR_MAX_LEVELS];
    int st = ml_levels(P, O, lv);
    if (st) return st;
    return ml_vcycle(P, O, lv, 0, u, NULL, g0, cg);
}

/* Multilevel FAS AT-MGRIT (Alg. 2) until ||g - A(u)||_2 <= tol, as or_atmgrit_solve: the guess is
   F-relaxed first, hist[0] is its residual norm, hist[i] the norm after V-cycle i. */
int or_ml_solve(const or_problem* P, const or_ml_options* O, double* u, double* hist, int32_t hist_cap,
                or_stats* S)
{
    const int64_t n = nspace(P);
    memset(S, 0, sizeof(*S));
    ml_level lv[OR_MAX_LEVELS];
    int st = ml_levels(P, O, lv);
    if (st) return S->status = st;
    double* g0 = malloc(sizeof(double) * n);
    double* r = malloc(sizeof(double) * (P->nt + 1) * n);
    memcpy(g0, u, sizeof(double) * n);
    if (O->nested) st = or_ml_nested(P, O, u, &S->cg_iters);
    if (!st) st = ml_f_relax(P, &lv[0], u, NULL, &S->cg_iters);
    double res = 0.0;
    if (!st) st = or_residual(P, u, g0, r, &S->cg_iters);
    if (!st) res = or_norm2((P->nt + 1) * n, r);
    if (!st && hist && hist_cap > 0) hist[0] = res;
    int it = 0;
    while (!st && !(res <= O->tol)) {
        if (!isfinite(res)) {
            st = OR_DIVERGED;
            break;
        }
        if (it >= O->max_iter) {
            st = OR_NOT_CONVERGED;
            break;
        }
        st = ml_vcycle(P, O, lv, 0, u, NULL, g0, &S->cg_iters);
        if (st) break;
        ++it;
        st = or_residual(P, u, g0, r, &S->cg_iters);
        if (!st) res = or_norm2((P->nt + 1) * n, r);
        if (!st && hist && it < hist_cap) hist[it] = res;
    }
    if (!st && !isfinite(res)) st = OR_DIVERGED;
    S->iterations = it;
    S->final_residual = res;
    S->status = st;
    free(r);
    free(g0);
    return st;
}
