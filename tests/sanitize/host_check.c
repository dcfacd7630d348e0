/* The library's host-side argument checks and workspace layout, built host-only (no device code) with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Reads one configuration
 * per line on stdin -- kind nx ny nt m k relax precision coarse_solver coarse_form levels m_coarse
 * nested coarse_substeps -- and prints, for each, the workspace size, the interval count and the
 * status of a solve called without a workspace (refused before any device call).  Then checks the
 * refusals of invalid arguments. */
#include "../../include/atm.h"

#include <stdio.h>
#include <string.h>

static int failures = 0;
#define CHECK(c)                                                 \
    do {                                                         \
        if (!(c)) {                                              \
            printf("check failed, line %d: %s\n", __LINE__, #c); \
            ++failures;                                          \
        }                                                        \
    } while (0)

static atm_problem problem(int kind, int nx, int ny, long long nt)
{
    atm_problem p;
    memset(&p, 0, sizeof(p));
    p.kind = kind;
    p.nx = nx;
    p.ny = ny;
    p.nt = nt;
    p.length = 1.0;
    p.nu = 1.0;
    p.eps = 1.0;
    p.t0 = 0.0;
    p.tf = 1.0;
    p.cg_rtol = 1e-12;
    p.cg_max_iter = 1000;
    return p;
}

static atm_options options(int m, int k)
{
    atm_options o;
    memset(&o, 0, sizeof(o));
    o.m = m;
    o.k = k;
    o.relax = 1;
    o.tol = 1e-8;
    o.max_iter = 100;
    o.coarse_substeps = 1;
    o.levels = 2;
    return o;
}

int main(void)
{
    int kind, nx, ny, m, k, relax, precision, solver, form, levels, m_coarse, nested, substeps;
    long long nt;
    while (scanf("%d %d %d %lld %d %d %d %d %d %d %d %d %d %d", &kind, &nx, &ny, &nt, &m, &k, &relax, &precision,
                 &solver, &form, &levels, &m_coarse, &nested, &substeps) == 14) {
        atm_problem p = problem(kind, nx, ny, nt);
        atm_options o = options(m, k);
        o.relax = relax;
        o.precision = precision;
        o.coarse_solver = solver;
        o.coarse_form = form;
        o.levels = levels;
        o.m_coarse = m_coarse;
        o.nested = nested;
        o.coarse_substeps = substeps;
        const size_t ws = atm_workspace_bytes(&p, &o);
        const long long NT = (long long)atm_num_intervals(&p, &o);
        double u[1];
        const atm_status st = atm_solve(&p, &o, u, NULL, 0, NULL, 0, NULL, NULL);
        printf("%zu %lld %d\n", ws, NT, (int)st);
        CHECK(ws == 0 || st == ATM_ERR_WORKSPACE);
        CHECK(strlen(atm_last_error()) > 0);
    }
    /* refusals */
    atm_problem p = problem(ATM_HEAT2D, 16, 16, 32);
    atm_options o = options(4, 2);
    double u[1];
    p.nx = 0;
    CHECK(atm_solve(&p, &o, u, NULL, 0, NULL, 0, NULL, NULL) == ATM_ERR_INVALID_ARG);
    p.nx = 16;
    o.m = 1;
    CHECK(atm_solve(&p, &o, u, NULL, 0, NULL, 0, NULL, NULL) == ATM_ERR_INVALID_ARG);
    o.m = 4;
    o.k = 0;
    CHECK(atm_workspace_bytes(&p, &o) == 0);
    o.k = 2;
    CHECK(atm_solve(NULL, &o, u, NULL, 0, NULL, 0, NULL, NULL) == ATM_ERR_INVALID_ARG);
    CHECK(atm_solve(&p, NULL, u, NULL, 0, NULL, 0, NULL, NULL) == ATM_ERR_INVALID_ARG);
    CHECK(atm_sweep(&p, &o, 7, u, NULL, u, NULL, 0, NULL) != ATM_OK);
    CHECK(atm_window_start(5, 2) == 4 && atm_window_start(0, 3) == 0);
    CHECK(atm_static_scratch_bytes() > 0);
    CHECK(atm_cnn_param_count() > 0);
    CHECK(strlen(atm_status_string(ATM_ERR_INVALID_ARG)) > 0);
    printf("%s\n", failures ? "FAILED" : "all checks passed");
    return failures ? 1 : 0;
}
