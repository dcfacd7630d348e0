/* Runs the C oracle's entry points on small problems of every kind, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  The oracle is compiled into this file so that
 * its types are in scope; every call's status is checked, and any sanitizer report fails the run. */
#include "../../oracle/atm_oracle.c"

#include <stdio.h>

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            printf("check failed, line %d: %s\n", __LINE__, #c);          \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

static or_problem problem(int32_t kind, int32_t nx, int32_t ny, int64_t nt)
{
    or_problem P;
    memset(&P, 0, sizeof(P));
    P.kind = kind;
    P.nx = nx;
    P.ny = ny;
    P.nt = nt;
    P.length = 1.0;
    P.nu = kind == OR_AC2D ? 1.0 : 0.1;
    P.eps = 0.1;
    P.tf = kind == OR_AC2D ? nt * 2e-3 : 0.5;
    P.cg_rtol = 1e-12;
    P.cg_max_iter = 2000;
    return P;
}

static or_options options(int32_t m, int32_t k, int32_t relax, int32_t form)
{
    or_options O;
    memset(&O, 0, sizeof(O));
    O.tol = 1e-9;
    O.m = m;
    O.k = k;
    O.relax = relax;
    O.max_iter = 40;
    O.coarse_substeps = 1;
    O.coarse_form = form;
    return O;
}

/* initial condition: a smooth bump (heat) or small values (Allen-Cahn), zero guess elsewhere */
static double* guess(const or_problem* P)
{
    const int64_t n = (int64_t)P->nx * P->ny;
    double* u = calloc((size_t)(P->nt + 1) * n, sizeof(double));
    for (int64_t i = 0; i < n; ++i) u[i] = 0.5 * sin(0.7 * (double)i) * (P->kind == OR_AC2D ? 0.5 : 1.0);
    return u;
}

static void two_level(int32_t kind, int32_t nx, int32_t ny, int64_t nt, int32_t m, int32_t k, int32_t relax, int32_t form)
{
    const or_problem P = problem(kind, nx, ny, nt);
    const or_options O = options(m, k, relax, form);
    const int64_t n = (int64_t)nx * ny, NT = or_num_intervals(&P, &O);
    double* u = guess(&P);
    double* seq = guess(&P);
    int64_t cg = 0;
    CHECK(or_sequential(&P, seq, &cg) == OR_OK);
    /* the pieces of one cycle */
    double* w = guess(&P);
    CHECK(or_f_relax(&P, &O, w, &cg) == OR_OK);
    CHECK(or_c_relax(&P, &O, w, &cg) == OR_OK);
    double* r = calloc((size_t)(nt + 1) * n, sizeof(double));
    CHECK(or_residual(&P, w, w, r, &cg) == OR_OK);
    double* rc = calloc((size_t)(NT + 1) * n, sizeof(double));
    double* vc = calloc((size_t)(NT + 1) * n, sizeof(double));
    double* e = calloc((size_t)(NT + 1) * n, sizeof(double));
    for (int64_t j = 0; j <= NT; ++j) {
        memcpy(vc + j * n, w + j * m * n, sizeof(double) * n);
        if (j > 0) memcpy(rc + j * n, r + j * m * n, sizeof(double) * n);
    }
    int64_t ns = 0;
    CHECK(or_local_solves(&P, &O, rc, vc, e, &cg, &ns) == OR_OK);
    CHECK(or_correct(&P, &O, w, e, &cg) == OR_OK);
    /* a whole solve reaches the sequential solution */
    double hist[64];
    or_stats S;
    memset(&S, 0, sizeof(S));
    const int st = or_atmgrit_solve(&P, &O, u, hist, 64, &S);
    CHECK(st == OR_OK);
    double err = 0.0;
    for (int64_t i = 0; i < (nt + 1) * n; ++i) err = fmax(err, fabs(u[i] - seq[i]));
    CHECK(err < 1e-7);
    printf("kind %d %dx%d nt %lld m %d k %d relax %d form %d: status %d, %d cycles, max |u - seq| %.2e\n", kind, nx,
           ny, (long long)nt, m, k, relax, form, st, S.iterations, err);
    free(u);
    free(seq);
    free(w);
    free(r);
    free(rc);
    free(vc);
    free(e);
}

static void three_level(int nested)
{
    const or_problem P = problem(OR_HEAT2D, 12, 10, 32);
    or_ml_options O;
    memset(&O, 0, sizeof(O));
    O.tol = 1e-9;
    O.levels = 3;
    O.m[0] = 4;
    O.m[1] = 2;
    O.k = 2;
    O.relax = 1;
    O.max_iter = 60;
    O.coarse_substeps = 1;
    O.nested = nested;
    double* u = guess(&P);
    double hist[80];
    or_stats S;
    memset(&S, 0, sizeof(S));
    const int st = or_ml_solve(&P, &O, u, hist, 80, &S);
    CHECK(st == OR_OK);
    printf("three levels, nested %d: status %d, %d cycles\n", nested, st, S.iterations);
    free(u);
}

int main(void)
{
    two_level(OR_HEAT1D, 15, 1, 24, 4, 2, 1, 1);
    two_level(OR_HEAT1D, 9, 1, 21, 4, 7, 0, 1);   /* ragged last interval, k beyond N_T (Parareal) */
    two_level(OR_HEAT2D, 7, 5, 16, 4, 3, 1, 1);
    two_level(OR_HEAT2D, 6, 9, 12, 3, 2, 1, 2);   /* FAS form on a linear problem */
    two_level(OR_AC2D, 8, 8, 16, 4, 2, 1, 2);
    three_level(0);
    three_level(1);
    /* invalid arguments are refused, not read past */
    or_problem P = problem(OR_HEAT2D, 0, 5, 8);
    or_options O = options(4, 2, 1, 1);
    double u[8];
    or_stats S;
    CHECK(or_atmgrit_solve(&P, &O, u, NULL, 0, &S) == OR_INVALID);
    printf("%s\n", failures ? "FAILED" : "all checks passed");
    return failures ? 1 : 0;
}
