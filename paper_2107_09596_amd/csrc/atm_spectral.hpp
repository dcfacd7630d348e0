// Psi's implicit solve in the eigenbasis of the constant-coefficient operator: the tables and the
// basis, shared by the on-chip (small grid) and global-scratch (large grid) kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "atm_kernels.hpp"

namespace atm {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Psi's implicit solve in the eigenbasis of M = I - dT nu L (constant coefficients).
//
// The 1D second differences are diagonalised by orthonormal bases: Dirichlet (n interior points)
// Q[x][k] = sqrt(2/(n+1)) sin(pi (x+1)(k+1)/(n+1)), angle theta_k = pi (k+1)/(n+1); periodic (n
// points) the real Fourier basis, column 0 constant, columns 2m-1 / 2m cos / sin of 2 pi m x / n,
// (and for even n the last column (-1)^x), angle 2 pi m / n.  The 5-point operator
// M v = (1 + 2cx + 2cy) v - cx (w + e) - cy (n + s) has the eigenvalue
// 1 + 2cx ex[kx] + 2cy ey[ky], e = 1 - cos theta, on Qy[:, ky] (x) Qx[:, kx], so with the field b as
// an ny x nx matrix, M^-1 b = Qy ((Qy^T b Qx) ./ mu) Qx^T: four dense products; and as the bases
// are orthonormal, |M^-1 b| = |(Qy^T b Qx) ./ mu|: two.
// ---------------------------------------------------------------------------

constexpr double kPi = 3.14159265358979323846;

struct SpecTables {
    const double *qx, *qxt, *qy, *qyt, *ex, *ey;
};

__device__ __forceinline__ SpecTables spec_tables(const KArgs& a)
{
    const int64_t nx = a.g.nx, ny = a.g.ny;
    SpecTables t;
    t.qx = a.spec;
    t.qxt = t.qx + nx * nx;
    t.qy = t.qxt + nx * nx;
    t.qyt = t.qy + ny * ny;
    t.ex = t.qyt + ny * ny;
    t.ey = t.ex + nx;
    return t;
}

// basis entry Q[x][k] and mode angle of column k
__device__ __forceinline__ double basis(int n, bool periodic, int x, int k, double* theta)
{
    if (!periodic) {
        // angles reduced with integer arithmetic: pi t / (n + 1), t = (x+1)(k+1) mod 2(n+1)
        const int64_t t = ((int64_t)(x + 1) * (k + 1)) % (2 * (int64_t)(n + 1));
        *theta = kPi * (double)(k + 1) / (double)(n + 1);
        return sqrt(2.0 / (double)(n + 1)) * sin(kPi * (double)t / (double)(n + 1));
    }
    const int m = (k + 1) / 2;
    *theta = 2.0 * kPi * (double)m / (double)n;
    if (k == 0) return sqrt(1.0 / (double)n);
    const int64_t t = ((int64_t)m * x) % n;
    const double ang = 2.0 * kPi * (double)t / (double)n;
    if (2 * m == n) return sqrt(1.0 / (double)n) * ((x & 1) ? -1.0 : 1.0);
    return sqrt(2.0 / (double)n) * ((k & 1) ? cos(ang) : sin(ang));
}

}  // namespace atm
