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

// ---------------------------------------------------------------------------
// The same solve on the BF16 matrix cores with split operands (coarse_solver 2; grids up to 128 per
// side, padded with zeros to multiples of 16 (rows, columns) and 32 (the products' inner dimension)).
// Padding stays zero through the four products: the task clears its LDS first, the table planes are
// zero beyond n, and the mode factors beyond n are zero (mu = 1).  Every operand is a pair hi + lo of BF16 values (hi = bf16(v),
// lo = bf16(v - hi)), and each product takes hi*hi + hi*lo + lo*hi in FP32 on
// v_mfma_f32_16x16x32_bf16: about 16 significant bits per operand, so the step is accurate to about
// 1e-5 relative, an approximation of the coarse propagator like an inexact CG (Psi only approximates
// Phi^m).  The tables are the four FP64 tables above in the same layouts, as hi and lo planes.
// ---------------------------------------------------------------------------

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__host__ __device__ inline int bf_r16(int n) { return (n + 15) & ~15; }
__host__ __device__ inline int bf_r32(int n) { return (n + 31) & ~31; }

// LDS geometry for grids of at most R points per side (R = 128, or 64 in the small-LDS variant): row
// pitch R + 8 BF16, so that the 16-byte fragments of 16 consecutive rows fall on distinct banks; four
// planes, then the mode factors ex, ey as R floats each
template <int R>
struct BfGeom {
    static constexpr int P = R + 8;
    static constexpr int plane = R * P;
};

// the BF16 planes start after the FP64 tables, at an even number of doubles (16-byte aligned)
__host__ __device__ inline int64_t bf_table_offset(int nx, int ny)
{
    const int64_t d = 2 * (int64_t)nx * nx + 2 * (int64_t)ny * ny + nx + ny;
    return (d + 1) & ~(int64_t)1;
}

// table t = qyt, qxt, qy, qx in turn (n = ny, nx, ny, nx): a [r16(n)][r32(n)] hi plane then lo plane
__device__ __forceinline__ const __bf16* bf_table(const KArgs& a, int t, int lo)
{
    const int nx = a.g.nx, ny = a.g.ny;
    const __bf16* base = reinterpret_cast<const __bf16*>(a.spec + bf_table_offset(nx, ny));
    const int64_t sy = (int64_t)bf_r16(ny) * bf_r32(ny), sx = (int64_t)bf_r16(nx) * bf_r32(nx);
    const int64_t sz = (t & 1) ? sx : sy;
    const int64_t off = (t == 0) ? 0 : (t == 1) ? 2 * sy : (t == 2) ? 2 * sy + 2 * sx : 4 * sy + 2 * sx;
    return base + off + (lo ? sz : 0);
}

// out[col][row] = epi(row, col, sum_k in[row][k] T[col][k]) for row < M, col < N (M, N multiples of
// 16, K of 32, N <= 128): `in` and `out` are LDS hi/lo planes with row pitch P, T a global table
// [N][ldt].  Wave w owns output columns 16w .. 16w+15 and walks the row blocks; no barrier inside.
template <int P, typename E>
__device__ __forceinline__ void bf_mm(const __bf16* ih, const __bf16* il, const __bf16* __restrict__ th,
                                      const __bf16* __restrict__ tl, int ldt, int M, int N, int K, __bf16* oh,
                                      __bf16* ol, E&& epi)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    if (16 * wave >= N) return;  // uniform over the wave
    const int col = 16 * wave + li;
    const int nk = K >> 5;
    // one accumulator per row block: the blocks' product chains are independent and interleave; the
    // k-steps stay a loop so that only one step's fragments are live, the next step's table
    // fragments being loaded while the current step's products run
    const int mb = M >> 4;
    f32x4_t acc[8];
#pragma unroll
    for (int ib = 0; ib < 8; ++ib) acc[ib] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    uint32_t to = (uint32_t)col * (uint32_t)ldt + (uint32_t)(8 * lk);
    bf16x8_t bh = *reinterpret_cast<const bf16x8_t*>(th + to);
    bf16x8_t bl = *reinterpret_cast<const bf16x8_t*>(tl + to);
#pragma unroll 1
    for (int kk = 0; kk < nk; ++kk) {
        bf16x8_t nh = bh, nl = bl;
        if (kk + 1 < nk) {
            to += 32;
            nh = *reinterpret_cast<const bf16x8_t*>(th + to);
            nl = *reinterpret_cast<const bf16x8_t*>(tl + to);
        }
#pragma unroll
        for (int ib = 0; ib < 8; ++ib)
            if (ib < mb) {
                const int o = (16 * ib + li) * P + 32 * kk + 8 * lk;
                const bf16x8_t ah = *reinterpret_cast<const bf16x8_t*>(ih + o);
                const bf16x8_t al = *reinterpret_cast<const bf16x8_t*>(il + o);
                acc[ib] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[ib], 0, 0, 0);
                acc[ib] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[ib], 0, 0, 0);
                acc[ib] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[ib], 0, 0, 0);
            }
        bh = nh;
        bl = nl;
    }
    // item r of the lane: row 16 ib + 4 lk + r, column col
#pragma unroll
    for (int ib = 0; ib < 8; ++ib)
        if (ib < mb) {
            bf16x4_t vh, vl;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float v = epi(16 * ib + 4 * lk + r, col, acc[ib][r]);
                const __bf16 h = (__bf16)v;
                vh[r] = h;
                vl[r] = (__bf16)(v - (float)h);
            }
            const int o = col * P + 16 * ib + 4 * lk;
            *reinterpret_cast<bf16x4_t*>(oh + o) = vh;
            *reinterpret_cast<bf16x4_t*>(ol + o) = vl;
        }
}

}  // namespace atm
