// Task bodies shared by the one-launch-per-phase kernels and the batched
// persistent kernel: each runs one interval or window of one instance on the
// calling workgroup, with LDS passed in by the caller.
#pragma once

#include "atm_device.hpp"
#include "atm_kernels.hpp"

namespace atm {

// ---------------------------------------------------------------------------
// 1D heat: PCR tridiagonal steps, one workgroup (nx rounded up to wave64) per task
// ---------------------------------------------------------------------------

__device__ __forceinline__ void sweep1d_body(const KArgs& a, int64_t j, double* lds)
{
    const int i = threadIdx.x;
    const bool act = i < a.nx;
    Pcr1D f;
    pcr_setup(f, a.nx, a.fine.cx, lds);
    double x = 0.0;
    bool same = true;
    if (act) {
        x = sweep_start(a, j, i);
        same = !(x != a.u[(j * a.m) * a.n + i]);
        if (a.mode != 0) a.u[(j * a.m) * a.n + i] = x;
    }
    const int64_t total = (j < a.NT) ? a.m : (a.nt - a.NT * a.m);
    if (a.skip_unchanged && __syncthreads_and(same)) {
        skip_interval(a, j, total, i, 0, act ? 1 : 0);
        return;
    }
    for (int64_t t = 1; t <= total; ++t) {
        x = pcr_solve(f, a.nx, x, lds);
        if (act) {
            if (t < a.m)
                a.u[(j * a.m + t) * a.n + i] = x;
            else
                a.y[(j + 1) * a.n + i] = x;
        }
    }
}

// Psi: s substeps with the coarse factors
__device__ __forceinline__ double psi1d(const KArgs& a, const Pcr1D& fc, double x, double* lds)
{
    for (int q = 0; q < a.substeps; ++q) x = pcr_solve(fc, a.nx, x, lds);
    return x;
}

__device__ __forceinline__ void coarse1d_body(const KArgs& a, int64_t p, double* lds)
{
    const int i = threadIdx.x;
    const bool act = i < a.nx;
    Pcr1D fc;
    pcr_setup(fc, a.nx, a.coarse.cx, lds);
    const int64_t s = p - a.k + 1 > 0 ? p - a.k + 1 : 0;
    double w = 0.0, vs = 0.0;
    if (act) {
        if (a.fas) {
            vs = a.u[(s * a.m) * a.n + i];
            w = vs + cpoint_residual(a, s, i);
        } else {
            w = cpoint_residual(a, s, i);
        }
    }
    for (int64_t jj = s + 1; jj <= p; ++jj) {
        w = psi1d(a, fc, w, lds);
        if (act) w = w + (a.fas ? a.tau[jj * a.n + i] : cpoint_residual(a, jj, i));
    }
    if (act) a.e[p * a.n + i] = a.fas ? w - a.u[(p * a.m) * a.n + i] : w;
}

// ---------------------------------------------------------------------------
// 2D: one 512-thread workgroup per task, CG with p in LDS
// ---------------------------------------------------------------------------

template <int S>
struct Strip2DState {
    double x[S], r[S], q[S];
};

// One integrator step of size given by coefficients c, on the strip state.
template <int S, bool EX, bool PER>
__device__ __forceinline__ int step2d(const KArgs& a, const StepCoef& c, double rtol2, const Strip& st,
                                      Strip2DState<S>& v, double* lp, double* red, int& slot)
{
#pragma unroll
    for (int s = 0; s < S; ++s) v.r[s] = explicit_part(c, v.x[s]);
    return cg2d<double, S, EX, PER, true>(a.g, c, st, v.x, v.r, v.q, lp, red, slot, rtol2, a.maxit, a.fail);
}

template <int S, bool EX, bool PER, int COLS = kMaxSide2D + 2>
__device__ __forceinline__ void sweep2d_body(const KArgs& a, int64_t j, double* lp, double* red)
{
    int slot = 0;
    const Strip st = make_strip<double>(a.g);
    lds_clear<COLS>(lp);
    Strip2DState<S> v;
    const int nx = a.g.nx;
    bool same = true;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        v.x[s] = 0.0;
        if (row_ok<EX, S>(st, s)) {
            const int64_t idx = (int64_t)(st.gbase + s * nx);
            v.x[s] = sweep_start(a, j, idx);
            const double old = a.u[(j * a.m) * a.n + idx];
            same = same && !(v.x[s] != old);
            if (a.mode != 0) a.u[(j * a.m) * a.n + idx] = v.x[s];
        }
    }
    const int64_t total = (j < a.NT) ? a.m : (a.nt - a.NT * a.m);
    if (a.skip_unchanged && __syncthreads_and(same)) {
        skip_interval(a, j, total, st.gbase, nx, EX ? S : st.nr);
        return;
    }
    // Each step's CG starts from the linear extrapolation 2 x_{t-1} - x_{t-2} of the two previous
    // slices (x_{t-2} was stored by this workgroup one step earlier and is read back from L2; q is
    // free between solves); the first step starts from the C-point.  For a solution smooth in time
    // the start is off by O(dt^2) instead of O(dt).
    double* const base = a.u + (j * a.m) * a.n;
    long long its = 0;
    for (int64_t t = 1; t <= total; ++t) {
#pragma unroll
        for (int s = 0; s < S; ++s) v.r[s] = explicit_part(a.fine, v.x[s]);
        if (t >= 2) {
            const double* older = base + (t - 2) * a.n;
            const int64_t off = opaque_off(st.gbase);
#pragma unroll
            for (int s = 0; s < S; ++s) v.q[s] = row_ok<EX, S>(st, s) ? older[off + (int64_t)s * nx] : 0.0;
#pragma unroll
            for (int s = 0; s < S; ++s) v.x[s] = v.x[s] + (v.x[s] - v.q[s]);
        }
        its += cg2d<double, S, EX, PER, true>(a.g, a.fine, st, v.x, v.r, v.q, lp, red, slot, a.rtol2, a.maxit,
                                              a.fail);
        double* dst = (t < a.m) ? base + t * a.n : a.y + (j + 1) * a.n;
        strip_store<S, EX>(dst, st, nx, v.x);
    }
    count_cg(a, its);
}

template <int S, bool EX, bool PER>
__device__ __forceinline__ long long psi2d(const KArgs& a, const Strip& st, Strip2DState<S>& v, double* lp,
                                           double* red, int& slot)
{
    long long its = 0;
    for (int q = 0; q < a.substeps; ++q) its += step2d<S, EX, PER>(a, a.coarse, a.rtol2_coarse, st, v, lp, red, slot);
    return its;
}

template <int S, bool EX, bool PER, int COLS = kMaxSide2D + 2>
__device__ __forceinline__ void coarse2d_body(const KArgs& a, int64_t p, double* lp, double* red)
{
    int slot = 0;
    const int64_t s0 = p - a.k + 1 > 0 ? p - a.k + 1 : 0;
    const Strip st = make_strip<double>(a.g);
    lds_clear<COLS>(lp);
    const int nx = a.g.nx;
    Strip2DState<S> v;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        v.x[s] = 0.0;
        if (row_ok<EX, S>(st, s)) {
            const int64_t idx = (int64_t)(st.gbase + s * nx);
            const double r = cpoint_residual(a, s0, idx);
            v.x[s] = a.fas ? a.u[(s0 * a.m) * a.n + idx] + r : r;
        }
    }
    long long its = 0;
    for (int64_t jj = s0 + 1; jj <= p; ++jj) {
        its += psi2d<S, EX, PER>(a, st, v, lp, red, slot);
        const int64_t off = opaque_off(st.gbase);
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (row_ok<EX, S>(st, s)) {
                const int64_t idx = off + (int64_t)s * nx;
                v.x[s] = v.x[s] + (a.fas ? a.tau[jj * a.n + idx] : cpoint_residual(a, jj, idx));
            }
    }
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (row_ok<EX, S>(st, s)) {
            const int64_t idx = (int64_t)(st.gbase + s * nx);
            a.e[p * a.n + idx] = a.fas ? v.x[s] - a.u[(p * a.m) * a.n + idx] : v.x[s];
        }
    count_cg(a, its);
}

template <int S, bool EX, bool PER, int COLS = kMaxSide2D + 2>
__device__ __forceinline__ void tau2d_body(const KArgs& a, int64_t j, double* lp, double* red)
{
    int slot = 0;
    const Strip st = make_strip<double>(a.g);
    lds_clear<COLS>(lp);
    const int nx = a.g.nx;
    Strip2DState<S> v;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        v.x[s] = 0.0;
        if (row_ok<EX, S>(st, s)) v.x[s] = a.u[((j - 1) * a.m) * a.n + (int64_t)(st.gbase + s * nx)];
    }
    long long its = psi2d<S, EX, PER>(a, st, v, lp, red, slot);
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (row_ok<EX, S>(st, s)) {
            const int64_t idx = (int64_t)(st.gbase + s * nx);
            const double vj = a.u[(j * a.m) * a.n + idx];
            a.tau[j * a.n + idx] = (vj - v.x[s]) + cpoint_residual(a, j, idx);
        }
    count_cg(a, its);
}

// ---------------------------------------------------------------------------
// 2D precision form (FP32 fine solves, FP64 defect and update)
// ---------------------------------------------------------------------------

// Zero the halo cells of an LDS vector of a Dirichlet grid: columns -1 and nx
// (rows -1..ny) and rows -1 and ny of every column.  The mixed sweep reuses one
// LDS block for an FP64 and an FP32 vector, so each layout's halo is cleared
// before that layout is written.
template <typename T>
__device__ __forceinline__ void lds_clear_halo(const Grid2D& g, T* lp)
{
    constexpr int H = Lds2D<T>::H, V = Lds2D<T>::V;
    const int rows = g.ny + 2;
    for (int i = threadIdx.x; i < 2 * rows; i += blockDim.x) {
        const int col = (i < rows) ? 0 : g.nx + 1;
        const int y = (i < rows) ? i : i - rows;
        lp[col * H + V - 1 + y] = (T)0;
    }
    for (int i = threadIdx.x; i < 2 * g.nx; i += blockDim.x) {
        const int col = 1 + (i >> 1);
        lp[col * H + ((i & 1) ? V + g.ny : V - 1)] = (T)0;
    }
}

// Mixed sweep over interval j (one workgroup per task, modes as in the FP64
// sweep).  The starting value of the step that produces y_{j+1} = Phi(u_{jm+m-1})
// is, by mode: 0 the C-point u_{(j+1)m}; 1 y_{j+1} on entry (y is in/out);
// 2 aux_{j+1} (the Phi values of the previous sweep).
template <int S, bool EX, bool PER, int COLS = kMaxSide2D + 2>
__device__ __forceinline__ void sweep2d_mixed_body(const KArgs& a, int64_t j, double* ldsd, double* red)
{
    // one LDS block holds the FP64 staging of u_i^old for the defect and then
    // the FP32 search direction of the CG (the FP32 layout is the smaller one)
    static_assert(Lds2D<float>::H * sizeof(float) <= Lds2D<double>::H * sizeof(double), "LDS alias");
    float* lpf = reinterpret_cast<float*>(ldsd);
    int slot = 0;
    const Strip sd = make_strip<double>(a.g);
    const Strip sf = make_strip<float>(a.g);
    const int nx = a.g.nx;
    lds_clear<COLS>(ldsd);
    double up[S];
    float x[S], r[S], q[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        up[s] = 0.0;
        if (row_ok<EX, S>(sd, s)) {
            const int64_t idx = (int64_t)(sd.gbase + s * nx);
            up[s] = sweep_start(a, j, idx);
            if (a.mode != 0) a.u[(j * a.m) * a.n + idx] = up[s];
        }
    }
    const int64_t total = (j < a.NT) ? a.m : (a.nt - a.NT * a.m);
    long long its = 0;
    for (int64_t t = 1; t <= total; ++t) {
        const bool ystep = (t == a.m);
        const double* xo;
        if (!ystep)
            xo = a.u + (j * a.m + t) * a.n;
        else
            xo = (a.mode == 0 ? a.u + ((j + 1) * a.m) * a.n : (a.mode == 1 ? a.y : a.aux) + (j + 1) * a.n);
        double* dst = ystep ? a.y + (j + 1) * a.n : a.u + (j * a.m + t) * a.n;
        // defect of the starting value in FP64, rounded to FP32 as the CG right-hand side
        if (!PER) lds_clear_halo(a.g, ldsd);
        {
            const int64_t off = opaque_off(sd.gbase);
            lds_put_fn<double, S, EX, PER, false>(a.g, sd, ldsd,
                                                  [&](int s, double) { return xo[off + (int64_t)s * nx]; });
        }
        __syncthreads();
        if (EX || sd.nr > 0)
            strip_stencil<double, S, EX>(sd, ldsd, [&](int s, double u_, double c_, double d_, double w_, double e_) {
                const double res = explicit_part(a.fine, up[s]) - stencil_value(a.fine, u_, c_, d_, w_, e_);
                r[s] = (float)res;
                return res;
            });
        __syncthreads();  // every read of the FP64 staging precedes its reuse as FP32
        if (!PER) lds_clear_halo(a.g, lpf);
#pragma unroll
        for (int s = 0; s < S; ++s) x[s] = 0.0f;
        its += cg2d<float, S, EX, PER, true>(a.g, a.fine, sf, x, r, q, lpf, red, slot, a.rtol2_mixed, a.maxit,
                                             a.fail);
        {
            const int64_t off = opaque_off(sd.gbase);
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (row_ok<EX, S>(sd, s)) {
                    const double v = xo[off + (int64_t)s * nx] + (double)x[s];
                    up[s] = v;
                    dst[off + (int64_t)s * nx] = v;
                }
        }
        __syncthreads();  // the next step's FP64 staging overwrites the FP32 direction
    }
    count_cg(a, its);
}

}  // namespace atm
