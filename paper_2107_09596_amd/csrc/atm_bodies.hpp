// Task bodies shared by the one-launch-per-phase kernels and the batched
// persistent kernel: each runs one interval or window of one instance on the
// calling workgroup, with LDS passed in by the caller.
#pragma once

#include "atm_device.hpp"
#include "atm_kernels.hpp"
#include "atm_spectral.hpp"

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
        if (a.src && act) x = x + a.dt * a.src[(j * a.m + t) * a.n + i];
        for (int q = 0; q < a.fine_substeps; ++q) x = pcr_solve(f, a.nx, x, lds);
        if (a.gadd && act) x = x + a.gadd[(j * a.m + t) * a.n + i];
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

// LV: a level below the finest (substeps and the additive FAS right-hand side of the multilevel
// cycle); a separate instantiation keeps the finest level's kernel as it is
template <int S, bool EX, bool PER, int COLS = kMaxSide2D + 2, bool LV = false>
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
    long long its = 0;
    for (int64_t t = 1; t <= total; ++t) {
        if constexpr (LV) {
            for (int q = 0; q < a.fine_substeps; ++q) its += step2d<S, EX, PER>(a, a.fine, a.rtol2, st, v, lp, red, slot);
            if (a.gadd) {
                const double* g = a.gadd + (j * a.m + t) * a.n;
#pragma unroll
                for (int s = 0; s < S; ++s)
                    if (row_ok<EX, S>(st, s)) v.x[s] = v.x[s] + g[(int64_t)(st.gbase + s * nx)];
            }
        } else {
            its += step2d<S, EX, PER>(a, a.fine, a.rtol2, st, v, lp, red, slot);
        }
        double* dst = (t < a.m) ? a.u + (j * a.m + t) * a.n : a.y + (j + 1) * a.n;
        strip_store<S, EX>(dst, st, nx, v.x);
    }
    count_cg(a, its);
}

// ---------------------------------------------------------------------------
// On-chip eigenbasis step (grids up to 128 per side): the field is a dense row-major matrix in the
// workgroup's LDS, row pitch P (odd, so that the 16 rows of a column fragment fall on distinct
// banks); the products alternate a table operand (global, L2-resident) with the LDS matrix on
// v_mfma_f64_16x16x4f64.  Output tile t = w + 8q (q < 8) of wave w: at most 64 tiles of 16 x 16.
// ---------------------------------------------------------------------------

constexpr int kSpecTiles = 8;  // output tiles per wave (8 waves: 128 x 128 at most)
constexpr int kSpecPass = 4;   // tiles accumulated at a time

// acc[q] (q < kSpecTiles) = the wave's tiles of X Y with X [M x K], Y [K x N].  XL: X is the LDS matrix D
// (pitch P) and Y a table in global memory (leading dimension ldq); otherwise Y is D and X a table, passed
// as its transpose Xt [K x M] so that a fragment reads 16 consecutive entries of a row.  Tile
// t = wave + 8 q covers rows 16 (t / nt) and columns 16 (t % nt), nt = ceil(N / 16); when nt divides 8
// every tile of a wave has the same columns and their Y fragment is read once.  Offsets are 32-bit from
// uniform bases; four tiles are accumulated at a time.
template <int P, bool XL>
__device__ __forceinline__ void spec_mm(const double* __restrict__ X, const double* __restrict__ Y, int ldq, int M,
                                        int N, int K, f64x4 (&acc)[kSpecTiles])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nt = (N + 15) >> 4, ntiles = ((M + 15) >> 4) * nt;
    const int ldy = XL ? ldq : P;
    const bool shared_y = (8 % nt) == 0;
#pragma unroll
    for (int q = 0; q < kSpecTiles; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int g = 0; g < kSpecTiles; g += kSpecPass) {
        if (wave + 8 * g >= ntiles) break;  // uniform over the wave
        // row offsets into X and columns of Y of this pass's tiles (-1: outside)
        int xo[kSpecPass], yj[kSpecPass];
#pragma unroll
        for (int q = 0; q < kSpecPass; ++q) {
            const int t = wave + 8 * (g + q);
            const int i = (t / nt) * 16 + li, j = (t % nt) * 16 + li;
            xo[q] = (t < ntiles && i < M) ? (XL ? i * P : i) : -1;
            yj[q] = (t < ntiles && j < N) ? j : -1;
        }
        auto load = [&](int k0, double (&fa)[kSpecPass], double (&fb)[kSpecPass]) {
            const int k = k0 + lk;
            const bool kin = k < K;
            const uint32_t yrow = (uint32_t)k * (uint32_t)ldy;
            const uint32_t xrow = XL ? 0u : (uint32_t)k * (uint32_t)ldq;
#pragma unroll
            for (int q = 0; q < kSpecPass; ++q)
                fa[q] = (kin && xo[q] >= 0) ? (XL ? X[(uint32_t)(xo[q] + k)] : X[xrow + (uint32_t)xo[q]]) : 0.0;
            if (shared_y) {
                const double b = (kin && yj[0] >= 0) ? Y[yrow + (uint32_t)yj[0]] : 0.0;
#pragma unroll
                for (int q = 0; q < kSpecPass; ++q) fb[q] = b;
            } else {
#pragma unroll
                for (int q = 0; q < kSpecPass; ++q) fb[q] = (kin && yj[q] >= 0) ? Y[yrow + (uint32_t)yj[q]] : 0.0;
            }
        };
#pragma unroll 1
        for (int k0 = 0; k0 < K; k0 += 4) {
            double fa[kSpecPass], fb[kSpecPass];
            load(k0, fa, fb);
#pragma unroll
            for (int q = 0; q < kSpecPass; ++q)
                acc[g + q] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[q], fb[q], acc[g + q], 0, 0, 0);
        }
    }
}

// D[i][j] = epi(i, j, acc) for the wave's tiles (result item r of lane l: row 4r + l/16, column l%16)
template <int P, typename F>
__device__ __forceinline__ void spec_store(double* D, int M, int N, const f64x4 (&acc)[kSpecTiles], F&& epi)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nt = (N + 15) >> 4, ntiles = ((M + 15) >> 4) * nt;
#pragma unroll
    for (int q = 0; q < kSpecTiles; ++q) {
        const int t = wave + 8 * q;
        if (t >= ntiles) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = (t / nt) * 16 + 4 * r + lk, j = (t % nt) * 16 + li;
            if (i < M && j < N) D[i * P + j] = epi(i, j, acc[q][r]);
        }
    }
}

// one Psi substep x <- M^-1 psi(x) (coarse coefficients) on the strip state, exactly in the eigenbasis
template <int S, bool EX, int P>
__device__ __forceinline__ void spectral_step2d(const KArgs& a, const Strip& st, double (&x)[S], double* D)
{
    const SpecTables T = spec_tables(a);
    const int nx = a.g.nx, ny = a.g.ny;
    const double cx2 = 2.0 * a.coarse.cx, cy2 = 2.0 * a.coarse.cy;
    auto same = [](int, int, double v) { return v; };
    f64x4 acc[kSpecTiles];
    __syncthreads();  // earlier readers of the LDS block are done
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (row_ok<EX, S>(st, s)) D[(st.y0 + s) * P + st.tx] = explicit_part(a.coarse, x[s]);
    __syncthreads();
    spec_mm<P, false>(T.qy, D, ny, ny, nx, ny, acc);   // Qy^T b (Qy^T read through its transpose Qy)
    __syncthreads();
    spec_store<P>(D, ny, nx, acc, same);
    __syncthreads();
    spec_mm<P, true>(D, T.qx, nx, ny, nx, nx, acc);    // (.. Qx) ./ mu
    __syncthreads();
    spec_store<P>(D, ny, nx, acc, [&](int i, int j, double v) { return v / (1.0 + (cx2 * T.ex[j] + cy2 * T.ey[i])); });
    __syncthreads();
    spec_mm<P, false>(T.qyt, D, ny, ny, nx, ny, acc);  // Qy .. (read through Qy^T)
    __syncthreads();
    spec_store<P>(D, ny, nx, acc, same);
    __syncthreads();
    spec_mm<P, true>(D, T.qxt, nx, ny, nx, nx, acc);   // .. Qx^T
    __syncthreads();
    spec_store<P>(D, ny, nx, acc, same);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S; ++s) x[s] = row_ok<EX, S>(st, s) ? D[(st.y0 + s) * P + st.tx] : 0.0;
    __syncthreads();  // the LDS block is free again (the CG's staging may follow)
}

// one Psi substep in the eigenbasis on the BF16 matrix cores with split operands (the four products
// of spectral_step2d, on dimensions padded to 16 and 32; LDS holds two hi/lo plane pairs of the
// geometry BfGeom<R>, which ping-pong between the products, and behind them the mode factors).  With
// `ay` non-null the step returns Psi(x) + ay at the strip's points; those loads are issued before the
// products, into the strip registers (free while the products run), so that their latency hides
// behind them.  LIN: x already is the right-hand side (M^-1 x, no explicit part).
template <int S, bool EX, int R, bool LIN = false>
__device__ __forceinline__ void bf_step2d(const KArgs& a, const Strip& st, double (&x)[S], double* lp,
                                          const double* ay)
{
    typedef BfGeom<R> G;
    __bf16* L = reinterpret_cast<__bf16*>(lp);
    __bf16 *r0h = L, *r0l = L + G::plane, *r1h = L + 2 * G::plane, *r1l = L + 3 * G::plane;
    const float* fex = reinterpret_cast<const float*>(L + 4 * G::plane);
    const float* fey = fex + R;
    const int nx = a.g.nx, ny = a.g.ny;
    const int mx = bf_r16(nx), my = bf_r16(ny), kx = bf_r32(nx), ky = bf_r32(ny);
    const float cx2 = (float)(2.0 * a.coarse.cx), cy2 = (float)(2.0 * a.coarse.cy);
    auto same = [](int, int, float v) { return v; };
    __syncthreads();  // earlier readers of the LDS block are done
    // b^T: column x of the field at row x of plane 0
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (row_ok<EX, S>(st, s)) {
            const double b = LIN ? x[s] : explicit_part(a.coarse, x[s]);
            const __bf16 h = (__bf16)b;
            const int o = st.tx * G::P + st.y0 + s;
            r0h[o] = h;
            r0l[o] = (__bf16)(b - (double)h);
        }
    if (ay) {
        const int64_t off = opaque_off(st.gbase);
#pragma unroll
        for (int s = 0; s < S; ++s)
            x[s] = row_ok<EX, S>(st, s) ? ay[off + (int64_t)s * nx] : 0.0;
    }
    __syncthreads();
    bf_mm<G::P>(r0h, r0l, bf_table(a, 0, 0), bf_table(a, 0, 1), ky, mx, my, ky, r1h, r1l, same);  // (Qy^T b)^T
    __syncthreads();
    bf_mm<G::P>(r1h, r1l, bf_table(a, 1, 0), bf_table(a, 1, 1), kx, my, mx, kx, r0h, r0l,         // .. Qx ./ mu
                [&](int i, int j, float v) { return v / (1.0f + (cx2 * fex[j] + cy2 * fey[i])); });
    __syncthreads();
    bf_mm<G::P>(r0h, r0l, bf_table(a, 2, 0), bf_table(a, 2, 1), ky, mx, my, ky, r1h, r1l, same);  // (Qy ..)^T
    __syncthreads();
    bf_mm<G::P>(r1h, r1l, bf_table(a, 3, 0), bf_table(a, 3, 1), kx, my, mx, kx, r0h, r0l, same);  // .. Qx^T
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int o = st.tx * G::P + st.y0 + s;
        const double v = (double)(float)r0h[o] + (double)(float)r0l[o];
        x[s] = row_ok<EX, S>(st, s) ? (ay ? v + x[s] : v) : 0.0;
    }
    __syncthreads();  // the LDS block is free again
}

// the mode factors of the BF16 eigenbasis step, staged as floats behind its LDS planes (once per
// task; zero beyond the grid, so that the padding keeps mu = 1)
template <int R>
__device__ __forceinline__ void bf_stage_modes(const KArgs& a, double* lp)
{
    float* fex = reinterpret_cast<float*>(reinterpret_cast<__bf16*>(lp) + 4 * BfGeom<R>::plane);
    const SpecTables T = spec_tables(a);
    for (int i = threadIdx.x; i < R; i += blockDim.x) {
        fex[i] = i < a.g.nx ? (float)T.ex[i] : 0.0f;
        fex[R + i] = i < a.g.ny ? (float)T.ey[i] : 0.0f;
    }
}

// Psi: s substeps, by CG, (SP) in the eigenbasis, or (BF) in the eigenbasis on the BF16 matrix
// cores; separate instantiations so that each kernel's registers serve one solver
template <int S, bool EX, bool PER, int COLS, bool SP, bool BF = false>
__device__ __forceinline__ long long psi2d(const KArgs& a, const Strip& st, Strip2DState<S>& v, double* lp,
                                           double* red, int& slot)
{
    long long its = 0;
    for (int q = 0; q < a.substeps; ++q) {
        if constexpr (BF)
            bf_step2d<S, EX, COLS - 2>(a, st, v.x, lp, nullptr);
        else if constexpr (SP)
            spectral_step2d<S, EX, COLS - 1>(a, st, v.x, lp);
        else
            its += step2d<S, EX, PER>(a, a.coarse, a.rtol2_coarse, st, v, lp, red, slot);
    }
    return its;
}

// BF: Psi in the eigenbasis on the BF16 matrix cores; BFC: with the residual rows a.cres formed
// beforehand (the single-instance launch), else r = y - u read after each step (the batch); BFF: the
// FAS form in terms of e = w - v (else the linear form)
template <int S, bool EX, bool PER, int COLS = kMaxSide2D + 2, bool SP = false, bool BF = false, bool BFC = true,
          bool BFF = false>
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
            const double r = (BF && BFC) ? a.cres[s0 * a.n + idx] : cpoint_residual(a, s0, idx);
            v.x[s] = (a.fas && !BF) ? a.u[(s0 * a.m) * a.n + idx] + r : r;  // BF carries e = w - v
        }
    }
    long long its = 0;
    if constexpr (BF) {
        // linear form: e_jj = Psi(e_{jj-1}) + r_jj; with the residual rows formed beforehand (BFC) the
        // last substep loads r_jj during its products, otherwise r_jj = y_jj - u_{jj m} is read after
        bf_stage_modes<COLS - 2>(a, lp);
        for (int64_t jj = s0 + 1; jj <= p; ++jj) {
            for (int q = 0; q + 1 < a.substeps; ++q) bf_step2d<S, EX, COLS - 2>(a, st, v.x, lp, nullptr);
            if constexpr (BFF) {
                // FAS in terms of e = w - v (one substep): e_jj = M^-1 (psi(v + e) - psi(v)) + r_jj with
                // v = u_{(jj-1) m}; the explicit parts' difference e + react (e - e (3 v^2 + 3 v e + e^2))
                // is formed in FP64, so the solve's error scales with e and vanishes with it
                const double react = a.coarse.react;
                const int64_t off = opaque_off(st.gbase);
                const double* vrow = a.u + ((jj - 1) * a.m) * a.n;
#pragma unroll
                for (int s = 0; s < S; ++s)
                    if (row_ok<EX, S>(st, s)) {
                        const double vv = vrow[off + (int64_t)s * nx], ee = v.x[s];
                        v.x[s] = ee + react * (ee - ee * (3.0 * vv * vv + 3.0 * vv * ee + ee * ee));
                    }
                if constexpr (BFC) {
                    bf_step2d<S, EX, COLS - 2, true>(a, st, v.x, lp, a.cres + jj * a.n);
                } else {
                    bf_step2d<S, EX, COLS - 2, true>(a, st, v.x, lp, nullptr);
                    const int64_t o2 = opaque_off(st.gbase);
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        if (row_ok<EX, S>(st, s)) v.x[s] = v.x[s] + cpoint_residual(a, jj, o2 + (int64_t)s * nx);
                }
            } else if constexpr (BFC) {
                bf_step2d<S, EX, COLS - 2>(a, st, v.x, lp, a.cres + jj * a.n);
            } else {
                bf_step2d<S, EX, COLS - 2>(a, st, v.x, lp, nullptr);
                const int64_t off = opaque_off(st.gbase);
#pragma unroll
                for (int s = 0; s < S; ++s)
                    if (row_ok<EX, S>(st, s)) v.x[s] = v.x[s] + cpoint_residual(a, jj, off + (int64_t)s * nx);
            }
        }
    } else {
        for (int64_t jj = s0 + 1; jj <= p; ++jj) {
            its += psi2d<S, EX, PER, COLS, SP, BF>(a, st, v, lp, red, slot);
            const int64_t off = opaque_off(st.gbase);
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (row_ok<EX, S>(st, s)) {
                    const int64_t idx = off + (int64_t)s * nx;
                    v.x[s] = v.x[s] + (a.fas ? a.tau[jj * a.n + idx] : cpoint_residual(a, jj, idx));
                }
        }
    }
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (row_ok<EX, S>(st, s)) {
            const int64_t idx = (int64_t)(st.gbase + s * nx);
            a.e[p * a.n + idx] = (a.fas && !BF) ? v.x[s] - a.u[(p * a.m) * a.n + idx] : v.x[s];
        }
    count_cg(a, its);
}

template <int S, bool EX, bool PER, int COLS = kMaxSide2D + 2, bool SP = false>
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
    long long its = psi2d<S, EX, PER, COLS, SP>(a, st, v, lp, red, slot);
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (row_ok<EX, S>(st, s)) {
            const int64_t idx = (int64_t)(st.gbase + s * nx);
            if (a.psi_only) {
                a.y[j * a.n + idx] = v.x[s];
            } else {
                const double vj = a.u[(j * a.m) * a.n + idx];
                a.tau[j * a.n + idx] = (vj - v.x[s]) + cpoint_residual(a, j, idx);
            }
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
        double psi2 = 0.0;
        if (EX || sd.nr > 0)
            strip_stencil<double, S, EX>(sd, ldsd, [&](int s, double u_, double c_, double d_, double w_, double e_) {
                const double ps = explicit_part(a.fine, up[s]);
                psi2 += ps * ps;
                const double res = ps - stencil_value(a.fine, u_, c_, d_, w_, e_);
                r[s] = (float)res;
                return res;
            });
        // (its barrier: every read of the FP64 staging precedes its reuse as FP32)
        psi2 = block_sum1(psi2, red, slot, kWaves2D);
        if (!PER) lds_clear_halo(a.g, lpf);
#pragma unroll
        for (int s = 0; s < S; ++s) x[s] = 0.0f;
        its += cg2d<float, S, EX, PER, true>(a.g, a.fine, sf, x, r, q, lpf, red, slot, a.rtol2_mixed, a.maxit,
                                             a.fail, defect_floor2(a.fine) * psi2);
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
