// Device building blocks for the AT-MGRIT kernels (gfx950, wave64).
//
//  * block_sum2      -- deterministic two-value block reduction (wave butterfly + LDS).
//  * Pcr1D           -- batched constant-coefficient tridiagonal solve by parallel
//                       cyclic reduction; the per-level elimination factors depend
//                       only on the matrix, so they are formed once per kernel.
//  * cg2d            -- Jacobi-preconditioned conjugate gradients for
//                       M = d I - cx (E + W) - cy (N + S) with one workgroup per
//                       system: the search direction p lives in LDS (it is the only
//                       vector the stencil reads at neighbours), x, r and M p live
//                       in VGPRs as a vertical strip of `rows` points per thread
//                       (512 threads: up to 32 FP64 rows x 3 vectors = 192 VGPRs).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace atm {

constexpr int kBlock2D = 512;  // 8 wave64s (2 per SIMD, 256 VGPRs each): one workgroup per interval owns a CU
constexpr int kWaves2D = kBlock2D / 64;

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

// Move a double through a DPP lane permutation (two 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave.  Each 16-lane row is summed by rotations
// (row_ror 8, 4, 2, 1: every lane of the row ends with the row total, in a
// lane-dependent order), then lane 0 of every row is read into a scalar and
// the four row totals are added in a fixed order, so every lane returns the
// same, reproducible value.  No LDS traffic.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0x128>(v);  // row_ror:8
    v += dpp_f64<0x124>(v);  // row_ror:4
    v += dpp_f64<0x122>(v);  // row_ror:2
    v += dpp_f64<0x121>(v);  // row_ror:1
    const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
    const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
    return (r0 + r1) + (r2 + r3);
}

// Sum two doubles over the block.  `red` holds 2 * 2 * nwaves doubles; the
// caller alternates `slot` between calls so a slow reader of the previous
// result never races a fast writer of the next one.  All threads return the
// same values (fixed summation order).
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red, int& slot, int nwaves)
{
    // keep surrounding strip loops from being interleaved into the reduction
    // (that would keep whole strips of loaded values live across it)
    __builtin_amdgcn_sched_barrier(0);
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    double* base = red + slot * 2 * nwaves;
    if (lane == 0) {
        base[wave] = a;
        base[nwaves + wave] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < nwaves; ++w) {
        sa += base[w];
        sb += base[nwaves + w];
    }
    a = sa;
    b = sb;
    slot ^= 1;
    __builtin_amdgcn_sched_barrier(0);
}

// One-value form of block_sum2.
__device__ __forceinline__ double block_sum1(double a, double* red, int& slot, int nwaves)
{
    __builtin_amdgcn_sched_barrier(0);
    a = wave_sum(a);
    double* base = red + slot * 2 * nwaves;
    if ((threadIdx.x & 63) == 0) base[threadIdx.x >> 6] = a;
    __syncthreads();
    double sa = 0.0;
    for (int w = 0; w < nwaves; ++w) sa += base[w];
    slot ^= 1;
    __builtin_amdgcn_sched_barrier(0);
    return sa;
}

// ---------------------------------------------------------------------------
// 1D: constant tridiagonal (1 + 2c) x_i - c x_{i-1} - c x_{i+1} = d_i, zero ends
// ---------------------------------------------------------------------------

constexpr int kPcrLevels = 10;  // n <= 1024

struct Pcr1D {
    double k1[kPcrLevels];
    double k2[kPcrLevels];
    double invb;
    int levels;
};

// Form the elimination factors of row i (thread i, i < n).  `lds` holds
// 3 * blockDim doubles.  Every thread of the block must call it.
__device__ inline void pcr_setup(Pcr1D& f, int n, double c, double* lds)
{
    const int i = threadIdx.x;
    const int nb = blockDim.x;
    double* A = lds;
    double* B = lds + nb;
    double* C = lds + 2 * nb;
    double a = (i > 0 && i < n) ? -c : 0.0;
    double b = 1.0 + 2.0 * c;
    double cc = (i < n - 1) ? -c : 0.0;
    int levels = 0;
    for (int s = 1; s < n; s <<= 1) ++levels;
    f.levels = levels;
#pragma unroll
    for (int l = 0; l < kPcrLevels; ++l) {
        f.k1[l] = 0.0;
        f.k2[l] = 0.0;
    }
    for (int l = 0; l < levels; ++l) {
        const int s = 1 << l;
        __syncthreads();
        A[i] = a;
        B[i] = b;
        C[i] = cc;
        __syncthreads();
        const int im = i - s, ip = i + s;
        double k1 = 0.0, k2 = 0.0, na = 0.0, nc = 0.0, nb2 = b;
        if (i < n) {
            if (im >= 0) {
                k1 = a / B[im];
                na = -A[im] * k1;
                nb2 -= C[im] * k1;
            }
            if (ip < n) {
                k2 = cc / B[ip];
                nc = -C[ip] * k2;
                nb2 -= A[ip] * k2;
            }
        }
        // levels is uniform across the block, so this indexing stays in registers after unrolling
#pragma unroll
        for (int q = 0; q < kPcrLevels; ++q)
            if (q == l) {
                f.k1[q] = k1;
                f.k2[q] = k2;
            }
        a = na;
        cc = nc;
        b = nb2;
    }
    f.invb = 1.0 / b;
    __syncthreads();
}

// Solve with right-hand side d (row i in thread i); returns x_i.  `lds` holds
// 2 * blockDim doubles (double buffer).  Every thread must call it.
__device__ inline double pcr_solve(const Pcr1D& f, int n, double d, double* lds)
{
    const int i = threadIdx.x;
    const int nb = blockDim.x;
#pragma unroll
    for (int l = 0; l < kPcrLevels; ++l) {
        if (l < f.levels) {
            double* buf = lds + (l & 1) * nb;
            buf[i] = d;
            __syncthreads();
            const int s = 1 << l;
            const int im = i - s, ip = i + s;
            const double dm = (im >= 0) ? buf[im] : 0.0;
            const double dp = (ip < n) ? buf[ip] : 0.0;
            d = d - f.k1[l] * dm - f.k2[l] * dp;
        }
    }
    __syncthreads();
    return d * f.invb;
}

// ---------------------------------------------------------------------------
// 2D: strip decomposition and CG
// ---------------------------------------------------------------------------

struct Grid2D {
    int nx, ny;
    int tx_log2;  // threads along x: TX = 1 << tx_log2 >= nx (TX in {64, 128})
    int rows;     // rows per thread strip: a multiple of 16 / sizeof(T), <= the template S
    int periodic;
};

struct StepCoef {
    double cx, cy;   // nu dt / hx^2, nu dt / hy^2
    double d;        // diagonal 1 + 2 cx + 2 cy
    double inv_d;    // Jacobi scaling
    double react;    // dt / eps^2 for the explicit Allen-Cahn term, 0 for heat
};

// The LDS copy of a vector is stored column by column with a one-cell halo:
// element (x, y) sits at (x + 1) * H + y + V, V = 16 / sizeof(T) values per
// 16-byte access.  A thread owns rows y0 .. y0+rows-1 of column x, so its strip
// and the strips of its west and east neighbours are contiguous runs at a
// fixed distance H: one base register plus immediate offsets, 16-byte loads.
// H is padded so that consecutive lanes (stride H) spread 16-byte loads over
// all banks.  The halo (column -1 and nx, rows -1 and ny) is zero for Dirichlet
// problems and a copy of the opposite edge for periodic ones.
constexpr int kMaxSide2D = 128;
template <typename T>
struct Lds2D;
template <>
struct Lds2D<double> {
    static constexpr int V = 2;
    static constexpr int H = 146;  // >= 128 + 2 + 8 * V; 2H mod 32 = 4
    static constexpr int size = (kMaxSide2D + 2) * H;
    typedef double2 vec;
};
template <>
struct Lds2D<float> {
    static constexpr int V = 4;
    static constexpr int H = 164;  // >= 128 + 4 + 8 * V; H mod 32 = 4
    static constexpr int size = (kMaxSide2D + 2) * H;
    typedef float4 vec;
};

template <typename T>
union VecU {
    typename Lds2D<T>::vec v;
    T a[Lds2D<T>::V];
};

struct Strip {
    int tx, y0, nr;
    int lbase;  // LDS index of (tx, y0)
    int gbase;  // global index of (tx, y0): y0 * nx + tx
};

template <typename T>
__device__ __forceinline__ Strip make_strip(const Grid2D& g)
{
    Strip st;
    st.tx = threadIdx.x & ((1 << g.tx_log2) - 1);
    st.y0 = (threadIdx.x >> g.tx_log2) * g.rows;
    int nr = g.ny - st.y0;
    nr = nr < g.rows ? nr : g.rows;
    st.nr = (st.tx < g.nx && nr > 0) ? nr : 0;
    st.lbase = (st.tx + 1) * Lds2D<T>::H + st.y0 + Lds2D<T>::V;
    st.gbase = st.y0 * g.nx + st.tx;
    return st;
}

// EXACT: the grid is tiled exactly (nx == TX, ny == TY * S), so no row is masked.
template <bool EXACT, int S>
__device__ __forceinline__ bool row_ok(const Strip& st, int s)
{
    return EXACT ? true : s < st.nr;
}

// Zero the whole LDS vector including its halo (once per kernel; ends with a
// barrier so no clear can land after a strip store of another thread).
// COLS: LDS columns held by the caller (grid columns + 2 halo columns at most;
// the full size fits every grid up to the largest side).
template <int COLS = kMaxSide2D + 2, typename T>
__device__ __forceinline__ void lds_clear(T* lp)
{
    for (int i = threadIdx.x; i < COLS * Lds2D<T>::H; i += blockDim.x) lp[i] = (T)0;
    __syncthreads();
}

// Write the strip into LDS one 16-byte chunk at a time, value of row s given
// by f(s, old) where old is the value currently stored there (read only when
// READ_OLD).  Periodic grids mirror edge values into the halo.  Rows past the
// grid edge are not written.  Each thread touches only its own cells and
// their halo copies.
template <typename T, int S, bool EXACT, bool PER, bool READ_OLD, typename F>
__device__ __forceinline__ void lds_put_fn(const Grid2D& g, const Strip& st, T* lp, F&& f)
{
    constexpr int V = Lds2D<T>::V;
    constexpr int H = Lds2D<T>::H;
    typedef typename Lds2D<T>::vec vec;
    if (!EXACT && st.nr == 0) return;
    const bool xedge = PER && (st.tx == 0 || st.tx == g.nx - 1);
    const int xoff = (st.tx == 0) ? g.nx * H : -g.nx * H;
    int base = st.lbase;
#pragma unroll
    for (int s = 0; s < S; s += V) {
        VecU<T> u;
        u.a[0] = (T)0;
        if (EXACT || s < st.nr) {
            if (READ_OLD) u.v = *reinterpret_cast<const vec*>(lp + base + s);
#pragma unroll
            for (int i = 0; i < V; ++i) u.a[i] = (EXACT || s + i < st.nr) ? f(s + i, u.a[i]) : (T)0;
            if (EXACT || s + V <= st.nr) {
                *reinterpret_cast<vec*>(lp + base + s) = u.v;
            } else {
                // a chunk cut by the grid edge: rows past it belong to the halo
                // (periodic copies of row 0) and must not be overwritten
#pragma unroll
                for (int i = 0; i < V; ++i)
                    if (s + i < st.nr) lp[base + s + i] = u.a[i];
            }
            if (PER) {
#pragma unroll
                for (int i = 0; i < V; ++i)
                    if (EXACT || s + i < st.nr) {
                        const int y = st.y0 + s + i;
                        const int o = base + s + i;
                        if (xedge) lp[o + xoff] = u.a[i];
                        if (y == 0) lp[o + g.ny] = u.a[i];
                        if (y == g.ny - 1) lp[o - g.ny] = u.a[i];
                    }
            }
        }
        __asm__ volatile("" : "+v"(base) : "v"(u.a[0]));
    }
}

// Walk the strip in chunks of V rows and call f(s, up, cen, dn, w, e) per row,
// with the 5-point neighbourhood of p read from LDS.
template <typename T, int S, bool EXACT, typename F>
__device__ __forceinline__ void strip_stencil(const Strip& st, const T* lp, F&& f)
{
    constexpr int V = Lds2D<T>::V;
    constexpr int H = Lds2D<T>::H;
    typedef typename Lds2D<T>::vec vec;
    // `base` is passed through an empty asm after every chunk, with that chunk's
    // last result as an input: the next chunk's loads then depend on the current
    // chunk's arithmetic and cannot be hoisted above it, which bounds the number
    // of loaded values alive at once.  f returns a value it computed.
    int base = st.lbase;
    T up = lp[base - 1];
    VecU<T> cur;
    cur.v = *reinterpret_cast<const vec*>(lp + base);
#pragma unroll
    for (int s = 0; s < S; s += V) {
        VecU<T> nxt, w, e;
        if (s + V < S)
            nxt.v = *reinterpret_cast<const vec*>(lp + base + s + V);
        else
            nxt.a[0] = lp[base + S];
        w.v = *reinterpret_cast<const vec*>(lp + base + s - H);
        e.v = *reinterpret_cast<const vec*>(lp + base + s + H);
        T last = (T)0;
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const T dn = (i + 1 < V) ? cur.a[i + 1] : nxt.a[0];
            if (row_ok<EXACT, S>(st, s + i)) last = f(s + i, up, cur.a[i], dn, w.a[i], e.a[i]);
            up = cur.a[i];
        }
        cur = nxt;
        __asm__ volatile("" : "+v"(base) : "v"(last));
    }
}

template <typename T>
__device__ __forceinline__ T stencil_value(const StepCoef& c, T up, T cen, T dn, T w, T e)
{
    return (T)c.d * cen - (T)c.cx * (w + e) - (T)c.cy * (up + dn);
}

// Jacobi-preconditioned CG for M x = b on one workgroup.  M has the constant
// diagonal d, so the Jacobi preconditioner is the scalar 1/d: with the scaled
// direction p~ = d p the iterates x_k, r_k are exactly those of Jacobi-PCG
// (alpha~ = (r,r)/(p~,Mp~), beta = (r',r')/(r,r)), without the division and
// without the second dot product.
//   x : in the initial guess, out the solution (strip registers)
//   r : in b, out the final recursive residual (strip registers)
//   q : scratch strip registers (M p~ of the current iteration, then p~)
//   lp: column-major haloed LDS vector (halo zeroed by the caller; periodic
//       halos are maintained by lds_put_fn);  red: LDS reduction scratch
// Stops when (r, r) <= rtol2 (b, b); b = 0 returns x = 0.  On reaching maxit
// sets *fail and returns with the current iterate.  Returns the iteration count.
template <typename T, int S, bool EXACT, bool PER, bool STOREQ>
__device__ int cg2d(const Grid2D& g, const StepCoef& c, const Strip& st, T (&x)[S], T (&r)[S], T (&q)[S], T* lp,
                    double* red, int& slot, double rtol2, int maxit, int* fail, double bb_floor = 0.0)
{
    constexpr int V = Lds2D<T>::V;
    typedef typename Lds2D<T>::vec vec;
    const bool any = EXACT || st.nr > 0;
    // stage the initial guess for the stencil; (b, b)
    double bb = 0.0, rr = 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (row_ok<EXACT, S>(st, s)) bb += (double)r[s] * (double)r[s];
    lds_put_fn<T, S, EXACT, PER, false>(g, st, lp, [&](int s, T) { return x[s]; });
    __syncthreads();
    if (any)
        strip_stencil<T, S, EXACT>(st, lp, [&](int s, T up, T cen, T dn, T w, T e) {
            r[s] = r[s] - stencil_value(c, up, cen, dn, w, e);
            rr += (double)r[s] * (double)r[s];
            return r[s];
        });
    block_sum2(bb, rr, red, slot, kWaves2D);
    // b = 0 has the solution x = 0 (set after the loop, which is skipped); so does a b at or below
    // bb_floor (a defect at the rounding level of its own evaluation)
    const bool bzero = !(bb > bb_floor);
    const double thresh = rtol2 * bb;
    double gamma = rr;
    // p~ = r (every reader of the staged x has passed the reduction's barrier)
    lds_put_fn<T, S, EXACT, PER, false>(g, st, lp, [&](int s, T) { return r[s]; });
    __syncthreads();
    int it = 0;
    while (!bzero && rr > thresh && it < maxit) {
        // q = M p~ and (p~, q)
        double pq = 0.0;
        if (any)
            strip_stencil<T, S, EXACT>(st, lp, [&](int s, T up, T cen, T dn, T w, T e) {
                const T v = stencil_value(c, up, cen, dn, w, e);
                if (STOREQ) q[s] = v;
                pq += (double)cen * (double)v;
                return v;
            });
        pq = block_sum1(pq, red, slot, kWaves2D);
        const T alpha = (T)(gamma / pq);
        // x += alpha p~, r -= alpha q; q takes p~ for the direction update
        rr = 0.0;
        if (any && STOREQ) {
            int base = st.lbase;
#pragma unroll
            for (int s = 0; s < S; s += V) {
                VecU<T> p;
                p.v = *reinterpret_cast<const vec*>(lp + base + s);
#pragma unroll
                for (int i = 0; i < V; ++i)
                    if (row_ok<EXACT, S>(st, s + i)) {
                        x[s + i] = x[s + i] + alpha * p.a[i];
                        r[s + i] = r[s + i] - alpha * q[s + i];
                        rr += (double)r[s + i] * (double)r[s + i];
                        q[s + i] = p.a[i];
                    }
                __asm__ volatile("" : "+v"(base) : "v"(r[s]));
            }
        } else if (any) {
            strip_stencil<T, S, EXACT>(st, lp, [&](int s, T up, T cen, T dn, T w, T e) {
                const T v = stencil_value(c, up, cen, dn, w, e);
                x[s] = x[s] + alpha * cen;
                r[s] = r[s] - alpha * v;
                rr += (double)r[s] * (double)r[s];
                return r[s];
            });
        }
        rr = block_sum1(rr, red, slot, kWaves2D);
        const T beta = (T)(rr / gamma);
        gamma = rr;
        // p~ = r + beta p~ (each thread rewrites only its own cells and halo copies)
        if (STOREQ)
            lds_put_fn<T, S, EXACT, PER, false>(g, st, lp, [&](int s, T) { return r[s] + beta * q[s]; });
        else
            lds_put_fn<T, S, EXACT, PER, true>(g, st, lp, [&](int s, T old) { return r[s] + beta * old; });
        __syncthreads();
        ++it;
    }
    if (!bzero && rr > thresh && threadIdx.x == 0) atomicOr(fail, 1);  // cg_max_iter reached
    if (bzero) {
#pragma unroll
        for (int s = 0; s < S; ++s) x[s] = (T)0;
    }
    return it;
}

}  // namespace atm
