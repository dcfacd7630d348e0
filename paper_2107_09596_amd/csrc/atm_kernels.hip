// HIP kernels of the two-level AT-MGRIT hot path (FP64 form), gfx950.
//
// Layout: u is [nt+1][n] FP64, t = j m + i; y, e, tau are [N_T+1][n].
// One workgroup owns one coarse interval (relaxation sweeps) or one local coarse
// grid (window solves); the sequential time loop of that interval/window runs
// inside the workgroup with the current state held on chip, so HBM sees each
// fine point written once per sweep and never re-read by the sweep.
#include "atm_device.hpp"
#include "atm_kernels.hpp"
#include "atm_spectral.hpp"
#include "atm_bodies.hpp"

namespace atm {

// ---------------------------------------------------------------------------
// 1D heat: PCR tridiagonal steps, one workgroup (nx rounded up to wave64) per task
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void sweep1d_kernel(KArgs a)
{
    __shared__ double lds[3 * 1024];
    sweep1d_body(a, blockIdx.x, lds);
}

__global__ __launch_bounds__(1024) void coarse1d_kernel(KArgs a)
{
    __shared__ double lds[3 * 1024];
    coarse1d_body(a, blockIdx.x, lds);
}

// tau_j = (v_j - Psi(v_{j-1})) + r_j, j = 1..N_T (FAS right-hand side, shared by all windows)
__global__ __launch_bounds__(1024) void tau1d_kernel(KArgs a)
{
    __shared__ double lds[3 * 1024];
    const int64_t j = blockIdx.x + 1;
    const int i = threadIdx.x;
    const bool act = i < a.nx;
    Pcr1D fc;
    pcr_setup(fc, a.nx, a.coarse.cx, lds);
    double v = act ? a.u[((j - 1) * a.m) * a.n + i] : 0.0;
    v = psi1d(a, fc, v, lds);
    if (act) {
        if (a.psi_only) {
            a.y[j * a.n + i] = v;
        } else {
            const double vj = a.u[(j * a.m) * a.n + i];
            a.tau[j * a.n + i] = (vj - v) + cpoint_residual(a, j, i);
        }
    }
}

__global__ __launch_bounds__(1024) void seq1d_kernel(KArgs a)
{
    __shared__ double lds[3 * 1024];
    const int i = threadIdx.x;
    const bool act = i < a.nx;
    Pcr1D f;
    pcr_setup(f, a.nx, a.fine.cx, lds);
    double x = act ? a.u[i] : 0.0;
    for (int64_t t = 1; t <= a.nt; ++t) {
        if (a.src && act) x = x + a.dt * a.src[t * a.n + i];
        x = pcr_solve(f, a.nx, x, lds);
        if (act) a.u[t * a.n + i] = x;
    }
}

// ---------------------------------------------------------------------------
// 2D: one 512-thread workgroup per task, CG with p in LDS
// ---------------------------------------------------------------------------


template <int S, bool EX, bool PER>
__global__ __launch_bounds__(kBlock2D) void sweep2d_kernel(KArgs a)
{
    __shared__ __align__(16) double lp[Lds2D<double>::size];
    __shared__ double red[4 * kWaves2D];
    sweep2d_body<S, EX, PER>(a, blockIdx.x, lp, red);
}

// a level below the finest of the multilevel cycle (substeps, additive FAS right-hand side)
template <int S, bool EX, bool PER>
__global__ __launch_bounds__(kBlock2D) void sweep2d_lv_kernel(KArgs a)
{
    __shared__ __align__(16) double lp[Lds2D<double>::size];
    __shared__ double red[4 * kWaves2D];
    sweep2d_body<S, EX, PER, kMaxSide2D + 2, true>(a, blockIdx.x, lp, red);
}

// The window a workgroup takes.  Workgroups are dealt to the eight XCDs in turn (block b to XCD
// b mod 8), and window p reads the C-point residuals of its k slices s..p: windows p, p+1, ... share
// k - 1 of them.  Block b takes window (b mod 8) * per + b / 8 (per = count / 8), so that every XCD
// runs a run of consecutive windows and serves their shared slices from its own L2; the blocks past
// 8 * per take the remaining windows in order.
__device__ __forceinline__ int64_t xcd_window(int64_t b, int64_t count)
{
    const int64_t per = count / 8;
    return b < 8 * per ? (b % 8) * per + b / 8 : b;
}

template <int S, bool EX, bool PER>
__global__ __launch_bounds__(kBlock2D) void coarse2d_kernel(KArgs a)
{
    __shared__ __align__(16) double lp[Lds2D<double>::size];
    __shared__ double red[4 * kWaves2D];
    coarse2d_body<S, EX, PER>(a, xcd_window(blockIdx.x, gridDim.x), lp, red);
}

template <int S, bool EX, bool PER>
__global__ __launch_bounds__(kBlock2D) void tau2d_kernel(KArgs a)
{
    __shared__ __align__(16) double lp[Lds2D<double>::size];
    __shared__ double red[4 * kWaves2D];
    tau2d_body<S, EX, PER>(a, blockIdx.x + 1, lp, red);  // windows 1..N_T
}

// the same with Psi in the eigenbasis
template <int S, bool EX, bool PER>
__global__ __launch_bounds__(kBlock2D) void coarse2d_spec_kernel(KArgs a)
{
    __shared__ __align__(16) double lp[Lds2D<double>::size];
    __shared__ double red[4 * kWaves2D];
    coarse2d_body<S, EX, PER, kMaxSide2D + 2, true>(a, xcd_window(blockIdx.x, gridDim.x), lp, red);
}

// Psi in the eigenbasis on the BF16 matrix cores: linear form, and FAS in terms of e = w - v
template <int S, bool EX, bool PER>
__global__ __launch_bounds__(kBlock2D) void coarse2d_bf_kernel(KArgs a)
{
    __shared__ __align__(16) double lp[Lds2D<double>::size];
    __shared__ double red[4 * kWaves2D];
    coarse2d_body<S, EX, PER, kMaxSide2D + 2, false, true, true, false>(a, xcd_window(blockIdx.x, gridDim.x), lp, red);
}

template <int S, bool EX, bool PER>
__global__ __launch_bounds__(kBlock2D) void coarse2d_bf_fas_kernel(KArgs a)
{
    __shared__ __align__(16) double lp[Lds2D<double>::size];
    __shared__ double red[4 * kWaves2D];
    coarse2d_body<S, EX, PER, kMaxSide2D + 2, false, true, true, true>(a, xcd_window(blockIdx.x, gridDim.x), lp, red);
}

template <int S, bool EX, bool PER>
__global__ __launch_bounds__(kBlock2D) void tau2d_spec_kernel(KArgs a)
{
    __shared__ __align__(16) double lp[Lds2D<double>::size];
    __shared__ double red[4 * kWaves2D];
    tau2d_body<S, EX, PER, kMaxSide2D + 2, true>(a, blockIdx.x + 1, lp, red);
}

template <int S, bool EX, bool PER>
__global__ __launch_bounds__(kBlock2D) void seq2d_kernel(KArgs a)
{
    __shared__ __align__(16) double lp[Lds2D<double>::size];
    __shared__ double red[4 * kWaves2D];
    int slot = 0;
    const Strip st = make_strip<double>(a.g);
    lds_clear(lp);
    const int nx = a.g.nx;
    Strip2DState<S> v;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        v.x[s] = 0.0;
        if (row_ok<EX, S>(st, s)) v.x[s] = a.u[(int64_t)(st.gbase + s * nx)];
    }
    long long its = 0;
    for (int64_t t = 1; t <= a.nt; ++t) {
        its += step2d<S, EX, PER>(a, a.fine, a.rtol2, st, v, lp, red, slot);
        strip_store<S, EX>(a.u + t * a.n, st, nx, v.x);
    }
    count_cg(a, its);
}

// ---------------------------------------------------------------------------
// residual norm: deterministic two-stage sum of ||y_j - u_{jm}||^2, j = 1..N_T; each C-point row is
// cut into `chunks` pieces so that the first stage fills the chip (2048 workgroups at most, the size
// of the partials array)
// ---------------------------------------------------------------------------

constexpr int kNormBlock = 256;

static int64_t norm_chunks(const KArgs& a)
{
    int64_t c = kResidBlocks / (a.NT > 0 ? a.NT : 1);
    const int64_t by_size = (a.n + kNormBlock - 1) / kNormBlock;  // at least one element per thread
    if (c > by_size) c = by_size;
    if (c > 16) c = 16;
    return c < 1 ? 1 : c;
}

__global__ __launch_bounds__(kNormBlock) void norm_partial_kernel(KArgs a, int64_t chunks)
{
    __shared__ double red[2 * 2 * (kNormBlock / 64)];
    int slot = 0;
    const int64_t j = blockIdx.x / chunks + 1, q = blockIdx.x % chunks;
    const int64_t lo = q * a.n / chunks, hi = (q + 1) * a.n / chunks;
    double acc = 0.0, unused = 0.0;
    for (int64_t idx = lo + threadIdx.x; idx < hi; idx += kNormBlock) {
        const double r = a.y[j * a.n + idx] - a.u[(j * a.m) * a.n + idx];
        acc += r * r;
    }
    block_sum2(acc, unused, red, slot, kNormBlock / 64);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kNormBlock) void norm_final_kernel(KArgs a, int64_t count)
{
    __shared__ double red[2 * 2 * (kNormBlock / 64)];
    int slot = 0;
    double acc = 0.0, unused = 0.0;
    for (int64_t j = threadIdx.x; j < count; j += kNormBlock) acc += a.partials[j];
    block_sum2(acc, unused, red, slot, kNormBlock / 64);
    if (threadIdx.x == 0) {
        a.hdr->norm2 = acc;
        publish_header(a);
    }
}

// The same sum in one workgroup for small problems (N_T n <= kNormSmall): thread t adds the squares of
// the elements t, t + 1024, ... of the C-point residuals in order, then the block sum
constexpr int kNormSmallBlock = 1024;
constexpr int64_t kNormSmall = 1 << 16;
__global__ __launch_bounds__(kNormSmallBlock) void norm_small_kernel(KArgs a)
{
    __shared__ double red[2 * 2 * (kNormSmallBlock / 64)];
    int slot = 0;
    double acc = 0.0, unused = 0.0;
    const int64_t total = a.NT * a.n;
    for (int64_t e = threadIdx.x; e < total; e += kNormSmallBlock) {
        const int64_t j = e / a.n + 1, idx = e % a.n;
        const double r = a.y[j * a.n + idx] - a.u[(j * a.m) * a.n + idx];
        acc += r * r;
    }
    block_sum2(acc, unused, red, slot, kNormSmallBlock / 64);
    if (threadIdx.x == 0) {
        a.hdr->norm2 = acc;
        publish_header(a);
    }
}

__global__ void reset_header_kernel(Header* h)
{
    if (threadIdx.x == 0) {
        h->norm2 = 0.0;
        h->fail = 0;
        h->cg_fine = 0ull;
        h->cg_coarse = 0ull;
        h->skipped = 0ull;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define ATM_LAUNCH_S(kernel, S, EX, PER, grid, stream, args)                                                 \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(kernel<S, EX, PER>), dim3(grid), dim3(kBlock2D), 0, (hipStream_t)(stream), \
                       args)

#define ATM_LAUNCH_EP(kernel, S, grid, stream, args)                             \
    do {                                                                         \
        if ((args).exact) {                                                      \
            if ((args).g.periodic) ATM_LAUNCH_S(kernel, S, true, true, grid, stream, args);    \
            else ATM_LAUNCH_S(kernel, S, true, false, grid, stream, args);                     \
        } else {                                                                 \
            if ((args).g.periodic) ATM_LAUNCH_S(kernel, S, false, true, grid, stream, args);   \
            else ATM_LAUNCH_S(kernel, S, false, false, grid, stream, args);                    \
        }                                                                        \
    } while (0)

// strip length S in {8, 16, 32}; EX = exact tiling (no masked rows); PER = periodic halo
#define ATM_LAUNCH_2D(kernel, grid, stream, args)                      \
    do {                                                               \
        switch ((args).s_tmpl) {                                       \
            case 8: ATM_LAUNCH_EP(kernel, 8, grid, stream, args); break;   \
            case 16: ATM_LAUNCH_EP(kernel, 16, grid, stream, args); break; \
            default: ATM_LAUNCH_EP(kernel, 32, grid, stream, args); break; \
        }                                                              \
    } while (0)

static int block1d(const KArgs& a) { return ((a.nx + 63) / 64) * 64; }

void launch_reset(Header* h, hipStream_t s) { hipLaunchKernelGGL(reset_header_kernel, dim3(1), dim3(64), 0, s, h); }

void launch_sweep(const KArgs& a, int64_t n_tasks, hipStream_t s)
{
    if (a.is1d)
        hipLaunchKernelGGL(sweep1d_kernel, dim3(n_tasks), dim3(block1d(a)), 0, s, a);
    else if (a.gadd || a.fine_substeps > 1)
        ATM_LAUNCH_2D(sweep2d_lv_kernel, n_tasks, s, a);
    else
        ATM_LAUNCH_2D(sweep2d_kernel, n_tasks, s, a);
}

// dst[r] = src[r * stride_rows] for rows r = 0..rows-1 of n doubles (injection to C-points)
__global__ __launch_bounds__(256) void gather_rows_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                          int64_t n, int64_t stride_rows, int64_t rows)
{
    const int64_t total = n * rows;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
        const int64_t r = q / n, x = q - r * n;
        dst[q] = src[r * stride_rows * n + x];
    }
}

// r_j = y_j - u_{jm} for j = 1..N_T, r_0 = 0 (the C-point residuals of the windows, coarse_solver 2)
__global__ __launch_bounds__(256) void cpoint_residuals_kernel(KArgs a)
{
    const int64_t total = a.n * (a.NT + 1);
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
        const int64_t j = q / a.n, x = q - j * a.n;
        a.cres[q] = cpoint_residual(a, j, x);
    }
}

void launch_cpoint_residuals(const KArgs& a, hipStream_t s)
{
    const int64_t total = a.n * (a.NT + 1);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) return;
    hipLaunchKernelGGL(cpoint_residuals_kernel, dim3(blocks), dim3(256), 0, s, a);
}

void launch_gather(const double* src, double* dst, int64_t n, int64_t stride_rows, int64_t rows, hipStream_t s)
{
    const int64_t total = n * rows;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) return;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks), dim3(256), 0, s, src, dst, n, stride_rows, rows);
}

void launch_tau(const KArgs& a, hipStream_t s)
{
    if (a.NT < 1) return;
    if (a.is1d)
        hipLaunchKernelGGL(tau1d_kernel, dim3(a.NT), dim3(block1d(a)), 0, s, a);
    else if (a.spectral)
        ATM_LAUNCH_2D(tau2d_spec_kernel, a.NT, s, a);
    else
        ATM_LAUNCH_2D(tau2d_kernel, a.NT, s, a);
}

void launch_coarse(const KArgs& a, hipStream_t s)
{
    if (a.is1d)
        hipLaunchKernelGGL(coarse1d_kernel, dim3(a.NT + 1), dim3(block1d(a)), 0, s, a);
    else if (a.spectral == 2) {
        launch_cpoint_residuals(a, s);
        if (a.fas)
            ATM_LAUNCH_2D(coarse2d_bf_fas_kernel, a.NT + 1, s, a);
        else
            ATM_LAUNCH_2D(coarse2d_bf_kernel, a.NT + 1, s, a);
    }
    else if (a.spectral)
        ATM_LAUNCH_2D(coarse2d_spec_kernel, a.NT + 1, s, a);
    else
        ATM_LAUNCH_2D(coarse2d_kernel, a.NT + 1, s, a);
}

void launch_norm(const KArgs& a, hipStream_t s)
{
    if (a.NT * a.n <= kNormSmall) {
        hipLaunchKernelGGL(norm_small_kernel, dim3(1), dim3(kNormSmallBlock), 0, s, a);
        return;
    }
    const int64_t chunks = norm_chunks(a);
    const int64_t blocks = a.NT >= 1 ? a.NT * chunks : 0;
    if (blocks > 0) hipLaunchKernelGGL(norm_partial_kernel, dim3(blocks), dim3(kNormBlock), 0, s, a, chunks);
    hipLaunchKernelGGL(norm_final_kernel, dim3(1), dim3(kNormBlock), 0, s, a, blocks);
}

void launch_sequential(const KArgs& a, hipStream_t s)
{
    if (a.is1d)
        hipLaunchKernelGGL(seq1d_kernel, dim3(1), dim3(block1d(a)), 0, s, a);
    else
        ATM_LAUNCH_2D(seq2d_kernel, 1, s, a);
}

// ---------------------------------------------------------------------------
// eigenbasis tables of the 2D operator (see atm_spectral.hpp): they depend on the grid only
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void spectral_tables_kernel(KArgs a)
{
    const int nx = a.g.nx, ny = a.g.ny;
    const bool per = a.g.periodic != 0;
    double* qx = a.spec;
    double* qxt = qx + (int64_t)nx * nx;
    double* qy = qxt + (int64_t)nx * nx;
    double* qyt = qy + (int64_t)ny * ny;
    double* ex = qyt + (int64_t)ny * ny;
    double* ey = ex + nx;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double th;
    for (int64_t i = first; i < (int64_t)nx * nx; i += stride) {
        const int x = (int)(i / nx), k = (int)(i % nx);
        const double v = basis(nx, per, x, k, &th);
        qx[(int64_t)x * nx + k] = v;
        qxt[(int64_t)k * nx + x] = v;
    }
    for (int64_t i = first; i < (int64_t)ny * ny; i += stride) {
        const int y = (int)(i / ny), k = (int)(i % ny);
        const double v = basis(ny, per, y, k, &th);
        qy[(int64_t)y * ny + k] = v;
        qyt[(int64_t)k * ny + y] = v;
    }
    for (int64_t k = first; k < nx; k += stride) {
        (void)basis(nx, per, 0, (int)k, &th);
        ex[k] = 1.0 - cos(th);
    }
    for (int64_t k = first; k < ny; k += stride) {
        (void)basis(ny, per, 0, (int)k, &th);
        ey[k] = 1.0 - cos(th);
    }
}


size_t spectral_table_doubles(int nx, int ny) { return 2 * (size_t)nx * nx + 2 * (size_t)ny * ny + nx + ny; }

// the BF16 hi/lo planes of qyt, qxt, qy, qx ([r16(n)][r32(n)] each, zero padded), after the FP64
// tables rounded up to an even number of doubles: in doubles, counted from the FP64 tables' start
size_t spectral_bf16_doubles(int nx, int ny)
{
    const size_t sx = (size_t)bf_r16(nx) * bf_r32(nx), sy = (size_t)bf_r16(ny) * bf_r32(ny);
    return (size_t)(bf_table_offset(nx, ny) - (int64_t)spectral_table_doubles(nx, ny)) + sx + sy;
}

__global__ __launch_bounds__(256) void spectral_bf16_kernel(KArgs a)
{
    const int nx = a.g.nx, ny = a.g.ny;
    const double* src[4] = {a.spec + 2 * (int64_t)nx * nx + (int64_t)ny * ny, a.spec + (int64_t)nx * nx,
                            a.spec + 2 * (int64_t)nx * nx, a.spec};  // qyt, qxt, qy, qx
    __bf16* dst = reinterpret_cast<__bf16*>(a.spec + bf_table_offset(nx, ny));
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int t = 0; t < 4; ++t) {
        const int n = (t & 1) ? nx : ny;
        const int rows = bf_r16(n), cols = bf_r32(n);
        const int64_t sz = (int64_t)rows * cols;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < sz; i += stride) {
            const int r = (int)(i / cols), c = (int)(i % cols);
            const double v = (r < n && c < n) ? src[t][(int64_t)r * n + c] : 0.0;
            const __bf16 h = (__bf16)v;
            dst[i] = h;
            dst[sz + i] = (__bf16)(v - (double)h);
        }
        dst += 2 * sz;
    }
}

void launch_spectral_tables(const KArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(spectral_tables_kernel, dim3(64), dim3(256), 0, s, a);
    if (a.spectral == 2) hipLaunchKernelGGL(spectral_bf16_kernel, dim3(64), dim3(256), 0, s, a);
}

}  // namespace atm
