// Mixed-precision form of the hot path: FP32 fine solves, FP64 residual,
// correction and iterate, so that the AT-MGRIT cycle acts as iterative
// refinement.
//
// Every fine step of a mixed sweep updates u_i in defect-correction form:
//     rho   = psi(u_{i-1}) - M u_i^old          FP64 stencil of the stored iterate
//     M d   = rho                               FP32 CG to relative tolerance rtol_mixed
//     u_i^new = u_i^old + d                     FP64
// with M = I - dt nu L and psi(v) = v (heat) or v + dt (v - v^3) / eps^2
// (Allen-Cahn), u_{i-1} the slice just produced.  In exact arithmetic this is
// u_i = Phi(u_{i-1}); the FP32 error is a fraction rtol_mixed of |d|, so it
// vanishes as the iteration converges and the fixed point is the FP64 one
// (u_i = M^-1 psi(u_{i-1}) to FP64 rounding).
//
// The stopping test uses the FP64 implicit residual rho_i = psi(u_{i-1}) - M u_i
// over all points: r_i = M^-1 rho_i and |M^-1| <= 1 (M = I - dt nu L, L <= 0),
// so |r| <= |rho|.  The final paper-form residual |r| is formed by solving
// M r_i = rho_i in FP64 (step_residual kernels), which avoids the cancellation
// of Phi(u_{i-1}) - u_i.
#include "atm_device.hpp"
#include "atm_kernels.hpp"
#include "atm_bodies.hpp"

namespace atm {

template <int S, bool EX, bool PER>
__global__ __launch_bounds__(kBlock2D) void sweep2d_mixed_kernel(KArgs a)
{
    __shared__ __align__(16) double ldsd[Lds2D<double>::size];
    __shared__ double red[4 * kWaves2D];
    sweep2d_mixed_body<S, EX, PER>(a, blockIdx.x, ldsd, red);
}

// FP64 implicit residual |rho|^2 = sum_i |psi(u_{i-1}) - M u_i|^2, i = 1..nt.
// HBM-bound: each slice leaves HBM once.  A workgroup (4 waves) owns a tile of 64 columns x 4 kResRows
// rows of the slice over a chunk of consecutive time indices; lane l of wave w holds column x0 + l, rows
// y0 + w kResRows .. + kResRows - 1, and keeps the previous slice's values there in registers.  Per step
// a lane loads its own points (coalesced over the wave) and the two halo rows; the north / south
// neighbours come from its registers, the west / east ones from lanes l -+ 1 by DPP wave shifts (the
// wave's edge lanes and the grid's edge columns load theirs).  Work units are numbered so that the
// tiles of one chunk run on one XCD (the dispatcher deals workgroups to the 8 XCDs in turn) and share
// its L2 for the halo rows.
constexpr int kResidThreads = 256;
constexpr int kResRows = 8;
constexpr int kResTileRows = 4 * kResRows;

// the value of v held by lane l - 1 (dir = 0) or l + 1 (dir = 1) of the wave (0 where there is none)
__device__ __forceinline__ double wave_shift(double v, int dir)
{
    const long long b = __double_as_longlong(v);
    int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
    if (dir == 0) {
        lo = __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xf, 0xf, true);  // wave_shr:1
        hi = __builtin_amdgcn_update_dpp(0, hi, 0x138, 0xf, 0xf, true);
    } else {
        lo = __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xf, 0xf, true);  // wave_shl:1
        hi = __builtin_amdgcn_update_dpp(0, hi, 0x130, 0xf, 0xf, true);
    }
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

__global__ __launch_bounds__(kResidThreads) void implicit_residual_kernel(KArgs a, int64_t ntile, int64_t chunk,
                                                                          int64_t units)
{
    __shared__ double red[2 * 2 * (kResidThreads / 64)];
    int slot = 0;
    const int64_t per_xcd = gridDim.x / 8;
    const int64_t w = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (w >= units) return;  // whole workgroup, before any barrier
    const int nx = a.nx;
    const int ny = (int)(a.n / nx);
    const int tiles_x = (nx + 63) / 64;
    const int64_t tile = w % ntile;
    const int64_t i0 = 1 + (w / ntile) * chunk;
    const int64_t i1 = (i0 + chunk - 1 < a.nt) ? i0 + chunk - 1 : a.nt;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x = (int)(tile % tiles_x) * 64 + lane;
    const int y0 = (int)(tile / tiles_x) * kResTileRows + wv * kResRows;
    const bool per = a.g.periodic != 0;
    const bool colok = x < nx;
    // columns whose west / east neighbour is loaded: the wave's edge lanes and the grid's edge columns
    const int xw = x == 0 ? (per ? nx - 1 : -1) : x - 1;
    const int xe = x == nx - 1 ? (per ? 0 : -1) : x + 1;
    const bool load_w = colok && (lane == 0 || x == 0);
    const bool load_e = colok && (lane == 63 || x == nx - 1);
    // halo rows: above the first row, below the last (zero outside a Dirichlet boundary)
    const int yu = y0 == 0 ? (per ? ny - 1 : -1) : y0 - 1;
    const int ylast = (y0 + kResRows < ny ? y0 + kResRows : ny) - 1;  // last row of the strip in the grid
    const int yd = ylast == ny - 1 ? (per ? 0 : -1) : ylast + 1;
    const StepCoef c = a.fine;
    const double* __restrict__ u = a.u;
    double prev[kResRows], cen[kResRows];
    double acc = 0.0;
    // the previous slice of the chunk's first step
    {
        const double* up0 = u + (i0 - 1) * a.n;
#pragma unroll
        for (int r = 0; r < kResRows; ++r) {
            const int y = y0 + r;
            prev[r] = (colok && y < ny) ? up0[(uint32_t)(y * nx + x)] : 0.0;
        }
    }
    for (int64_t i = i0; i <= i1; ++i) {
        const double* ui = u + i * a.n;
        double hu = 0.0, hd = 0.0, ew[kResRows], ee[kResRows];
#pragma unroll
        for (int r = 0; r < kResRows; ++r) {
            const int y = y0 + r;
            const bool ok = colok && y < ny;
            cen[r] = ok ? ui[(uint32_t)(y * nx + x)] : 0.0;
            ew[r] = (ok && load_w && xw >= 0) ? ui[(uint32_t)(y * nx + xw)] : 0.0;
            ee[r] = (ok && load_e && xe >= 0) ? ui[(uint32_t)(y * nx + xe)] : 0.0;
        }
        if (colok && y0 < ny) {
            if (yu >= 0) hu = ui[(uint32_t)(yu * nx + x)];
            if (yd >= 0) hd = ui[(uint32_t)(yd * nx + x)];
        }
#pragma unroll
        for (int r = 0; r < kResRows; ++r) {
            // every lane takes part in the shifts (their sources are all lanes of the wave)
            const double sw = wave_shift(cen[r], 0), se = wave_shift(cen[r], 1);
            const int y = y0 + r;
            if (colok && y < ny) {
                const double wv_ = load_w ? ew[r] : sw;
                const double ev_ = load_e ? ee[r] : se;
                const double nv = r == 0 ? hu : cen[r - 1];
                const double sv = y == ylast ? hd : cen[r + 1 < kResRows ? r + 1 : r];
                double rho = explicit_part(c, prev[r]) - stencil_value(c, nv, cen[r], sv, wv_, ev_);
                if (a.src) rho += a.dt * a.src[i * a.n + (uint32_t)(y * nx + x)];
                acc += rho * rho;
            }
            prev[r] = cen[r];
        }
    }
    double unused = 0.0;
    block_sum2(acc, unused, red, slot, kResidThreads / 64);
    if (threadIdx.x == 0) a.partials[w] = acc;
}

// Paper-form residual of the exact step, |r|^2 = sum_i |M^-1 rho_i|^2, i = 1..nt,
// one workgroup per interval (task N_T takes the ragged tail).  M r_i = rho_i is
// solved in FP64 by CG from zero to the fine tolerance relative to |rho_i|.
template <int S, bool EX, bool PER>
__global__ __launch_bounds__(kBlock2D) void step_residual2d_kernel(KArgs a)
{
    __shared__ __align__(16) double lp[Lds2D<double>::size];
    __shared__ double red[4 * kWaves2D];
    int slot = 0;
    const int64_t j = blockIdx.x;
    const Strip st = make_strip<double>(a.g);
    const int nx = a.g.nx;
    lds_clear(lp);
    const int64_t total = (j < a.NT) ? a.m : (a.nt - a.NT * a.m);
    double x[S], r[S], q[S];
    double acc = 0.0;
    long long its = 0;
    for (int64_t t = 1; t <= total; ++t) {
        const int64_t i = j * a.m + t;
        {
            const int64_t off = opaque_off(st.gbase);
#pragma unroll
            for (int s = 0; s < S; ++s)
                r[s] = row_ok<EX, S>(st, s) ? explicit_part(a.fine, a.u[(i - 1) * a.n + off + (int64_t)s * nx]) : 0.0;
        }
        {
            const int64_t off = opaque_off(st.gbase);
            const double* ui = a.u + i * a.n;
            lds_put_fn<double, S, EX, PER, false>(a.g, st, lp,
                                                  [&](int s, double) { return ui[off + (int64_t)s * nx]; });
        }
        __syncthreads();
        if (EX || st.nr > 0)
            strip_stencil<double, S, EX>(st, lp, [&](int s, double u_, double c_, double d_, double w_, double e_) {
                r[s] = r[s] - stencil_value(a.fine, u_, c_, d_, w_, e_);
                return r[s];
            });
        __syncthreads();  // the CG overwrites the staged slice
#pragma unroll
        for (int s = 0; s < S; ++s) x[s] = 0.0;
        its += cg2d<double, S, EX, PER, true>(a.g, a.fine, st, x, r, q, lp, red, slot, a.rtol2, a.maxit, a.fail);
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (row_ok<EX, S>(st, s)) acc += x[s] * x[s];
    }
    double unused = 0.0;
    block_sum2(acc, unused, red, slot, kWaves2D);
    if (threadIdx.x == 0) a.partials[j] = acc;
    count_cg(a, its);
}

// 1D form: M = tridiag(-c, 1 + 2c, -c) solved directly by PCR.
__global__ __launch_bounds__(1024) void step_residual1d_kernel(KArgs a)
{
    __shared__ double lds[3 * 1024];
    __shared__ double red[2 * 2 * 16];
    int slot = 0;
    const int64_t j = blockIdx.x;
    const int i = threadIdx.x;
    const int nx = a.nx;
    const bool act = i < nx;
    Pcr1D f;
    pcr_setup(f, nx, a.fine.cx, lds);
    const int64_t total = (j < a.NT) ? a.m : (a.nt - a.NT * a.m);
    const double c = a.fine.cx;
    double acc = 0.0;
    for (int64_t t = 1; t <= total; ++t) {
        const int64_t ti = j * a.m + t;
        double rho = 0.0;
        if (act) {
            const double* ui = a.u + ti * a.n;
            const double w = i > 0 ? ui[i - 1] : 0.0;
            const double e = i < nx - 1 ? ui[i + 1] : 0.0;
            rho = a.u[(ti - 1) * a.n + i] - (a.fine.d * ui[i] - c * (w + e));
            if (a.src) rho += a.dt * a.src[ti * a.n + i];
        }
        const double z = pcr_solve(f, nx, rho, lds);
        if (act) acc += z * z;
    }
    double unused = 0.0;
    block_sum2(acc, unused, red, slot, (int)(blockDim.x / 64));
    if (threadIdx.x == 0) a.partials[j] = acc;
}

// hdr->norm2 = sum of partials[0 .. count-1] in a fixed order
__global__ __launch_bounds__(256) void sum_partials_kernel(KArgs a, int64_t count)
{
    __shared__ double red[2 * 2 * 4];
    int slot = 0;
    double acc = 0.0, unused = 0.0;
    for (int64_t b = threadIdx.x; b < count; b += 256) acc += a.partials[b];
    block_sum2(acc, unused, red, slot, 4);
    if (threadIdx.x == 0) {
        a.hdr->norm2 = acc;
        publish_header(a);
    }
}

#define ATM_MIXED_S(kernel, S, EX, PER, grid, stream, a) \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(kernel<S, EX, PER>), dim3(grid), dim3(kBlock2D), 0, stream, a)

#define ATM_MIXED_EP(kernel, S, grid, stream, a)                                      \
    do {                                                                              \
        if ((a).exact) {                                                              \
            if ((a).g.periodic) ATM_MIXED_S(kernel, S, true, true, grid, stream, a);  \
            else ATM_MIXED_S(kernel, S, true, false, grid, stream, a);                \
        } else {                                                                      \
            if ((a).g.periodic) ATM_MIXED_S(kernel, S, false, true, grid, stream, a); \
            else ATM_MIXED_S(kernel, S, false, false, grid, stream, a);               \
        }                                                                             \
    } while (0)

#define ATM_MIXED_2D(kernel, grid, stream, a)                                \
    do {                                                                     \
        switch ((a).s_tmpl) {                                                \
            case 8: ATM_MIXED_EP(kernel, 8, grid, stream, a); break;         \
            case 16: ATM_MIXED_EP(kernel, 16, grid, stream, a); break;       \
            default: ATM_MIXED_EP(kernel, 32, grid, stream, a); break;       \
        }                                                                    \
    } while (0)

void launch_sweep_mixed(const KArgs& a, int64_t n_tasks, hipStream_t s)
{
    ATM_MIXED_2D(sweep2d_mixed_kernel, n_tasks, s, a);
}

namespace {
struct ResidGrid {
    int64_t ntile, chunk, units, blocks;
};
ResidGrid resid_grid(const KArgs& a)
{
    ResidGrid r;
    const int64_t ny = a.n / a.nx;
    r.ntile = ((a.nx + 63) / 64) * ((ny + kResTileRows - 1) / kResTileRows);
    int64_t nchunk = kResidBlocks / r.ntile;
    if (nchunk < 1) nchunk = 1;
    if (nchunk > a.nt) nchunk = a.nt;
    r.chunk = (a.nt + nchunk - 1) / nchunk;
    nchunk = (a.nt + r.chunk - 1) / r.chunk;
    r.units = r.ntile * nchunk;
    r.blocks = (r.units + 7) / 8 * 8;
    return r;
}
}  // namespace

int64_t implicit_residual_blocks(const KArgs& a) { return resid_grid(a).units; }

void launch_implicit_residual(const KArgs& a, hipStream_t s)
{
    const ResidGrid r = resid_grid(a);
    hipLaunchKernelGGL(implicit_residual_kernel, dim3(r.blocks), dim3(kResidThreads), 0, s, a, r.ntile, r.chunk,
                       r.units);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, a, r.units);
}

void launch_step_residual(const KArgs& a, int64_t n_tasks, hipStream_t s)
{
    if (a.is1d)
        hipLaunchKernelGGL(step_residual1d_kernel, dim3(n_tasks), dim3(((a.nx + 63) / 64) * 64), 0, s, a);
    else
        ATM_MIXED_2D(step_residual2d_kernel, n_tasks, s, a);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, a, n_tasks);
}

}  // namespace atm
