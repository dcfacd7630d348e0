// Kernel argument block and launcher declarations shared by the host API and
// the kernel translation unit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "atm_device.hpp"

namespace atm {

// Small device-side header at the start of the workspace.
struct Header {
    double norm2;                  // last residual sum of squares
    int fail;                      // CG failure flag (sticky until reset)
    int pad;
    unsigned long long cg_fine;    // CG iterations inside Phi since the last reset
    unsigned long long cg_coarse;  // CG iterations inside Psi since the last reset
    unsigned long long skipped;    // fine steps not recomputed by sweeps with an unchanged C-point
};

struct KArgs {
    // space-time data
    double* u;          // [nt+1][n]
    const double* aux;  // sweep modes 1 (e) and 2 (y of the previous sweep)
    double* y;          // sweep: out; coarse/tau/norm: in (Phi of the last F-point)
    double* e;          // coarse: out
    double* tau;        // FAS right-hand side, [N_T+1][n]
    double* partials;   // [max(N_T+1, kResidBlocks)] partial sums of norms
    Header* hdr;
    Header* hdr_host;   // nullable: pinned host copy of the header, written by the kernel that ends a norm
    int* fail;
    unsigned long long* cg_count;
    // sizes
    int64_t nt, n, NT;
    int m, k, mode, fas, substeps, nx;
    int is1d, s_tmpl, exact;
    // PDE source b(x, t_i), [nt+1][n] (1D heat), or null: every fine step adds dt b(t_i) to its
    // right-hand side
    const double* src;
    double dt;
    // levels below the finest (the multilevel V-cycle): each fine step is fine_substeps steps with
    // the coefficients `fine`, and gadd [nt+1][n] (the level's FAS right-hand side) is added after
    // it: u_i = Phi(u_{i-1}) + gadd_i.  fine_substeps = 1 and gadd = null on the finest level.
    const double* gadd;
    int fine_substeps;
    // FAS right-hand-side kernels: 1 writes y_j = Psi(u_{(j-1)m}) instead of tau_j, so that the
    // window kernels see the coarse residual y_j - u_{jm} of the injected iterate (nested iteration)
    int psi_only;
    Grid2D g;
    StepCoef fine, coarse;
    double rtol2;         // squared CG tolerance of Phi
    double rtol2_coarse;  // squared CG tolerance of Psi
    double rtol2_mixed;   // squared tolerance of the FP32 CG of the mixed-precision sweeps
    int maxit;
    // FP64 sweeps inside a solve: an interval whose starting C-value equals the stored u_{jm}
    // bit for bit keeps its F-points (they are the relaxation of that value from the previous
    // sweep) and only provides y_{j+1}, copied from skip_y_src when that is not y itself
    int skip_unchanged;
    const double* skip_y_src;
    // grids beyond the on-chip strip layout: vectors of the step solves in a per-task scratch
    // (five n-vectors of doubles per interval or window)
    int large;
    double* large_scratch;
    // Psi's implicit solve in the eigenbasis of the constant-coefficient operator (large grids):
    // tables Qx [nx][nx], Qx^T, Qy [ny][ny], Qy^T and the mode factors ex [nx], ey [ny] of the coarse
    // step, built on the device before the windows
    int spectral;
    double* spec;
    // spectral 2: the C-point residuals r_j = y_j - u_{jm} (r_0 = 0), [N_T+1][n], formed once per
    // coarse solve so that each window step reads one row (grids up to 128 per side)
    double* cres;
    // spectral 2 on the paired large-grid windows, FAS form with s > 1 substeps: v_{j-1} carried
    // through Psi's first s - 1 substeps (the BF16 eigenbasis solve, stored in FP32), [N_T][s - 1][n]
    // (entry (j - 1, q - 1): q substeps from the C-point u_{(j-1)m})
    float* traj;
};

// ---------------------------------------------------------------------------
// shared helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ double cpoint_residual(const KArgs& a, int64_t j, int64_t idx)
{
    // r_0 = g_0 - u_0 = 0 (u_0 is never modified); r_j = Phi(u_{jm-1}) - u_{jm}
    if (j == 0) return 0.0;
    return a.y[j * a.n + idx] - a.u[(j * a.m) * a.n + idx];
}

// C-point value that starts interval j of a sweep
__device__ __forceinline__ double sweep_start(const KArgs& a, int64_t j, int64_t idx)
{
    const double uc = a.u[(j * a.m) * a.n + idx];
    if (a.mode == 1) return uc + a.aux[j * a.n + idx];
    if (a.mode == 2) return j == 0 ? uc : a.aux[j * a.n + idx];
    return uc;
}

// The kernel that ends a norm (thread 0, after writing norm2) copies the header into the caller's
// pinned host buffer with system-scope stores, so that the host reads it after synchronising without
// a separate copy.
__device__ __forceinline__ void publish_header(const KArgs& a)
{
    if (!a.hdr_host) return;
    const Header h = *a.hdr;
    __hip_atomic_store(&a.hdr_host->norm2, h.norm2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&a.hdr_host->fail, h.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&a.hdr_host->cg_fine, h.cg_fine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&a.hdr_host->cg_coarse, h.cg_coarse, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&a.hdr_host->skipped, h.skipped, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void count_cg(const KArgs& a, long long its)
{
    if (threadIdx.x == 0 && its) atomicAdd(a.cg_count, (unsigned long long)its);
}

// Interval j of a skipped sweep: provide y_{j+1} and count its steps.
__device__ __forceinline__ void skip_interval(const KArgs& a, int64_t j, int64_t total, int64_t idx0, int64_t stride,
                                              int64_t count)
{
    if (a.skip_y_src && j < a.NT)
        for (int64_t q = 0; q < count; ++q) {
            const int64_t idx = idx0 + q * stride;
            a.y[(j + 1) * a.n + idx] = a.skip_y_src[(j + 1) * a.n + idx];
        }
    if (threadIdx.x == 0 && total > 0) atomicAdd(&a.hdr->skipped, (unsigned long long)total);
}

// Explicit part of a step: psi(v) = v for heat, v + dt (v - v^3) / eps^2 for
// Allen-Cahn (the right-hand side of the implicit solve M x = psi(v)).
__device__ __forceinline__ double explicit_part(const StepCoef& c, double v)
{
    return c.react != 0.0 ? v + c.react * (v - v * v * v) : v;
}

// Strip offsets in global memory pass through an empty asm at every use, so
// the compiler recomputes the per-row addresses instead of hoisting all of
// them out of the time loop (which would cost a register pair per row).
__device__ __forceinline__ int64_t opaque_off(int v)
{
    __asm__ volatile("" : "+v"(v));
    return (int64_t)v;
}

template <int S, bool EX>
__device__ __forceinline__ void strip_store(double* dst, const Strip& st, int nx, const double (&v)[S])
{
    const int64_t off = opaque_off(st.gbase);
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (row_ok<EX, S>(st, s)) dst[off + (int64_t)s * nx] = v[s];
}

// the message returned by atm_last_error() on this thread
void set_last_error(const char* msg);

void launch_reset(Header* h, hipStream_t s);
void launch_sweep(const KArgs& a, int64_t n_tasks, hipStream_t s);
void launch_tau(const KArgs& a, hipStream_t s);
void launch_coarse(const KArgs& a, hipStream_t s);
void launch_norm(const KArgs& a, hipStream_t s);
void launch_sequential(const KArgs& a, hipStream_t s);
void launch_gather(const double* src, double* dst, int64_t n, int64_t stride_rows, int64_t rows, hipStream_t s);
void launch_cpoint_residuals(const KArgs& a, hipStream_t s);

// mixed-precision form (atm_mixed.hip)
constexpr int64_t kResidBlocks = 2048;  // most workgroups of the implicit-residual kernel
int64_t implicit_residual_blocks(const KArgs& a);
void launch_sweep_mixed(const KArgs& a, int64_t n_tasks, hipStream_t s);
void launch_implicit_residual(const KArgs& a, hipStream_t s);
void launch_step_residual(const KArgs& a, int64_t n_tasks, hipStream_t s);

// large 2D grids (atm_large.hip)
constexpr int kMaxSideLarge = 1024;
hipError_t launch_sweep_large(const KArgs& a, int64_t n_tasks, bool mixed, hipStream_t s);
// FP32-fine sweeps of the large grids on two CUs per interval (atm_pair.hip): the number of
// workgroup pairs for this grid and workspace (0 if the pair kernel does not take it), and the
// cooperative launch.  Header::fail bit 2 marks a pair whose partner did not arrive.
constexpr int kFailPairTimeout = 2;

// The FP32 defect-correction steps take no correction for a defect rho = psi(v_{t-1}) - M s_t with
// |rho| <= 4 eps (1 + 2 d) |psi(v_{t-1})| (eps = 2^-53, d the step operator's diagonal): the terms of
// its FP64 evaluation add up to about (1 + 2 d) |v| per point, so such a defect is of the order of
// that evaluation's own rounding, and d = 0 is as good as any FP32 solve of it.
__host__ __device__ inline double defect_floor2(const StepCoef& c)
{
    const double f = 4.0 * 1.1102230246251565e-16 * (1.0 + 2.0 * c.d);
    return f * f;
}
int sweep_pair_pairs(const KArgs& a, int64_t n_tasks);
// workgroups of threads threads of kernel fn resident at once on the current device (0 if unknown)
int resident_blocks(const void* fn, int threads);
hipError_t launch_sweep_pair(const KArgs& a, int pairs, hipStream_t s);
// the windows (and FAS right-hand sides) of the large grids; with the eigenbasis Psi on grids of
// 128 .. 256 columns they run on two CUs per window (cooperative launch)
hipError_t launch_coarse_large(const KArgs& a, hipStream_t s);
int coarse_pair_pairs(const KArgs& a);  // workgroup pairs of the paired window kernels (0: not taken)
// doubles of the eigenbasis tables of an nx x ny grid (KArgs::spec), and their construction
size_t spectral_table_doubles(int nx, int ny);
size_t spectral_bf16_doubles(int nx, int ny);
void launch_spectral_tables(const KArgs& a, hipStream_t s);
void launch_sequential_large(const KArgs& a, hipStream_t s);
void launch_step_residual_large(const KArgs& a, int64_t n_tasks, hipStream_t s);

}  // namespace atm
