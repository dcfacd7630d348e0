// Batched AT-MGRIT: many independent instances (1D heat, 2D heat, 2D Allen-Cahn of
// uneven sizes) advance together, one cycle per replay of a captured hipGraph.
//
// Each phase of a cycle (CF relaxation, FAS right-hand side, windows, correction
// with F-interpolation, norm pieces, norm sums, decision) is one launch per
// instance class over a task table of (instance, interval / window / piece)
// records, ordered by the autotuner (for example longest task first); the
// hardware dispatcher hands the workgroups out in that order.  Every body is
// the one the single-instance kernels run, so a class's launch has that
// kernel's registers and LDS.  Instances whose decision has stopped them skip
// their tasks, so replays after convergence cost only empty launches.
#include "atm_batch.hpp"
#include "atm_bodies.hpp"
#include "atm_device.hpp"
#include "atm_kernels.hpp"

namespace atm {
namespace batch {

// Grids of at most 64 columns (64 threads along x) need 66 LDS columns: with
// 8-row strips such a workgroup fits twice on a CU (LDS and registers).
constexpr int kSmallCols = 64 + 2;

#define BATCH_TASK_PRELUDE                       \
    const Task t = tasks[blockIdx.x];            \
    if (!ctl[t.inst].active) return;             \
    const KArgs& a = args[t.inst];

__global__ __launch_bounds__(512) void sweep1d_batch(const KArgs* __restrict__ args, const Task* __restrict__ tasks,
                                                     const InstCtl* __restrict__ ctl)
{
    __shared__ double lds[3 * 1024];
    BATCH_TASK_PRELUDE
    sweep1d_body(a, t.idx, lds);
}

__global__ __launch_bounds__(512) void coarse1d_batch(const KArgs* __restrict__ args, const Task* __restrict__ tasks,
                                                      const InstCtl* __restrict__ ctl)
{
    __shared__ double lds[3 * 1024];
    BATCH_TASK_PRELUDE
    coarse1d_body(a, t.idx, lds);
}

template <int S, bool PER, bool SMALL>
__global__ __launch_bounds__(kBlock2D) void sweep2d_batch(const KArgs* __restrict__ args,
                                                          const Task* __restrict__ tasks,
                                                          const InstCtl* __restrict__ ctl)
{
    constexpr int COLS = SMALL ? kSmallCols : kMaxSide2D + 2;
    __shared__ __align__(16) double lds[COLS * Lds2D<double>::H];
    __shared__ double red[4 * kWaves2D];
    BATCH_TASK_PRELUDE
    sweep2d_mixed_body<S, false, PER, COLS>(a, t.idx, lds, red);
}

template <int S, bool PER, bool SMALL>
__global__ __launch_bounds__(kBlock2D) void sweep2d64_batch(const KArgs* __restrict__ args,
                                                            const Task* __restrict__ tasks,
                                                            const InstCtl* __restrict__ ctl)
{
    constexpr int COLS = SMALL ? kSmallCols : kMaxSide2D + 2;
    __shared__ __align__(16) double lds[COLS * Lds2D<double>::H];
    __shared__ double red[4 * kWaves2D];
    BATCH_TASK_PRELUDE
    sweep2d_body<S, false, PER, COLS>(a, t.idx, lds, red);
}

template <int S, bool PER, bool SMALL>
__global__ __launch_bounds__(kBlock2D) void coarse2d_batch(const KArgs* __restrict__ args,
                                                           const Task* __restrict__ tasks,
                                                           const InstCtl* __restrict__ ctl)
{
    constexpr int COLS = SMALL ? kSmallCols : kMaxSide2D + 2;
    __shared__ __align__(16) double lds[COLS * Lds2D<double>::H];
    __shared__ double red[4 * kWaves2D];
    BATCH_TASK_PRELUDE
    coarse2d_body<S, false, PER, COLS>(a, t.idx, lds, red);
}

template <int S, bool PER, bool SMALL>
__global__ __launch_bounds__(kBlock2D) void coarse2d_spec_batch(const KArgs* __restrict__ args,
                                                           const Task* __restrict__ tasks,
                                                           const InstCtl* __restrict__ ctl)
{
    constexpr int COLS = SMALL ? kSmallCols : kMaxSide2D + 2;
    __shared__ __align__(16) double lds[COLS * Lds2D<double>::H];
    __shared__ double red[4 * kWaves2D];
    BATCH_TASK_PRELUDE
    coarse2d_body<S, false, PER, COLS, true>(a, t.idx, lds, red);
}

// windows with Psi on the BF16 matrix cores; the batch forms no residual rows, so each window step reads
// r = y - u after its products
template <int S, bool PER, bool SMALL>
__global__ __launch_bounds__(kBlock2D) void coarse2d_bf_batch(const KArgs* __restrict__ args,
                                                         const Task* __restrict__ tasks,
                                                         const InstCtl* __restrict__ ctl)
{
    constexpr int COLS = SMALL ? kSmallCols : kMaxSide2D + 2;
    __shared__ __align__(16) double lds[COLS * Lds2D<double>::H];
    __shared__ double red[4 * kWaves2D];
    BATCH_TASK_PRELUDE
    coarse2d_body<S, false, PER, COLS, false, true, false, false>(a, t.idx, lds, red);
}

template <int S, bool PER, bool SMALL>
__global__ __launch_bounds__(kBlock2D) void coarse2d_bf_fas_batch(const KArgs* __restrict__ args,
                                                             const Task* __restrict__ tasks,
                                                             const InstCtl* __restrict__ ctl)
{
    constexpr int COLS = SMALL ? kSmallCols : kMaxSide2D + 2;
    __shared__ __align__(16) double lds[COLS * Lds2D<double>::H];
    __shared__ double red[4 * kWaves2D];
    BATCH_TASK_PRELUDE
    coarse2d_body<S, false, PER, COLS, false, true, false, true>(a, t.idx, lds, red);
}

template <int S, bool PER, bool SMALL>
__global__ __launch_bounds__(kBlock2D) void tau2d_batch(const KArgs* __restrict__ args, const Task* __restrict__ tasks,
                                                        const InstCtl* __restrict__ ctl)
{
    constexpr int COLS = SMALL ? kSmallCols : kMaxSide2D + 2;
    __shared__ __align__(16) double lds[COLS * Lds2D<double>::H];
    __shared__ double red[4 * kWaves2D];
    BATCH_TASK_PRELUDE
    tau2d_body<S, false, PER, COLS>(a, t.idx, lds, red);
}

template <int S, bool PER, bool SMALL>
__global__ __launch_bounds__(kBlock2D) void tau2d_spec_batch(const KArgs* __restrict__ args, const Task* __restrict__ tasks,
                                                        const InstCtl* __restrict__ ctl)
{
    constexpr int COLS = SMALL ? kSmallCols : kMaxSide2D + 2;
    __shared__ __align__(16) double lds[COLS * Lds2D<double>::H];
    __shared__ double red[4 * kWaves2D];
    BATCH_TASK_PRELUDE
    tau2d_body<S, false, PER, COLS, true>(a, t.idx, lds, red);
}

constexpr int kNormThreads = 256;

// C-point residual piece: partials[j] = ||y_j - u_{jm}||^2
__global__ __launch_bounds__(kNormThreads) void normc_batch(const KArgs* __restrict__ args,
                                                            const Task* __restrict__ tasks,
                                                            const InstCtl* __restrict__ ctl)
{
    __shared__ double red[2 * 2 * (kNormThreads / 64)];
    BATCH_TASK_PRELUDE
    int slot = 0;
    const int64_t j = t.idx;
    double acc = 0.0, unused = 0.0;
    for (int64_t i = threadIdx.x; i < a.n; i += kNormThreads) {
        const double r = a.y[j * a.n + i] - a.u[(j * a.m) * a.n + i];
        acc += r * r;
    }
    block_sum2(acc, unused, red, slot, kNormThreads / 64);
    if (threadIdx.x == 0) a.partials[j] = acc;
}

// implicit residual piece over the steps of chunk c (of nchunk[inst]): partials[c]
__global__ __launch_bounds__(kNormThreads) void normi_batch(const KArgs* __restrict__ args,
                                                            const Task* __restrict__ tasks,
                                                            const InstCtl* __restrict__ ctl,
                                                            const int* __restrict__ nchunk)
{
    __shared__ double red[2 * 2 * (kNormThreads / 64)];
    BATCH_TASK_PRELUDE
    int slot = 0;
    const int64_t c = t.idx;
    const int64_t nc = nchunk[t.inst];
    const int64_t chunk = (a.nt + nc - 1) / nc;
    const int64_t i0 = 1 + c * chunk;
    const int64_t i1 = (i0 + chunk - 1 < a.nt) ? i0 + chunk - 1 : a.nt;
    const int nx = a.g.nx, ny = a.g.ny;
    const bool per = a.g.periodic != 0;
    double acc = 0.0;
    for (int64_t idx = threadIdx.x; idx < a.n; idx += kNormThreads) {
        const int x = (int)(idx % nx), y = (int)(idx / nx);
        const int64_t ow = x > 0 ? idx - 1 : (per ? idx + nx - 1 : -1);
        const int64_t oe = x < nx - 1 ? idx + 1 : (per ? idx - (nx - 1) : -1);
        const int64_t on = y > 0 ? idx - nx : (per ? idx + (int64_t)(ny - 1) * nx : -1);
        const int64_t os = y < ny - 1 ? idx + nx : (per ? idx - (int64_t)(ny - 1) * nx : -1);
        double prev = i0 <= i1 ? a.u[(i0 - 1) * a.n + idx] : 0.0;
        for (int64_t i = i0; i <= i1; ++i) {
            const double* ui = a.u + i * a.n;
            const double cen = ui[idx];
            const double wv = ow >= 0 ? ui[ow] : 0.0;
            const double ev = oe >= 0 ? ui[oe] : 0.0;
            const double nv = on >= 0 ? ui[on] : 0.0;
            const double sv = os >= 0 ? ui[os] : 0.0;
            const double rho = explicit_part(a.fine, prev) - stencil_value(a.fine, nv, cen, sv, wv, ev);
            acc += rho * rho;
            prev = cen;
        }
    }
    double unused = 0.0;
    block_sum2(acc, unused, red, slot, kNormThreads / 64);
    if (threadIdx.x == 0) a.partials[c] = acc;
}

// hdr->norm2 = sum of partials[first .. first + count) in a fixed order (task idx = count, first from the body)
__global__ __launch_bounds__(kNormThreads) void normf_batch(const KArgs* __restrict__ args,
                                                            const Task* __restrict__ tasks,
                                                            const InstCtl* __restrict__ ctl, int first_is_one,
                                                            const int* __restrict__ nchunk)
{
    __shared__ double red[2 * 2 * (kNormThreads / 64)];
    BATCH_TASK_PRELUDE
    int slot = 0;
    const int64_t first = first_is_one ? 1 : 0;
    const int64_t count = first_is_one ? a.NT : nchunk[t.inst];
    double acc = 0.0, unused = 0.0;
    for (int64_t b = first + threadIdx.x; b < first + count; b += kNormThreads) acc += a.partials[b];
    block_sum2(acc, unused, red, slot, kNormThreads / 64);
    if (threadIdx.x == 0) a.hdr->norm2 = acc;
}

__global__ void decide_batch(const KArgs* __restrict__ args, InstCtl* ctl, double* hist, int hist_cap, int n_inst,
                             int first)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst || !ctl[i].active) return;
    const Header* h = args[i].hdr;
    const double res = sqrt(h->norm2);
    const int it = first ? 0 : ctl[i].it + 1;
    ctl[i].it = it;
    ctl[i].res = res;
    if (hist && it < hist_cap) hist[(int64_t)i * hist_cap + it] = res;
    int active = 0;
    if (h->fail)
        ctl[i].status = kStInner;
    else if (!(res == res) || res > 1e300)
        ctl[i].status = kStDiverged;
    else if (res <= ctl[i].tol)
        ctl[i].status = kStOk;
    else if (it >= ctl[i].max_iter)
        ctl[i].status = kStNotConverged;
    else
        active = 1;
    ctl[i].active = active;
}

__global__ void reset_headers_batch(const KArgs* __restrict__ args, InstCtl* ctl, int n_inst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    Header* h = args[i].hdr;
    h->norm2 = 0.0;
    h->fail = 0;
    h->cg_fine = 0ull;
    h->cg_coarse = 0ull;
    h->skipped = 0ull;
    ctl[i].active = 1;
    ctl[i].it = 0;
    ctl[i].status = kStNotConverged;
    ctl[i].res = 0.0;
}

#define BATCH_S(kernel, PER, l, s)                                                                              \
    do {                                                                                                        \
        switch (S) {                                                                                            \
            case 8:                                                                                             \
                if (small)                                                                                      \
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(kernel<8, PER, true>), dim3(l.ntasks), dim3(kBlock2D), 0, \
                                       s, l.args, l.tasks, l.ctl);                                              \
                else                                                                                            \
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(kernel<8, PER, false>), dim3(l.ntasks), dim3(kBlock2D), 0, \
                                       s, l.args, l.tasks, l.ctl);                                              \
                break;                                                                                          \
            case 16:                                                                                            \
                hipLaunchKernelGGL(HIP_KERNEL_NAME(kernel<16, PER, false>), dim3(l.ntasks), dim3(kBlock2D), 0, s, \
                                   l.args, l.tasks, l.ctl);                                                     \
                break;                                                                                          \
            default:                                                                                            \
                hipLaunchKernelGGL(HIP_KERNEL_NAME(kernel<32, PER, false>), dim3(l.ntasks), dim3(kBlock2D), 0, s, \
                                   l.args, l.tasks, l.ctl);                                                     \
                break;                                                                                          \
        }                                                                                                       \
    } while (0)

#define BATCH_SP(kernel, l, s)                   \
    do {                                         \
        if (per)                                 \
            BATCH_S(kernel, true, l, s);         \
        else                                     \
            BATCH_S(kernel, false, l, s);        \
    } while (0)

void launch_tasks(Body body, int S, bool per, bool small, const Launch& l, hipStream_t s)
{
    if (l.ntasks <= 0) return;
    switch (body) {
        case kSweep1D:
            hipLaunchKernelGGL(sweep1d_batch, dim3(l.ntasks), dim3(512), 0, s, l.args, l.tasks, l.ctl);
            break;
        case kCoarse1D:
            hipLaunchKernelGGL(coarse1d_batch, dim3(l.ntasks), dim3(512), 0, s, l.args, l.tasks, l.ctl);
            break;
        case kSweep2D: BATCH_SP(sweep2d_batch, l, s); break;
        case kSweep2D64: BATCH_SP(sweep2d64_batch, l, s); break;
        case kCoarse2D: BATCH_SP(coarse2d_batch, l, s); break;
        case kTau2D: BATCH_SP(tau2d_batch, l, s); break;
        case kCoarse2DSpec: BATCH_SP(coarse2d_spec_batch, l, s); break;
        case kTau2DSpec: BATCH_SP(tau2d_spec_batch, l, s); break;
        case kCoarse2DBf: BATCH_SP(coarse2d_bf_batch, l, s); break;
        case kCoarse2DBfFas: BATCH_SP(coarse2d_bf_fas_batch, l, s); break;
        case kNormC:
            hipLaunchKernelGGL(normc_batch, dim3(l.ntasks), dim3(kNormThreads), 0, s, l.args, l.tasks, l.ctl);
            break;
        case kNormI:
            hipLaunchKernelGGL(normi_batch, dim3(l.ntasks), dim3(kNormThreads), 0, s, l.args, l.tasks, l.ctl,
                               l.nchunk);
            break;
        case kNormFinalC:
            hipLaunchKernelGGL(normf_batch, dim3(l.ntasks), dim3(kNormThreads), 0, s, l.args, l.tasks, l.ctl, 1,
                               l.nchunk);
            break;
        case kNormFinalI:
            hipLaunchKernelGGL(normf_batch, dim3(l.ntasks), dim3(kNormThreads), 0, s, l.args, l.tasks, l.ctl, 0,
                               l.nchunk);
            break;
    }
}

void launch_decide(const KArgs* args, InstCtl* ctl, double* hist, int hist_cap, int n_inst, bool first, hipStream_t s)
{
    hipLaunchKernelGGL(decide_batch, dim3((n_inst + 63) / 64), dim3(64), 0, s, args, ctl, hist, hist_cap, n_inst,
                       first ? 1 : 0);
}

void launch_reset_headers(const KArgs* args, InstCtl* ctl, int n_inst, hipStream_t s)
{
    hipLaunchKernelGGL(reset_headers_batch, dim3((n_inst + 63) / 64), dim3(64), 0, s, args, ctl, n_inst);
}

}  // namespace batch
}  // namespace atm
