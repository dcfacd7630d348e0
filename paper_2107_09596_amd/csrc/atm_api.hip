// Host side of libatmgrit.so: argument validation, workspace layout, launch
// sequencing of the two-level AT-MGRIT cycle (Alg. 1) and the C-ABI.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <string>

#include "../../include/atm.h"
#include "atm_cnn.hpp"
#include "atm_kernels.hpp"

namespace {

thread_local std::string g_last_error;

}  // namespace

void atm::set_last_error(const char* msg) { g_last_error = msg; }

namespace {

atm_status fail(atm_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
atm_status fail(atm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define ATM_HIP(call)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return fail(ATM_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr double kMixedRtolDefault = 1e-6;  // FP32 CG tolerance of the mixed sweeps
constexpr double kLearnedGrowthLimit = 1e6;  // learned coarse solve: give up beyond this growth of the residual
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t header, partials, ya, yb, e, tau, pk, d1, d2, large, total;
};

int64_t n_intervals(const atm_problem* p, const atm_options* o) { return p->nt / o->m; }
int64_t n_space(const atm_problem* p) { return (int64_t)p->nx * p->ny; }

// 2D grids beyond the on-chip strip layout run the global-scratch kernels
bool large_grid(const atm_problem* p)
{
    return p->kind != ATM_HEAT1D && (p->nx > atm::kMaxSide2D || p->ny > atm::kMaxSide2D);
}

// the plain coarse propagator's form (coarse_form 3 falls back to the automatic choice)
bool use_fas(const atm_problem* p, const atm_options* o)
{
    if (o->coarse_form == 1) return false;
    if (o->coarse_form == 2) return true;
    return p->kind == ATM_AC2D;
}

bool learned(const atm_options* o) { return o->coarse_form == 3; }

Layout layout(const atm_problem* p, const atm_options* o)
{
    const size_t NT = (size_t)n_intervals(p, o);
    const size_t slab = (NT + 1) * (size_t)n_space(p) * sizeof(double);
    Layout L;
    size_t off = 0;
    L.header = off;
    off += align_up(sizeof(atm::Header));
    L.partials = off;
    off += align_up((NT + 1 > (size_t)atm::kResidBlocks ? NT + 1 : (size_t)atm::kResidBlocks) * sizeof(double));
    L.ya = off;
    off += align_up(slab);
    L.yb = off;
    off += align_up(slab);
    L.e = off;
    off += align_up(slab);
    L.tau = off;
    off += use_fas(p, o) ? align_up(slab) : 0;
    // learned coarse solve: BF16 weights and two BF16 activation buffers for N_T + 1 fields
    const size_t act = learned(o) ? (size_t)n_space(p) * atm::cnn::C * 2 : 0;
    L.pk = off;
    off += learned(o) ? align_up(atm::cnn::PK_N * 2) : 0;
    L.d1 = off;
    off += align_up((NT + 1) * act);
    L.d2 = off;
    off += align_up((NT + 1) * act);
    L.large = off;
    off += large_grid(p) ? align_up((NT + 1) * 5 * (size_t)n_space(p) * sizeof(double)) : 0;
    L.total = off;
    return L;
}

atm_status validate(const atm_problem* p, const atm_options* o)
{
    if (!p || !o) return fail(ATM_ERR_INVALID_ARG, "null problem or options");
    if (p->kind != ATM_HEAT1D && p->kind != ATM_HEAT2D && p->kind != ATM_AC2D)
        return fail(ATM_ERR_INVALID_ARG, "unknown problem kind %d", p->kind);
    if (p->nx < 1 || p->ny < 1) return fail(ATM_ERR_INVALID_ARG, "nx, ny must be >= 1");
    if (p->kind == ATM_HEAT1D && p->ny != 1) return fail(ATM_ERR_INVALID_ARG, "ATM_HEAT1D needs ny == 1");
    if (!(p->length > 0.0) || !(p->nu > 0.0)) return fail(ATM_ERR_INVALID_ARG, "length and nu must be > 0");
    if (p->kind == ATM_AC2D && !(p->eps > 0.0)) return fail(ATM_ERR_INVALID_ARG, "eps must be > 0");
    if (!(p->tf > p->t0)) return fail(ATM_ERR_INVALID_ARG, "tf must exceed t0");
    if (p->nt < 1) return fail(ATM_ERR_INVALID_ARG, "nt must be >= 1");
    if (p->kind != ATM_HEAT1D && (!(p->cg_rtol >= 0.0) || p->cg_max_iter < 1))
        return fail(ATM_ERR_INVALID_ARG, "cg_rtol must be >= 0 and cg_max_iter >= 1");
    if (o->m < 2) return fail(ATM_ERR_INVALID_ARG, "coarsening factor m must be >= 2");
    if (p->nt < o->m) return fail(ATM_ERR_INVALID_ARG, "nt (%lld) must be >= m (%d)", (long long)p->nt, o->m);
    if (o->k < 1) return fail(ATM_ERR_INVALID_ARG, "k must be >= 1");
    if (o->relax != 0 && o->relax != 1) return fail(ATM_ERR_INVALID_ARG, "relax must be 0 (F) or 1 (FCF)");
    if (o->coarse_substeps < 1) return fail(ATM_ERR_INVALID_ARG, "coarse_substeps must be >= 1");
    if (o->coarse_form < 0 || o->coarse_form > 3) return fail(ATM_ERR_INVALID_ARG, "coarse_form must be 0, 1, 2 or 3");
    if (o->coarse_form == 3) {
        if (p->kind != ATM_AC2D)
            return fail(ATM_ERR_UNSUPPORTED, "the learned coarse propagator is built for the periodic ATM_AC2D grid");
        if (p->nx % 16 != 0 || p->nx > 128)
            return fail(ATM_ERR_UNSUPPORTED, "the learned coarse propagator needs nx a multiple of 16, at most 128");
        if (!o->cnn_params) return fail(ATM_ERR_INVALID_ARG, "coarse_form 3 needs cnn_params");
        if (!(o->fallback_ratio >= 0.0)) return fail(ATM_ERR_INVALID_ARG, "fallback_ratio must be >= 0");
    }
    if (o->max_iter < 0) return fail(ATM_ERR_INVALID_ARG, "max_iter must be >= 0");
    if (!(o->tol >= 0.0)) return fail(ATM_ERR_INVALID_ARG, "tol must be >= 0");
    if (o->precision != 0 && o->precision != 1) return fail(ATM_ERR_INVALID_ARG, "precision must be 0 or 1");
    if (o->precision == 1 && p->kind == ATM_HEAT1D)
        return fail(ATM_ERR_UNSUPPORTED, "precision 1 (FP32 fine solves) is available for the 2D kinds only");
    if (!(o->mixed_cg_rtol >= 0.0) || !(o->mixed_cg_rtol < 1.0))
        return fail(ATM_ERR_INVALID_ARG, "mixed_cg_rtol must be in [0, 1)");
    if (!(o->coarse_cg_rtol >= 0.0)) return fail(ATM_ERR_INVALID_ARG, "coarse_cg_rtol must be >= 0");
    if (o->profile != 0 && o->profile != 1) return fail(ATM_ERR_INVALID_ARG, "profile must be 0 or 1");
    if (p->kind == ATM_HEAT1D) {
        if (p->nx > 1024) return fail(ATM_ERR_UNSUPPORTED, "1D grids are limited to nx <= 1024");
    } else {
        if (p->nx > atm::kMaxSideLarge)
            return fail(ATM_ERR_UNSUPPORTED, "2D grids are limited to %d points per row", atm::kMaxSideLarge);
        if (p->kind == ATM_AC2D && (p->nx < 3 || p->ny < 3))
            return fail(ATM_ERR_UNSUPPORTED, "periodic grids need at least 3 points per side");
    }
    return ATM_OK;
}

atm::StepCoef step_coef(const atm_problem* p, double dt)
{
    atm::StepCoef c;
    const bool per = (p->kind == ATM_AC2D);
    const double hx = per ? p->length / p->nx : p->length / (p->nx + 1);
    const double hy = per ? p->length / p->ny : p->length / (p->ny + 1);
    c.cx = p->nu * dt / (hx * hx);
    c.cy = (p->kind == ATM_HEAT1D) ? 0.0 : p->nu * dt / (hy * hy);
    c.d = 1.0 + 2.0 * c.cx + 2.0 * c.cy;
    c.inv_d = 1.0 / c.d;
    c.react = (p->kind == ATM_AC2D) ? dt / (p->eps * p->eps) : 0.0;
    return c;
}

// Fill the kernel argument block for a workspace (or NULL for size-only).
atm_status make_args(const atm_problem* p, const atm_options* o, void* ws, size_t ws_bytes, atm::KArgs& a)
{
    atm_status st = validate(p, o);
    if (st) return st;
    const Layout L = layout(p, o);
    if (ws_bytes < L.total)
        return fail(ATM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, L.total);
    if (!ws) return fail(ATM_ERR_INVALID_ARG, "null workspace");
    if (((uintptr_t)ws) % kAlign) return fail(ATM_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
    memset(&a, 0, sizeof(a));
    char* base = (char*)ws;
    a.hdr = (atm::Header*)(base + L.header);
    a.fail = &a.hdr->fail;
    a.cg_count = &a.hdr->cg_fine;
    a.partials = (double*)(base + L.partials);
    a.tau = use_fas(p, o) ? (double*)(base + L.tau) : nullptr;
    a.nt = p->nt;
    a.n = n_space(p);
    a.NT = n_intervals(p, o);
    a.m = o->m;
    a.k = o->k;
    a.fas = use_fas(p, o) ? 1 : 0;
    a.substeps = o->coarse_substeps;
    a.nx = p->nx;
    a.is1d = (p->kind == ATM_HEAT1D);
    const double dt = (p->tf - p->t0) / (double)p->nt;
    a.fine = step_coef(p, dt);
    a.coarse = step_coef(p, dt * o->m / o->coarse_substeps);
    a.rtol2 = p->cg_rtol * p->cg_rtol;
    const double crtol = o->coarse_cg_rtol > 0.0 ? o->coarse_cg_rtol : p->cg_rtol;
    a.rtol2_coarse = crtol * crtol;
    const double mrtol = o->mixed_cg_rtol > 0.0 ? o->mixed_cg_rtol : kMixedRtolDefault;
    a.rtol2_mixed = mrtol * mrtol;
    a.maxit = p->cg_max_iter;
    if (large_grid(p)) {
        a.large = 1;
        a.large_scratch = (double*)(base + L.large);
        a.g.nx = p->nx;
        a.g.ny = p->ny;
        a.g.periodic = (p->kind == ATM_AC2D);
    } else if (!a.is1d) {
        // strips: TX = 64 or 128 threads along x, TY = 512 / TX strips along y,
        // rows a multiple of 2 (16-byte LDS accesses of doubles), of 4 for the
        // mixed-precision sweeps (16-byte accesses of floats)
        const int tx_log2 = p->nx > 64 ? 7 : 6;
        const int TX = 1 << tx_log2;
        const int TY = atm::kBlock2D / TX;
        const int chunk = o->precision == 1 ? 4 : 2;
        int rows = (p->ny + TY - 1) / TY;
        rows = (rows + chunk - 1) / chunk * chunk;
        a.g.nx = p->nx;
        a.g.ny = p->ny;
        a.g.tx_log2 = tx_log2;
        a.g.rows = rows;
        a.g.periodic = (p->kind == ATM_AC2D);
        a.s_tmpl = rows <= 8 ? 8 : (rows <= 16 ? 16 : 32);
        if (rows > 32) return fail(ATM_ERR_UNSUPPORTED, "grid needs %d rows per strip (max 32)", rows);
        a.exact = (p->nx == TX && rows * TY == p->ny && rows == a.s_tmpl) ? 1 : 0;
        // Every LDS access of a strip stays inside its own column of H values:
        // the deepest strip that owns rows starts at y0_last and touches column
        // indices up to y0_last + V + S (the value below its last row).
        const int H = atm::Lds2D<double>::H, V = atm::Lds2D<double>::V;
        const int y0_last = ((p->ny - 1) / rows) * rows;
        const int Hf = atm::Lds2D<float>::H, Vf = atm::Lds2D<float>::V;
        if (y0_last + V + a.s_tmpl >= H || y0_last + Vf + a.s_tmpl >= Hf || p->nx + 2 > atm::kMaxSide2D + 2)
            return fail(ATM_ERR_UNSUPPORTED, "grid %d x %d does not fit the LDS strip layout", p->nx, p->ny);
    }
    return ATM_OK;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

atm_status check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ATM_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    return ATM_OK;
}

// Intervals 0..N_T-1 plus task N_T, which owns C-point N_T (its correction and
// C-relaxation) and the F-points of a ragged tail after it (none when m | nt).
int64_t sweep_tasks(const atm_problem* p, const atm_options* o) { return n_intervals(p, o) + 1; }

// Read back the header (norm, failure flag, CG count) after synchronising.
atm_status read_header(const atm::KArgs& a, hipStream_t s, atm::Header* out)
{
    ATM_HIP(hipMemcpyAsync(out, a.hdr, sizeof(atm::Header), hipMemcpyDeviceToHost, s));
    ATM_HIP(hipStreamSynchronize(s));
    return ATM_OK;
}

atm_status do_sweep(atm::KArgs a, const atm_problem* p, const atm_options* o, int mode, double* u, const double* aux,
                    double* y, hipStream_t s, bool skip_unchanged = false, const double* skip_y_src = nullptr)
{
    a.mode = mode;
    a.skip_unchanged = skip_unchanged ? 1 : 0;
    a.skip_y_src = skip_y_src;
    a.u = u;
    a.aux = aux;
    a.y = y;
    if (a.large)
        atm::launch_sweep_large(a, sweep_tasks(p, o), o->precision == 1, s);
    else if (o->precision == 1)
        atm::launch_sweep_mixed(a, sweep_tasks(p, o), s);
    else
        atm::launch_sweep(a, sweep_tasks(p, o), s);
    return check_launch();
}

atm_status do_coarse(atm::KArgs a, double* u, double* y, double* e, hipStream_t s)
{
    a.cg_count = &a.hdr->cg_coarse;
    a.u = u;
    a.y = y;
    a.e = e;
    if (a.large) {
        atm::launch_coarse_large(a, s);
        return check_launch();
    }
    if (a.fas) {
        atm::launch_tau(a, s);
        atm_status st = check_launch();
        if (st) return st;
    }
    atm::launch_coarse(a, s);
    return check_launch();
}

atm_status do_norm(atm::KArgs a, double* u, double* y, hipStream_t s, double* norm_out, atm::Header* hdr)
{
    a.u = u;
    a.y = y;
    atm::launch_norm(a, s);
    atm_status st = check_launch();
    if (st) return st;
    st = read_header(a, s, hdr);
    if (st) return st;
    *norm_out = sqrt(hdr->norm2);
    if (hdr->fail) return fail(ATM_ERR_INNER_SOLVE, "a CG solve inside Phi or Psi did not reach cg_rtol within %d iterations",
                               a.maxit);
    return ATM_OK;
}

// The stopping norm of precision 1 (implicit residual) and the paper-form
// norm of the exact step; both synchronise and read the header.
atm_status finish_norm(const atm::KArgs& a, hipStream_t s, double* norm_out, atm::Header* hdr)
{
    atm_status st = check_launch();
    if (st) return st;
    st = read_header(a, s, hdr);
    if (st) return st;
    *norm_out = sqrt(hdr->norm2);
    if (hdr->fail) return fail(ATM_ERR_INNER_SOLVE, "a CG solve inside Phi or Psi did not reach its tolerance within %d iterations",
                               a.maxit);
    return ATM_OK;
}

atm_status do_implicit_norm(atm::KArgs a, const double* u, hipStream_t s, double* norm_out, atm::Header* hdr)
{
    // one partial sum per workgroup; the workspace holds max(N_T + 1, kResidBlocks) of them
    const int64_t cap = a.NT + 1 > atm::kResidBlocks ? a.NT + 1 : atm::kResidBlocks;
    if (atm::implicit_residual_blocks(a) > cap)
        return fail(ATM_ERR_UNSUPPORTED, "implicit residual: %lld partial sums exceed the workspace's %lld",
                    (long long)atm::implicit_residual_blocks(a), (long long)cap);
    a.u = (double*)u;
    atm::launch_implicit_residual(a, s);
    return finish_norm(a, s, norm_out, hdr);
}

atm_status do_step_norm(atm::KArgs a, const atm_problem* p, const atm_options* o, const double* u, hipStream_t s,
                        double* norm_out, atm::Header* hdr)
{
    a.u = (double*)u;
    if (a.large)
        atm::launch_step_residual_large(a, sweep_tasks(p, o), s);
    else
        atm::launch_step_residual(a, sweep_tasks(p, o), s);
    return finish_norm(a, s, norm_out, hdr);
}

// A norm call outside atm_solve ends the window in which CG failures of earlier
// calls on this workspace are reported: the header is cleared once it is read.
atm_status after_standalone_norm(const atm::KArgs& a, atm_status st, double norm, hipStream_t s)
{
    if (st == ATM_OK || st == ATM_ERR_INNER_SOLVE) {
        atm::launch_reset(a.hdr, s);
        atm_status st2 = check_launch();
        if (st2) return st2;
    }
    if (st == ATM_OK && !isfinite(norm)) return fail(ATM_ERR_DIVERGED, "non-finite residual norm");
    return st;
}

// one batched forward pass f of the learned propagator over nb FP64 fields x + map(b) * stride,
// ending in the layer-4 epilogue l4 (whose nb/h/w/in/w4/b4 are filled here)
void learned_forward(const float* params, const __bf16* pk, __bf16* d1, __bf16* d2, int64_t nb, int h, int w,
                     const double* x, int64_t stride, atm::cnn::FieldMap xmap, atm::cnn::L4Args l4, hipStream_t s)
{
    using namespace atm::cnn;
    L1Args l1;
    memset(&l1, 0, sizeof(l1));
    l1.nb = nb;
    l1.h = h;
    l1.w = w;
    l1.x = x;
    l1.x_f64 = 1;
    l1.x_stride = stride;
    l1.xmap = xmap;
    l1.w1 = pk + PK_W1;
    l1.b1 = params + OFF_B1;
    l1.out = d1;
    launch_l1(l1, s);
    ConvArgs cv;
    memset(&cv, 0, sizeof(cv));
    cv.nb = nb;
    cv.h = h;
    cv.w = w;
    cv.in = d1;
    cv.out = d2;
    cv.wpk = pk + PK_W2F;
    cv.bias = params + OFF_B2;
    launch_conv32(cv, s);
    cv.in = d2;
    cv.out = d1;
    cv.wpk = pk + PK_W3F;
    cv.bias = params + OFF_B3;
    launch_conv32(cv, s);
    l4.nb = nb;
    l4.h = h;
    l4.w = w;
    l4.in = d1;
    l4.w4 = pk + PK_W4;
    l4.b4 = params + OFF_B4;
    launch_l4(l4, s);
}

// Learned coarse solve in FAS form (Alg. 2, coarsest level) with Psi(v) = v + f(v):
// tau_j = (v_j - Psi(v_{j-1})) + r_j, then every window w_s = v_s + r_s,
// w_j = Psi(w_{j-1}) + tau_j, e_p = w_p - v_p; the windows active at a step are one batch.
atm_status do_coarse_learned(atm::KArgs a, const Layout& L, void* ws, const atm_problem* p, const atm_options* o,
                             double* u, double* y, double* e, hipStream_t s)
{
    using namespace atm::cnn;
    char* base = (char*)ws;
    __bf16* pk = (__bf16*)(base + L.pk);
    __bf16* d1 = (__bf16*)(base + L.d1);
    __bf16* d2 = (__bf16*)(base + L.d2);
    const int64_t NT = a.NT, n = a.n;
    const int h = p->ny, w = p->nx;
    const float* params = o->cnn_params;
    launch_pack(params, pk, s);
    if (NT >= 1) {
        // tau_j, j = 1..N_T, from Psi at the states v_{j-1}
        L4Args l4;
        memset(&l4, 0, sizeof(l4));
        l4.epi = EPI_TAU;
        l4.tau = a.tau;
        l4.ysol = y;
        l4.usol = u;
        l4.m = a.m;
        FieldMap xm;
        memset(&xm, 0, sizeof(xm));
        learned_forward(params, pk, d1, d2, NT, h, w, u, (int64_t)a.m * n, xm, l4, s);
    }
    launch_window_init(e, y, u, NT, n, a.m, a.k, s);
    const int64_t steps = (a.k - 1 < NT) ? a.k - 1 : NT;
    for (int64_t t = 1; t <= steps; ++t) {
        // windows p = t..N_T take step t towards C-point s_p + t
        FieldMap sm;
        memset(&sm, 0, sizeof(sm));
        sm.mode = 2;
        sm.t = (int)t;
        sm.k = a.k;
        FieldMap em;
        memset(&em, 0, sizeof(em));
        em.off = t;
        L4Args l4;
        memset(&l4, 0, sizeof(l4));
        l4.epi = EPI_WINDOW;
        l4.e = e;
        l4.emap = em;
        l4.smap = sm;
        l4.tau = a.tau;
        learned_forward(params, pk, d1, d2, NT + 1 - t, h, w, e, n, em, l4, s);
    }
    launch_window_final(e, u, NT, n, a.m, s);
    return check_launch();
}

// Options used by atm_sequential (only the workspace header is needed).
atm_options sequential_options(const atm_problem* p)
{
    atm_options o;
    memset(&o, 0, sizeof(o));
    // one coarse interval: the workspace holds one task's buffers
    o.m = (p->nt >= 2 && p->nt <= INT32_MAX) ? (int32_t)p->nt : 2;
    o.k = 1;
    o.max_iter = 1;
    o.coarse_substeps = 1;
    o.coarse_form = 1;
    return o;
}

// Optional per-launch device timing with HIP events on the solve's stream.
struct PhaseTimer {
    bool on = false;
    hipEvent_t ev[8];
    int used = 0;
    double ms[3] = {0.0, 0.0, 0.0};
    int phase[4];
    atm_status init(bool enable)
    {
        on = enable;
        if (!on) return ATM_OK;
        for (int i = 0; i < 8; ++i) ATM_HIP(hipEventCreate(&ev[i]));
        return ATM_OK;
    }
    atm_status begin(int ph, hipStream_t s)
    {
        if (!on) return ATM_OK;
        phase[used / 2] = ph;
        ATM_HIP(hipEventRecord(ev[used++], s));
        return ATM_OK;
    }
    atm_status end(hipStream_t s)
    {
        if (!on) return ATM_OK;
        ATM_HIP(hipEventRecord(ev[used++], s));
        return ATM_OK;
    }
    // after a stream synchronisation: fold the recorded pairs into the totals
    atm_status collect()
    {
        if (!on) return ATM_OK;
        if (used > 0) ATM_HIP(hipEventSynchronize(ev[used - 1]));
        for (int i = 0; i + 1 < used; i += 2) {
            float t = 0.0f;
            ATM_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
            ms[phase[i / 2]] += t;
        }
        used = 0;
        return ATM_OK;
    }
    ~PhaseTimer()
    {
        if (on)
            for (int i = 0; i < 8; ++i) (void)hipEventDestroy(ev[i]);
    }
};
enum { kPhSweep = 0, kPhCoarse = 1, kPhNorm = 2 };

int64_t window_psi_count(int64_t NT, int64_t k)
{
    // sum over p = 0..N_T of min(p, k-1)
    int64_t tot = 0;
    for (int64_t p = 0; p <= NT; ++p) tot += (p < k - 1 ? p : k - 1);
    return tot;
}

}  // namespace

extern "C" {

int64_t atm_num_intervals(const atm_problem* prob, const atm_options* opts)
{
    if (!prob || !opts || opts->m < 1) return 0;
    return n_intervals(prob, opts);
}

int64_t atm_window_start(int64_t p, int32_t k) { return p - k + 1 > 0 ? p - k + 1 : 0; }

size_t atm_workspace_bytes(const atm_problem* prob, const atm_options* opts)
{
    if (validate(prob, opts) != ATM_OK) return 0;
    return layout(prob, opts).total;
}

atm_status atm_sweep(const atm_problem* prob, const atm_options* opts, int32_t mode, double* u, const double* aux,
                     double* y, void* ws, size_t ws_bytes, void* stream)
{
    atm::KArgs a;
    atm_status st = make_args(prob, opts, ws, ws_bytes, a);
    if (st) return st;
    if (mode < 0 || mode > 2) return fail(ATM_ERR_INVALID_ARG, "sweep mode must be 0, 1 or 2");
    if (!u || !y) return fail(ATM_ERR_INVALID_ARG, "null u or y");
    if (mode != 0 && !aux) return fail(ATM_ERR_INVALID_ARG, "sweep modes 1 and 2 need aux");
    if (aux == y) return fail(ATM_ERR_INVALID_ARG, "aux and y must not alias");
    return do_sweep(a, prob, opts, mode, u, aux, y, as_stream(stream));
}

atm_status atm_coarse_solve(const atm_problem* prob, const atm_options* opts, const double* u, const double* y,
                            double* e, void* ws, size_t ws_bytes, void* stream)
{
    atm::KArgs a;
    atm_status st = make_args(prob, opts, ws, ws_bytes, a);
    if (st) return st;
    if (!u || !y || !e) return fail(ATM_ERR_INVALID_ARG, "null u, y or e");
    if (e == y) return fail(ATM_ERR_INVALID_ARG, "e and y must not alias");
    if (learned(opts))
        return do_coarse_learned(a, layout(prob, opts), ws, prob, opts, (double*)u, (double*)y, e, as_stream(stream));
    return do_coarse(a, (double*)u, (double*)y, e, as_stream(stream));
}

atm_status atm_residual_norm(const atm_problem* prob, const atm_options* opts, const double* u, const double* y,
                             double* norm_out, void* ws, size_t ws_bytes, void* stream)
{
    atm::KArgs a;
    atm_status st = make_args(prob, opts, ws, ws_bytes, a);
    if (st) return st;
    if (!u || !y || !norm_out) return fail(ATM_ERR_INVALID_ARG, "null u, y or norm_out");
    atm::Header h;
    st = do_norm(a, (double*)u, (double*)y, as_stream(stream), norm_out, &h);
    return after_standalone_norm(a, st, *norm_out, as_stream(stream));
}

atm_status atm_implicit_residual_norm(const atm_problem* prob, const atm_options* opts, const double* u,
                                      double* norm_out, void* ws, size_t ws_bytes, void* stream)
{
    atm::KArgs a;
    atm_status st = make_args(prob, opts, ws, ws_bytes, a);
    if (st) return st;
    if (!u || !norm_out) return fail(ATM_ERR_INVALID_ARG, "null u or norm_out");
    atm::Header h;
    st = do_implicit_norm(a, u, as_stream(stream), norm_out, &h);
    return after_standalone_norm(a, st, *norm_out, as_stream(stream));
}

atm_status atm_step_residual_norm(const atm_problem* prob, const atm_options* opts, const double* u, double* norm_out,
                                  void* ws, size_t ws_bytes, void* stream)
{
    atm::KArgs a;
    atm_status st = make_args(prob, opts, ws, ws_bytes, a);
    if (st) return st;
    if (!u || !norm_out) return fail(ATM_ERR_INVALID_ARG, "null u or norm_out");
    atm::Header h;
    st = do_step_norm(a, prob, opts, u, as_stream(stream), norm_out, &h);
    return after_standalone_norm(a, st, *norm_out, as_stream(stream));
}

atm_status atm_sequential(const atm_problem* prob, double* u, void* ws, size_t ws_bytes, void* stream)
{
    if (!prob) return fail(ATM_ERR_INVALID_ARG, "null problem");
    if (prob->nt < 2) return fail(ATM_ERR_INVALID_ARG, "atm_sequential needs nt >= 2");
    const atm_options o = sequential_options(prob);
    atm::KArgs a;
    atm_status st = make_args(prob, &o, ws, ws_bytes, a);
    if (st) return st;
    if (!u) return fail(ATM_ERR_INVALID_ARG, "null u");
    a.u = u;
    hipStream_t s = as_stream(stream);
    atm::launch_reset(a.hdr, s);
    if (a.large)
        atm::launch_sequential_large(a, s);
    else
        atm::launch_sequential(a, s);
    st = check_launch();
    if (st) return st;
    atm::Header h;
    st = read_header(a, s, &h);
    if (st) return st;
    if (h.fail) return fail(ATM_ERR_INNER_SOLVE, "a CG solve did not reach cg_rtol within %d iterations", a.maxit);
    return ATM_OK;
}

size_t atm_sequential_workspace_bytes(const atm_problem* prob)
{
    if (!prob || prob->nt < 2) return 0;
    const atm_options o = sequential_options(prob);
    return atm_workspace_bytes(prob, &o);
}

atm_status atm_solve(const atm_problem* prob, const atm_options* opts, double* u, void* ws, size_t ws_bytes,
                     double* hist, int32_t hist_cap, atm_stats* stats, void* stream)
{
    const auto t_start = std::chrono::steady_clock::now();
    atm::KArgs a;
    atm_status st = make_args(prob, opts, ws, ws_bytes, a);
    if (st) return st;
    if (!u) return fail(ATM_ERR_INVALID_ARG, "null u");
    if (hist_cap < 0) return fail(ATM_ERR_INVALID_ARG, "hist_cap must be >= 0");
    const Layout L = layout(prob, opts);
    char* base = (char*)ws;
    double* ya = (double*)(base + L.ya);
    double* yb = (double*)(base + L.yb);
    double* e = (double*)(base + L.e);
    hipStream_t s = as_stream(stream);
    atm::launch_reset(a.hdr, s);
    if ((st = check_launch())) return st;

    const int64_t NT = n_intervals(prob, opts);
    atm_stats S;
    memset(&S, 0, sizeof(S));
    atm::Header h;
    memset(&h, 0, sizeof(h));
    PhaseTimer T;
    if ((st = T.init(opts->profile == 1))) return st;
#define ATM_TIMED(ph, expr)                           \
    do {                                              \
        if ((st = T.begin((ph), s))) break;           \
        if ((st = (expr))) break;                     \
        if ((st = T.end(s))) break;                   \
    } while (0)
    const bool mixed = (opts->precision == 1);
    // After the first sweep every interval's F-points are the relaxation of its stored C-point, so a
    // later FP64 sweep that starts an interval from the same value (bit for bit) would recompute
    // them identically: it is skipped.  (FP32 sweeps refine their F-points and never skip.)
    const bool skip = !mixed;
    // stopping norm: the C-point residual (FP64 form) or the FP64 implicit residual (mixed form)
    auto stop_norm = [&](double* yv, double* out) {
        return mixed ? do_implicit_norm(a, u, s, out, &h) : do_norm(a, u, yv, s, out, &h);
    };
    // F-relax the initial guess, then its residual
    ATM_TIMED(kPhSweep, do_sweep(a, prob, opts, 0, u, nullptr, ya, s));
    if (st) return st;
    S.fine_steps += prob->nt;
    S.n_sweeps += 1;
    double res = 0.0;
    ATM_TIMED(kPhNorm, stop_norm(ya, &res));
    if (st == ATM_OK) st = T.collect();
    if (st == ATM_OK && hist && hist_cap > 0) hist[0] = res;
    // yprev holds Phi of every last F-point from the latest sweep
    double* yprev = ya;
    int it = 0;
    bool use_learned = learned(opts);
    const double fb_ratio = opts->fallback_ratio > 0.0 ? opts->fallback_ratio : 0.95;
    const double res0 = res;
    bool descent_seen = false;
    int stagnant = 0;
    while (st == ATM_OK && !(res <= opts->tol)) {
        if (!isfinite(res)) {
            st = fail(ATM_ERR_DIVERGED, "non-finite residual norm after %d cycles", it);
            break;
        }
        if (it >= opts->max_iter) {
            st = ATM_NOT_CONVERGED;
            break;
        }
        double* ycur = yprev;
        if (opts->relax == 1) {
            // CF: C-points take Phi of their preceding F-point (held in yprev), then F-relax
            ycur = (yprev == ya) ? yb : ya;
            ATM_TIMED(kPhSweep, do_sweep(a, prob, opts, 2, u, yprev, ycur, s, skip, yprev));
            if (st) break;
            S.fine_steps += prob->nt;
            S.n_sweeps += 1;
        }
        if (use_learned) {
            ATM_TIMED(kPhCoarse, do_coarse_learned(a, L, ws, prob, opts, u, ycur, e, s));
            if (st) break;
            S.coarse_steps += window_psi_count(NT, opts->k) + NT;
            S.learned_cycles += 1;
        } else {
            ATM_TIMED(kPhCoarse, do_coarse(a, u, ycur, e, s));
            if (st) break;
            S.coarse_steps += window_psi_count(NT, opts->k) + (a.fas ? NT : 0);
        }
        // correction u_{pm} += e_p and F-interpolation; ycur receives Phi of every
        // last F-point (in the mixed form its entries also start those steps)
        ATM_TIMED(kPhSweep, do_sweep(a, prob, opts, 1, u, e, ycur, s, skip, nullptr));
        if (st) break;
        S.fine_steps += prob->nt;
        S.n_sweeps += 1;
        yprev = ycur;
        ++it;
        const double prev_res = res;
        ATM_TIMED(kPhNorm, stop_norm(yprev, &res));
        if (st == ATM_OK) st = T.collect();
        if (st == ATM_OK && hist && it < hist_cap) hist[it] = res;
        if (use_learned) {
            // fallback: stagnation after the residual has started to decrease, or growth far beyond
            // the transient of the truncated method
            if (res < prev_res) descent_seen = true;
            stagnant = (descent_seen && !(res <= fb_ratio * prev_res)) ? stagnant + 1 : 0;
            if (stagnant >= 2 || !(res <= kLearnedGrowthLimit * res0)) use_learned = false;
        }
    }
    if (st == ATM_OK && !isfinite(res)) st = fail(ATM_ERR_DIVERGED, "non-finite residual norm");
    double final_res = res;
    if (mixed && (st == ATM_OK || st == ATM_NOT_CONVERGED)) {
        // the paper-form residual of the returned iterate (bounded by the stopping norm)
        atm_status st2 = ATM_OK;
        if ((st2 = T.begin(kPhNorm, s)) == ATM_OK && (st2 = do_step_norm(a, prob, opts, u, s, &final_res, &h)) == ATM_OK &&
            (st2 = T.end(s)) == ATM_OK)
            st2 = T.collect();
        if (st2 != ATM_OK) st = st2;
    }
#undef ATM_TIMED
    S.iterations = it;
    S.final_residual = final_res;
    S.cg_fine = (int64_t)h.cg_fine;
    S.cg_coarse = (int64_t)h.cg_coarse;
    S.fine_steps_skipped = (int64_t)h.skipped;
    S.fine_steps -= S.fine_steps_skipped;
    S.ms_sweep = T.ms[kPhSweep];
    S.ms_coarse = T.ms[kPhCoarse];
    S.ms_norm = T.ms[kPhNorm];
    S.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = S;
    return st;
}

const char* atm_status_string(atm_status status)
{
    switch (status) {
        case ATM_OK: return "ATM_OK";
        case ATM_NOT_CONVERGED: return "ATM_NOT_CONVERGED";
        case ATM_ERR_INVALID_ARG: return "ATM_ERR_INVALID_ARG";
        case ATM_ERR_UNSUPPORTED: return "ATM_ERR_UNSUPPORTED";
        case ATM_ERR_DEVICE: return "ATM_ERR_DEVICE";
        case ATM_ERR_DIVERGED: return "ATM_ERR_DIVERGED";
        case ATM_ERR_INNER_SOLVE: return "ATM_ERR_INNER_SOLVE";
        case ATM_ERR_WORKSPACE: return "ATM_ERR_WORKSPACE";
        default: return "ATM_UNKNOWN_STATUS";
    }
}

const char* atm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
