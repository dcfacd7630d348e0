// Host side of libatmgrit.so: argument validation, workspace layout, launch
// sequencing of the two-level AT-MGRIT cycle (Alg. 1) and the C-ABI.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/atm.h"
#include "atm_batch.hpp"
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
    size_t header, partials, ya, yb, e, tau, pk, d1, d2, large, spec, cres, traj, u1, y1a, y1b, tau2, e2, total;
};

int64_t n_intervals(const atm_problem* p, const atm_options* o) { return p->nt / o->m; }
int64_t n_space(const atm_problem* p) { return (int64_t)p->nx * p->ny; }

// 2D grids beyond the on-chip strip layout run the global-scratch kernels
bool large_grid(const atm_problem* p)
{
    return p->kind != ATM_HEAT1D && (p->nx > atm::kMaxSide2D || p->ny > atm::kMaxSide2D);
}

// large grids whose windows the paired BF16 kernel takes: rows of 128, 192 or 256 points, 128 or 256
// rows (two halves of 64 or 128)
bool bf_pair_grid(const atm_problem* p)
{
    return p->nx % 64 == 0 && p->nx >= 128 && p->nx <= 256 && (p->ny == 128 || p->ny == 256);
}

// the multilevel FAS V-cycle over three levels (Alg. 2)
bool three_level(const atm_options* o) { return o->levels == 3; }
// level-2 points of the three-level cycle: 0..floor(floor(nt/m)/m_coarse)
int64_t n_level2(const atm_problem* p, const atm_options* o) { return (p->nt / o->m) / o->m_coarse; }

// the plain coarse propagator's form (coarse_form 3 falls back to the automatic choice)
bool use_fas(const atm_problem* p, const atm_options* o)
{
    if (o->coarse_form == 1) return false;
    if (o->coarse_form == 2) return true;
    return p->kind == ATM_AC2D;
}

bool learned(const atm_options* o) { return o->coarse_form == 3; }

// Psi's implicit solve by the eigenbasis of the constant-coefficient operator (2D kinds, coarse_solver 0)
// three levels with coarse_solver 2: the coarsest level's windows on the BF16 matrix cores (level 1
// keeps CG, so that its FAS right-hand side and relaxation share Phi_1 exactly)
bool ml_bf(const atm_problem* p, const atm_options* o)
{
    return o->levels == 3 && o->coarse_solver == 2 && p->kind != ATM_HEAT1D;
}

bool spectral(const atm_problem* p, const atm_options* o)
{
    return p->kind != ATM_HEAT1D && (o->coarse_solver == 0 || o->coarse_solver == 2) && !three_level(o);
}

// rows of n of the trajectory of v through Psi's substeps (the paired BF16 windows' FAS form)
size_t traj_rows(const atm_problem* p, const atm_options* o)
{
    if (!(large_grid(p) && spectral(p, o) && o->coarse_solver == 2 && use_fas(p, o) && o->coarse_substeps > 1))
        return 0;
    return (size_t)n_intervals(p, o) * (size_t)(o->coarse_substeps - 1);
}

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
    L.tau = off;  // the FAS right-hand side of the windows; with three levels, that of level 1
    off += (use_fas(p, o) || three_level(o)) ? align_up(slab) : 0;
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
    const size_t slab2 = three_level(o) ? (size_t)(n_level2(p, o) + 1) * (size_t)n_space(p) * sizeof(double) : 0;
    L.spec = off;
    off += (spectral(p, o) || ml_bf(p, o))
               ? align_up((atm::spectral_table_doubles(p->nx, p->ny) +
                           (o->coarse_solver == 2 ? atm::spectral_bf16_doubles(p->nx, p->ny) : 0)) *
                          sizeof(double))
               : 0;
    L.cres = off;  // coarse_solver 2: the windows' C-point residuals (three levels: the coarsest level's)
    off += ml_bf(p, o) ? align_up(slab2)
                       : ((spectral(p, o) && o->coarse_solver == 2 && !large_grid(p)) ? align_up(slab) : 0);
    L.traj = off;  // the paired BF16 windows, FAS form with s > 1 substeps: v through Psi's first s - 1
    off += traj_rows(p, o) ? align_up((size_t)traj_rows(p, o) * (size_t)n_space(p) * sizeof(float)) : 0;
    // three levels: the level-1 iterate [N_T+1][n]; the level-1 sweeps' y (two), the level-2 FAS
    // right-hand side and corrections, [N_2+1][n] each
    L.u1 = off;
    off += three_level(o) ? align_up(slab) : 0;
    L.y1a = off;
    off += align_up(slab2);
    L.y1b = off;
    off += align_up(slab2);
    L.tau2 = off;
    off += align_up(slab2);
    L.e2 = off;
    off += align_up(slab2);
    L.total = off;
    return L;
}

// The window phase alone (atm_coarse_solve_static): the header, the norm partials, the FAS
// right-hand side tau, the eigenbasis tables and the BF16 form's C-point residuals; every other
// region is empty (offset 0, never touched by the window kernels).
Layout coarse_layout(const atm_problem* p, const atm_options* o)
{
    const size_t NT = (size_t)n_intervals(p, o);
    const size_t slab = (NT + 1) * (size_t)n_space(p) * sizeof(double);
    Layout L;
    memset(&L, 0, sizeof(L));
    size_t off = 0;
    L.header = off;
    off += align_up(sizeof(atm::Header));
    L.partials = off;
    off += align_up((NT + 1 > (size_t)atm::kResidBlocks ? NT + 1 : (size_t)atm::kResidBlocks) * sizeof(double));
    L.tau = off;
    off += use_fas(p, o) ? align_up(slab) : 0;
    L.spec = off;
    off += spectral(p, o) ? align_up((atm::spectral_table_doubles(p->nx, p->ny) +
                                      (o->coarse_solver == 2 ? atm::spectral_bf16_doubles(p->nx, p->ny) : 0)) *
                                     sizeof(double))
                          : 0;
    L.cres = off;
    off += (spectral(p, o) && o->coarse_solver == 2) ? align_up(slab) : 0;
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
    if (p->source && p->kind != ATM_HEAT1D)
        return fail(ATM_ERR_UNSUPPORTED, "a PDE source is supported for ATM_HEAT1D only");
    if (p->kind != ATM_HEAT1D && (!(p->cg_rtol >= 0.0) || p->cg_max_iter < 1))
        return fail(ATM_ERR_INVALID_ARG, "cg_rtol must be >= 0 and cg_max_iter >= 1");
    if (o->m < 2) return fail(ATM_ERR_INVALID_ARG, "coarsening factor m must be >= 2");
    if (p->nt < o->m) return fail(ATM_ERR_INVALID_ARG, "nt (%lld) must be >= m (%d)", (long long)p->nt, o->m);
    if (o->k < 1) return fail(ATM_ERR_INVALID_ARG, "k must be >= 1");
    if (o->relax != 0 && o->relax != 1) return fail(ATM_ERR_INVALID_ARG, "relax must be 0 (F) or 1 (FCF)");
    if (o->coarse_substeps < 1) return fail(ATM_ERR_INVALID_ARG, "coarse_substeps must be >= 1");
    if (o->coarse_form < 0 || o->coarse_form > 3) return fail(ATM_ERR_INVALID_ARG, "coarse_form must be 0, 1, 2 or 3");
    if (o->coarse_solver < 0 || o->coarse_solver > 2)
        return fail(ATM_ERR_INVALID_ARG, "coarse_solver must be 0 (auto), 1 (CG) or 2 (eigenbasis on BF16 matrix cores)");
    if (o->coarse_solver == 2 && o->levels != 3) {
        if (p->kind == ATM_HEAT1D || o->coarse_form == 3)
            return fail(ATM_ERR_UNSUPPORTED, "coarse_solver 2 is built for the plain coarse propagator of the 2D kinds");
        if (large_grid(p)) {
            if (!bf_pair_grid(p))
                return fail(ATM_ERR_UNSUPPORTED,
                            "coarse_solver 2 beyond 128 points per side takes rows of 128, 192 or 256 points and "
                            "128 or 256 rows");
        } else if (use_fas(p, o) && o->coarse_substeps != 1) {
            return fail(ATM_ERR_UNSUPPORTED, "coarse_solver 2 takes the FAS form with coarse_substeps 1");
        }
    }
    if (o->coarse_form == 3) {
        if (p->kind != ATM_AC2D)
            return fail(ATM_ERR_UNSUPPORTED, "the learned coarse propagator is built for the periodic ATM_AC2D grid");
        if (p->nx % 16 != 0 || p->nx > 128)
            return fail(ATM_ERR_UNSUPPORTED, "the learned coarse propagator needs nx a multiple of 16, at most 128");
        if (!o->cnn_params) return fail(ATM_ERR_INVALID_ARG, "coarse_form 3 needs cnn_params");
        if (!(o->fallback_ratio >= 0.0)) return fail(ATM_ERR_INVALID_ARG, "fallback_ratio must be >= 0");
    }
    if (o->max_iter < 0) return fail(ATM_ERR_INVALID_ARG, "max_iter must be >= 0");
    if (o->levels != 0 && o->levels != 2 && o->levels != 3)
        return fail(ATM_ERR_UNSUPPORTED, "levels must be 2 (or 0) or 3");
    if (o->levels == 3) {
        if (o->m_coarse < 2) return fail(ATM_ERR_INVALID_ARG, "levels 3 needs m_coarse >= 2");
        if (p->nt / o->m < o->m_coarse)
            return fail(ATM_ERR_INVALID_ARG, "levels 3 needs floor(nt/m) (%lld) >= m_coarse (%d)",
                        (long long)(p->nt / o->m), o->m_coarse);
        if (o->precision != 0) return fail(ATM_ERR_UNSUPPORTED, "levels 3 runs in precision 0");
        if (o->coarse_form == 3) return fail(ATM_ERR_UNSUPPORTED, "levels 3 uses the plain coarse propagator");
        if (large_grid(p)) return fail(ATM_ERR_UNSUPPORTED, "levels 3 takes grids up to 128 x 128");
        if (ml_bf(p, o) && o->coarse_substeps != 1)
            return fail(ATM_ERR_UNSUPPORTED, "levels 3 with coarse_solver 2 takes coarse_substeps 1");
    }
    if (o->nested != 0 && o->nested != 1) return fail(ATM_ERR_INVALID_ARG, "nested must be 0 or 1");
    if (o->nested == 1) {
        if (p->source) return fail(ATM_ERR_UNSUPPORTED, "nested iteration takes no PDE source");
        if (o->precision != 0) return fail(ATM_ERR_UNSUPPORTED, "nested iteration runs in precision 0");
        if (o->coarse_form == 3) return fail(ATM_ERR_UNSUPPORTED, "nested iteration uses the plain coarse propagator");
        if (large_grid(p)) return fail(ATM_ERR_UNSUPPORTED, "nested iteration takes grids up to 128 x 128");
    }
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
atm_status make_args_in(const atm_problem* p, const atm_options* o, void* ws, size_t ws_bytes, const Layout& L,
                        atm::KArgs& a);

atm_status make_args(const atm_problem* p, const atm_options* o, void* ws, size_t ws_bytes, atm::KArgs& a)
{
    atm_status st = validate(p, o);
    if (st) return st;
    return make_args_in(p, o, ws, ws_bytes, layout(p, o), a);
}

// the kernel arguments over a workspace laid out as L (p and o validated)
atm_status make_args_in(const atm_problem* p, const atm_options* o, void* ws, size_t ws_bytes, const Layout& L,
                        atm::KArgs& a)
{
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
    a.tau = (use_fas(p, o) || three_level(o)) ? (double*)(base + L.tau) : nullptr;
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
    a.src = p->source;
    a.dt = dt;
    a.gadd = nullptr;
    a.fine_substeps = 1;
    a.psi_only = 0;
    a.fine = step_coef(p, dt);
    a.coarse = step_coef(p, dt * o->m / o->coarse_substeps);
    a.rtol2 = p->cg_rtol * p->cg_rtol;
    const double crtol = o->coarse_cg_rtol > 0.0 ? o->coarse_cg_rtol : p->cg_rtol;
    a.rtol2_coarse = crtol * crtol;
    const double mrtol = o->mixed_cg_rtol > 0.0 ? o->mixed_cg_rtol : kMixedRtolDefault;
    a.rtol2_mixed = mrtol * mrtol;
    a.maxit = p->cg_max_iter;
    a.spectral = spectral(p, o) ? (o->coarse_solver == 2 ? 2 : 1) : 0;
    a.spec = (a.spectral || ml_bf(p, o)) ? (double*)(base + L.spec) : nullptr;
    a.cres = (a.spectral == 2 && !large_grid(p)) ? (double*)(base + L.cres) : nullptr;
    a.traj = traj_rows(p, o) ? (float*)(base + L.traj) : nullptr;
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

// Read back the header (norm, failure flag, CG count) after synchronising.  The copy lands in a
// pinned host buffer of the calling thread (allocated on its first readback and kept for the
// thread's life: 32 bytes), so the DMA writes it directly instead of staging a pageable copy.
// The failure flags of a header read back after a synchronisation: a workgroup pair of the large-grid
// FP32 sweep that gave up waiting for its partner, or a CG solve that missed its tolerance.
atm_status header_status(const atm::Header& h, int maxit)
{
    if (h.fail & atm::kFailPairTimeout)
        return fail(ATM_ERR_DEVICE, "a workgroup pair of the relaxation sweep did not meet within its wait limit");
    if (h.fail)
        return fail(ATM_ERR_INNER_SOLVE, "a CG solve inside Phi or Psi did not reach its tolerance within %d iterations",
                    maxit);
    return ATM_OK;
}

atm_status pinned_header(atm::Header** out)
{
    static thread_local atm::Header* pinned = nullptr;
    if (!pinned) {
        void* ptr = nullptr;
        ATM_HIP(hipHostMalloc(&ptr, sizeof(atm::Header), hipHostMallocDefault));
        pinned = static_cast<atm::Header*>(ptr);
    }
    *out = pinned;
    return ATM_OK;
}

atm_status read_header(const atm::KArgs& a, hipStream_t s, atm::Header* out)
{
    atm::Header* pinned = nullptr;
    atm_status st = pinned_header(&pinned);
    if (st) return st;
    ATM_HIP(hipMemcpyAsync(pinned, a.hdr, sizeof(atm::Header), hipMemcpyDeviceToHost, s));
    ATM_HIP(hipStreamSynchronize(s));
    *out = *pinned;
    return ATM_OK;
}

// The norm kernels publish the header into the pinned buffer themselves (publish_header): arm the
// buffer with a mark no norm produces before the launch, and read it after synchronising.
constexpr uint64_t kUnpublished = 0x7FF4DEADBEEF0002ull;

atm_status arm_published(atm::KArgs& a)
{
    atm::Header* pinned = nullptr;
    atm_status st = pinned_header(&pinned);
    if (st) return st;
    memcpy(&pinned->norm2, &kUnpublished, sizeof(double));
    a.hdr_host = pinned;
    return ATM_OK;
}

atm_status read_published(const atm::KArgs& a, hipStream_t s, atm::Header* out)
{
    ATM_HIP(hipStreamSynchronize(s));
    const volatile atm::Header* h = a.hdr_host;
    out->norm2 = h->norm2;
    out->fail = h->fail;
    out->cg_fine = h->cg_fine;
    out->cg_coarse = h->cg_coarse;
    out->skipped = h->skipped;
    uint64_t bits;
    memcpy(&bits, &out->norm2, sizeof(bits));
    if (bits == kUnpublished) return fail(ATM_ERR_DEVICE, "the norm kernel did not publish its header");
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
    if (a.large) {
        const hipError_t e = atm::launch_sweep_large(a, sweep_tasks(p, o), o->precision == 1, s);
        if (e != hipSuccess) return fail(ATM_ERR_DEVICE, "sweep launch: %s", hipGetErrorString(e));
    } else if (o->precision == 1)
        atm::launch_sweep_mixed(a, sweep_tasks(p, o), s);
    else
        atm::launch_sweep(a, sweep_tasks(p, o), s);
    return check_launch();
}

// tables_ready: the eigenbasis tables of the grid are already in the workspace (a solve builds them
// once before its cycles)
atm_status do_coarse(atm::KArgs a, double* u, double* y, double* e, hipStream_t s, bool tables_ready = false)
{
    a.cg_count = &a.hdr->cg_coarse;
    a.u = u;
    a.y = y;
    a.e = e;
    if (a.large) {
        const hipError_t err = atm::launch_coarse_large(a, s);
        if (err != hipSuccess) return fail(ATM_ERR_DEVICE, "window launch: %s", hipGetErrorString(err));
        return check_launch();
    }
    if (a.spectral && !tables_ready) atm::launch_spectral_tables(a, s);
    if (a.fas && a.spectral != 2) {  // the BF16 windows take FAS in terms of e and need no tau
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
    atm_status st = arm_published(a);
    if (st) return st;
    atm::launch_norm(a, s);
    st = check_launch();
    if (st) return st;
    st = read_published(a, s, hdr);
    if (st) return st;
    *norm_out = sqrt(hdr->norm2);
    return header_status(*hdr, a.maxit);
}

// The stopping norm of precision 1 (implicit residual) and the paper-form
// norm of the exact step; both synchronise and read the header.
atm_status finish_norm(const atm::KArgs& a, hipStream_t s, double* norm_out, atm::Header* hdr)
{
    atm_status st = check_launch();
    if (st) return st;
    st = read_published(a, s, hdr);
    if (st) return st;
    *norm_out = sqrt(hdr->norm2);
    return header_status(*hdr, a.maxit);
}

atm_status do_implicit_norm(atm::KArgs a, const double* u, hipStream_t s, double* norm_out, atm::Header* hdr)
{
    // one partial sum per workgroup; the workspace holds max(N_T + 1, kResidBlocks) of them
    const int64_t cap = a.NT + 1 > atm::kResidBlocks ? a.NT + 1 : atm::kResidBlocks;
    if (atm::implicit_residual_blocks(a) > cap)
        return fail(ATM_ERR_UNSUPPORTED, "implicit residual: %lld partial sums exceed the workspace's %lld",
                    (long long)atm::implicit_residual_blocks(a), (long long)cap);
    a.u = (double*)u;
    atm_status st = arm_published(a);
    if (st) return st;
    atm::launch_implicit_residual(a, s);
    return finish_norm(a, s, norm_out, hdr);
}

atm_status do_step_norm(atm::KArgs a, const atm_problem* p, const atm_options* o, const double* u, hipStream_t s,
                        double* norm_out, atm::Header* hdr)
{
    a.u = (double*)u;
    atm_status st = arm_published(a);
    if (st) return st;
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

// ---------------------------------------------------------------------------
// the multilevel FAS V-cycle over three levels (Alg. 2, section 2.2)
// ---------------------------------------------------------------------------

// Level 1 of the three-level cycle: every m-th fine point, step dt m in coarse_substeps substeps
// (CG to coarse_cg_rtol), coarsening m_coarse to level 2 (step dt m m_coarse), the coarsest, whose
// local grids are solved by the window kernels in FAS form.  gadd holds level 1's FAS right-hand
// side, tau the windows'.
atm::KArgs level1_args(const atm::KArgs& a0, const atm_problem* p, const atm_options* o, const Layout& L, char* base)
{
    atm::KArgs a1 = a0;
    const double dt1 = (p->tf - p->t0) / (double)p->nt * o->m;
    const int s = o->coarse_substeps;
    a1.nt = p->nt / o->m;
    a1.m = o->m_coarse;
    a1.NT = a1.nt / o->m_coarse;
    a1.fas = 1;
    a1.fine_substeps = s;
    a1.fine = step_coef(p, dt1 / s);
    a1.substeps = s;
    a1.coarse = step_coef(p, dt1 * o->m_coarse / s);
    a1.rtol2 = a0.rtol2_coarse;
    a1.src = nullptr;
    a1.gadd = (double*)(base + L.tau);
    a1.tau = (double*)(base + L.tau2);
    a1.cg_count = &a0.hdr->cg_coarse;
    a1.skip_unchanged = 0;
    a1.skip_y_src = nullptr;
    a1.spectral = ml_bf(p, o) ? 2 : 0;
    a1.cres = ml_bf(p, o) ? (double*)(base + L.cres) : nullptr;
    return a1;
}

// a sweep of level 1 (no interval skipping: its right-hand side changes every cycle)
atm_status do_level_sweep(atm::KArgs a, int mode, double* u, const double* aux, double* y, hipStream_t s)
{
    a.mode = mode;
    a.u = u;
    a.aux = aux;
    a.y = y;
    atm::launch_sweep(a, a.NT + 1, s);
    return check_launch();
}

// One cycle of level 1 for its system (right-hand side a1.gadd: level 1's FAS right-hand side, or
// null for the re-discretised system of nested iteration): F(CF)^nu relaxation, its C-point
// residuals and the local FAS problems of the coarsest level (windows), and the correction by ideal
// interpolation.
atm_status level1_cycle(const atm::KArgs& a1, const atm_options* o, double* u1, double* y1a, double* y1b, double* e2,
                        hipStream_t s, int64_t* psi_steps)
{
    atm_status st;
    if ((st = do_level_sweep(a1, 0, u1, nullptr, y1a, s))) return st;
    double* y1 = y1a;
    int sweeps = 2;
    if (o->relax == 1) {
        if ((st = do_level_sweep(a1, 2, u1, y1a, y1b, s))) return st;
        y1 = y1b;
        sweeps = 3;
    }
    atm::KArgs c1 = a1;
    c1.u = u1;
    c1.y = y1;
    c1.e = e2;
    if (c1.spectral != 2) {  // the BF16 windows take FAS in terms of e and need no tau
        atm::launch_tau(c1, s);
        if ((st = check_launch())) return st;
    }
    atm::launch_coarse(c1, s);
    if ((st = check_launch())) return st;
    if ((st = do_level_sweep(a1, 1, u1, e2, y1a, s))) return st;
    *psi_steps += sweeps * a1.nt + a1.NT + window_psi_count(a1.NT, a1.k);
    return ATM_OK;
}

// Everything of one V-cycle below the fine level, given the relaxed fine iterate u and y0_j =
// Phi(u_{jm-1}) (so the fine residual at C-point j is y0_j - u_{jm}): inject the iterate (u1 = v),
// level 1's FAS right-hand side tau1_j = (v_j - Phi_1(v_{j-1})) + r_j, and level 1's cycle.  On
// return u1 holds level 1's corrected iterate; the fine correction (e = u1 - v at the fine C-points,
// then F-interpolation) is the caller's sweep.
atm_status do_lower_levels(const atm::KArgs& a0, const atm::KArgs& a1, const atm_options* o, double* u, double* y0,
                           double* u1, double* tau1, double* y1a, double* y1b, double* e2, hipStream_t s,
                           int64_t* psi_steps)
{
    atm::launch_gather(u, u1, a0.n, a0.m, a1.nt + 1, s);
    atm_status st = check_launch();
    if (st) return st;
    atm::KArgs t0 = a0;
    t0.u = u;
    t0.y = y0;
    t0.tau = tau1;  // a1.gadd
    t0.cg_count = &a0.hdr->cg_coarse;
    atm::launch_tau(t0, s);
    if ((st = check_launch())) return st;
    *psi_steps += a1.nt;
    return level1_cycle(a1, o, u1, y1a, y1b, e2, s, psi_steps);
}

// Nested iteration (section 2.2): the initial guess rebuilt from the coarse levels up.  Two levels:
// the windows of the re-discretised coarse system from the injected guess, then the correction
// (C-points take the windows' values) with F-interpolation.  Three levels: inject to level 1, the
// coarsest windows, interpolation to level 1, one cycle of level 1's own system, interpolation to
// the fine level.  u ends F-relaxed.
atm_status nested_setup(const atm::KArgs& a, const atm::KArgs& a1, const atm_problem* p, const atm_options* o, double* u,
                        double* ya, double* e, double* u1, double* y1a, double* y1b, double* e2, hipStream_t s,
                        atm_stats& S);

// The coarsest level of nested iteration: y_j = Psi(v_{j-1}) for the injected guess v (the C-points
// of c.u), then the windows, which read the coarse residual y_j - v_j, into e (FAS: w_p - v_p).
atm_status nested_coarsest(atm::KArgs c, double* u, double* y, double* e, hipStream_t s)
{
    c.cg_count = &c.hdr->cg_coarse;
    c.u = u;
    c.y = y;
    c.e = e;
    if (c.spectral) atm::launch_spectral_tables(c, s);
    atm::KArgs q = c;
    q.psi_only = 1;
    atm::launch_tau(q, s);
    atm_status st = check_launch();
    if (st) return st;
    if (c.fas && c.spectral != 2) {
        atm::launch_tau(c, s);
        if ((st = check_launch())) return st;
    }
    atm::launch_coarse(c, s);
    return check_launch();
}

atm_status nested_setup(const atm::KArgs& a, const atm::KArgs& a1, const atm_problem* p, const atm_options* o, double* u,
                        double* ya, double* e, double* u1, double* y1a, double* y1b, double* e2, hipStream_t s,
                        atm_stats& S)
{
    atm_status st;
    if (!three_level(o)) {
        if ((st = nested_coarsest(a, u, ya, e, s))) return st;
        S.coarse_steps += a.NT * (a.fas ? 2 : 1) + window_psi_count(a.NT, a.k);
        S.fine_steps += p->nt;
        S.n_sweeps += 1;
        return do_sweep(a, p, o, 1, u, e, ya, s);
    }
    atm::launch_gather(u, u1, a.n, a.m, a1.nt + 1, s);
    if ((st = check_launch())) return st;
    atm::KArgs b1 = a1;
    b1.gadd = nullptr;  // level 1's own re-discretised system
    if ((st = nested_coarsest(b1, u1, y1a, e2, s))) return st;
    if ((st = do_level_sweep(b1, 1, u1, e2, y1b, s))) return st;
    int64_t steps = 2 * b1.NT + window_psi_count(b1.NT, b1.k) + b1.nt;
    if ((st = level1_cycle(b1, o, u1, y1a, y1b, e2, s, &steps))) return st;
    S.coarse_steps += steps;
    S.fine_steps += p->nt;
    S.n_sweeps += 1;
    return do_sweep(a, p, o, 2, u, u1, ya, s);
}

}  // namespace


// ---------------------------------------------------------------------------
// batched solves
// ---------------------------------------------------------------------------

namespace batchhost {

using atm::batch::Body;
using atm::batch::InstCtl;
using atm::batch::Task;

constexpr int kHistCap = 256;  // stopping norms kept per instance
constexpr int kNormChunks = 64;  // implicit-residual pieces of a 2D instance (at most nt)
enum { PH_S0, PH_N0, PH_NF0, PH_S2, PH_TAU, PH_C, PH_S1, PH_N, PH_NF, NPH };
enum { CLS_1D, CLS_2D, CLS_2DP, NCLS };

struct Inst {
    atm_problem p;
    atm_options o;
    double* u;  // the instance's iterate (device)
    Layout L;
    size_t off;  // of the instance's region in the workspace
    int cls, S, nchunk;
    bool mixed;
};

struct Group {
    int phase, cls, S;
    bool small;  // every instance has at most 64 columns (S = 8 only)
    Body body;
    size_t task_off;
    int ntasks;
};

size_t control_bytes(int n, size_t ntasks)
{
    return align_up((size_t)NPH * n * sizeof(atm::KArgs)) + align_up(n * sizeof(InstCtl)) + align_up(n * sizeof(int)) +
           align_up((size_t)n * kHistCap * sizeof(double)) + align_up(ntasks * sizeof(Task));
}

int phase_tasks(const Inst& in, int ph)
{
    const int64_t NT = n_intervals(&in.p, &in.o);
    const bool fas = use_fas(&in.p, &in.o) && in.cls != CLS_1D && in.o.coarse_solver != 2;
    switch (ph) {
        case PH_S0:
        case PH_S1: return (int)(NT + 1);
        case PH_S2: return in.o.relax == 1 ? (int)(NT + 1) : 0;
        case PH_TAU: return fas ? (int)NT : 0;
        case PH_C: return (int)(NT + 1);
        case PH_N0:
        case PH_N: return in.mixed ? in.nchunk : (int)NT;
        default: return 1;  // sums
    }
}

Body phase_body(const Inst& in, int ph)
{
    using namespace atm::batch;
    switch (ph) {
        case PH_S0:
        case PH_S2:
        case PH_S1: return in.cls == CLS_1D ? kSweep1D : (in.mixed ? kSweep2D : kSweep2D64);
        case PH_TAU: return spectral(&in.p, &in.o) ? kTau2DSpec : kTau2D;
        case PH_C:
            if (in.cls == CLS_1D) return kCoarse1D;
            if (spectral(&in.p, &in.o))
                return in.o.coarse_solver == 2 ? (use_fas(&in.p, &in.o) ? kCoarse2DBfFas : kCoarse2DBf) : kCoarse2DSpec;
            return kCoarse2D;
        case PH_N0:
        case PH_N: return in.mixed ? kNormI : kNormC;
        default: return in.mixed ? kNormFinalI : kNormFinalC;
    }
}

// relative cost of one task, for longest-first ordering
double task_cost(const Inst& in, int ph, int idx)
{
    const double n = (double)in.p.nx * in.p.ny;
    switch (ph) {
        case PH_S0:
        case PH_S2:
        case PH_S1: return n * in.o.m;
        case PH_TAU: return n * in.o.coarse_substeps;
        case PH_C: return n * in.o.coarse_substeps * std::min(idx, in.o.k - 1);
        case PH_N0:
        case PH_N: return in.mixed ? n * (double)in.p.nt / in.nchunk : n;
        default: return 1.0;
    }
}

}  // namespace batchhost

struct atm_batch {
    int n = 0;
    std::vector<batchhost::Inst> inst;
    char* ws = nullptr;
    size_t ctl_off = 0;
    atm::KArgs* args_dev = nullptr;  // [NPH][n]
    batchhost::InstCtl* ctl_dev = nullptr;
    int* nchunk_dev = nullptr;
    double* hist_dev = nullptr;
    batchhost::Task* tasks_dev = nullptr;
    size_t max_tasks = 0;
    std::vector<batchhost::Group> groups;
    int order = 1, tiles = 1;  // chosen by the autotuner: 0 natural / 1 longest first; 0 one tile / 1 per instance
    bool tuned = false;
    std::string cache;
    hipStream_t main = nullptr;
    hipStream_t br[batchhost::NCLS] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[batchhost::NCLS] = {nullptr, nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double ms_tune = 0.0;
    ~atm_batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (int c = 0; c < batchhost::NCLS; ++c) {
            if (br[c]) (void)hipStreamDestroy(br[c]);
            if (join[c]) (void)hipEventDestroy(join[c]);
        }
        if (fork) (void)hipEventDestroy(fork);
        if (main) (void)hipStreamDestroy(main);
    }
};

namespace batchhost {

size_t count_tasks(const std::vector<Inst>& v)
{
    size_t t = 0;
    for (const Inst& in : v)
        for (int ph = 0; ph < NPH; ++ph) t += phase_tasks(in, ph);
    return t;
}

atm_status describe(int32_t n, const atm_problem* probs, const atm_options* opts, std::vector<Inst>& v, size_t& total)
{
    if (n < 1) return fail(ATM_ERR_INVALID_ARG, "a batch needs at least one instance");
    if (!probs || !opts) return fail(ATM_ERR_INVALID_ARG, "null problems or options");
    v.resize(n);
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        Inst& in = v[i];
        in.p = probs[i];
        in.o = opts[i];
        atm_status st = validate(&in.p, &in.o);
        if (st) return fail(st, "instance %d: %s", i, g_last_error.c_str());
        if (learned(&in.o)) return fail(ATM_ERR_UNSUPPORTED, "instance %d: batches use the plain coarse propagator", i);
        if (large_grid(&in.p)) return fail(ATM_ERR_UNSUPPORTED, "instance %d: batches take grids up to 128 x 128", i);
        if (in.p.source) return fail(ATM_ERR_UNSUPPORTED, "instance %d: batches take no PDE source", i);
        if (three_level(&in.o)) return fail(ATM_ERR_UNSUPPORTED, "instance %d: batches run two levels", i);
        in.cls = in.p.kind == ATM_HEAT1D ? CLS_1D : (in.p.kind == ATM_AC2D ? CLS_2DP : CLS_2D);
        if (in.cls == CLS_1D && in.p.nx > 512)
            return fail(ATM_ERR_UNSUPPORTED, "instance %d: 1D batch instances take nx <= 512", i);
        in.mixed = in.o.precision == 1;
        in.nchunk = (int)std::min<int64_t>(kNormChunks, in.p.nt);
        in.L = layout(&in.p, &in.o);
        in.off = off;
        off += align_up(in.L.total);
    }
    total = off + control_bytes(n, count_tasks(v));
    return ATM_OK;
}

// the instance's arguments for each phase
atm_status phase_args(atm_batch* B, int i, atm::KArgs* out)
{
    Inst& in = B->inst[i];
    atm::KArgs a;
    atm_status st = make_args(&in.p, &in.o, B->ws + in.off, in.L.total, a);
    if (st) return st;
    char* base = B->ws + in.off;
    double* ya = (double*)(base + in.L.ya);
    double* yb = (double*)(base + in.L.yb);
    double* e = (double*)(base + in.L.e);
    const bool fcf = in.o.relax == 1;
    const bool skip = !in.mixed;
    in.S = a.s_tmpl;
    for (int ph = 0; ph < NPH; ++ph) {
        atm::KArgs k = a;
        k.u = in.u;
        k.cg_count = &k.hdr->cg_fine;
        switch (ph) {
            case PH_S0:
                k.mode = 0;
                k.y = ya;
                break;
            case PH_S2:
                k.mode = 2;
                k.aux = ya;
                k.y = yb;
                k.skip_unchanged = skip;
                k.skip_y_src = ya;
                break;
            case PH_TAU:
            case PH_C:
                k.y = fcf ? yb : ya;
                k.e = e;
                k.cg_count = &k.hdr->cg_coarse;
                break;
            case PH_S1:
                k.mode = 1;
                k.aux = e;
                k.y = ya;
                k.skip_unchanged = skip;
                k.skip_y_src = fcf ? yb : nullptr;
                break;
            default:
                k.y = ya;
                break;
        }
        out[ph * B->n + i] = k;
    }
    return ATM_OK;
}

// task tables (host), grouped by phase, class and strip template, in the chosen order
void build_tables(atm_batch* B, std::vector<Task>& tasks)
{
    tasks.clear();
    B->groups.clear();
    for (int ph = 0; ph < NPH; ++ph)
        for (int cls = 0; cls < NCLS; ++cls) {
            // distinct (body, tile) of this phase and class; tile = S, plus 256 for the small-grid form
            auto tile_of = [&](const Inst& in) {
                if (cls == CLS_1D) return 0;
                const int S = B->tiles ? in.S : 32;
                return S + ((S == 8 && in.p.nx <= 64) ? 256 : 0);
            };
            std::vector<std::pair<int, int>> keys;
            for (int i = 0; i < B->n; ++i) {
                const Inst& in = B->inst[i];
                if (in.cls != cls || phase_tasks(in, ph) == 0) continue;
                const std::pair<int, int> key((int)phase_body(in, ph), tile_of(in));
                if (std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
            }
            for (const auto& key : keys) {
                std::vector<std::pair<double, Task>> g;
                for (int i = 0; i < B->n; ++i) {
                    const Inst& in = B->inst[i];
                    if (in.cls != cls || (int)phase_body(in, ph) != key.first) continue;
                    if (tile_of(in) != key.second) continue;
                    const int nt = phase_tasks(in, ph);
                    const int first = (ph == PH_TAU || ((ph == PH_N0 || ph == PH_N) && !in.mixed)) ? 1 : 0;
                    for (int t = 0; t < nt; ++t) g.push_back({task_cost(in, ph, t + first), Task{i, t + first}});
                }
                if (B->order == 1)
                    std::stable_sort(g.begin(), g.end(),
                                     [](const std::pair<double, Task>& x, const std::pair<double, Task>& y) {
                                         return x.first > y.first;
                                     });
                Group gr;
                gr.phase = ph;
                gr.cls = cls;
                gr.S = key.second & 255;
                gr.small = key.second >= 256;
                gr.body = (Body)key.first;
                gr.task_off = tasks.size();
                gr.ntasks = (int)g.size();
                for (const auto& x : g) tasks.push_back(x.second);
                B->groups.push_back(gr);
            }
        }
}

atm_status upload_tables(atm_batch* B)
{
    std::vector<Task> tasks;
    build_tables(B, tasks);
    if (tasks.size() > B->max_tasks) return fail(ATM_ERR_WORKSPACE, "batch task tables exceed their reserved space");
    ATM_HIP(hipMemcpyAsync(B->tasks_dev, tasks.data(), tasks.size() * sizeof(Task), hipMemcpyHostToDevice, B->main));
    ATM_HIP(hipStreamSynchronize(B->main));
    return ATM_OK;
}

// launches of the given phases, one branch stream per class present, joined on the main stream; with a
// single class present they go to the main stream itself (no fork or join to record or replay)
atm_status enqueue_phases(atm_batch* B, const int* phases, int nphases)
{
    bool used[NCLS] = {false, false, false};
    for (int q = 0; q < nphases; ++q)
        for (const Group& g : B->groups)
            if (g.phase == phases[q]) used[g.cls] = true;
    int nused = 0;
    for (int c = 0; c < NCLS; ++c) nused += used[c] ? 1 : 0;
    const bool fork = nused > 1;
    if (fork) {
        ATM_HIP(hipEventRecord(B->fork, B->main));
        for (int c = 0; c < NCLS; ++c)
            if (used[c]) ATM_HIP(hipStreamWaitEvent(B->br[c], B->fork, 0));
    }
    for (int q = 0; q < nphases; ++q)
        for (const Group& g : B->groups) {
            if (g.phase != phases[q]) continue;
            atm::batch::Launch l;
            l.args = B->args_dev + (size_t)g.phase * B->n;
            l.tasks = B->tasks_dev + g.task_off;
            l.ntasks = g.ntasks;
            l.ctl = B->ctl_dev;
            l.nchunk = B->nchunk_dev;
            const bool per = g.cls == CLS_2DP;
            atm::batch::launch_tasks(g.body, g.S, per, g.small, l, fork ? B->br[g.cls] : B->main);
        }
    if (fork)
        for (int c = 0; c < NCLS; ++c)
            if (used[c]) {
                ATM_HIP(hipEventRecord(B->join[c], B->br[c]));
                ATM_HIP(hipStreamWaitEvent(B->main, B->join[c], 0));
            }
    return check_launch();
}

atm_status enqueue_cycle(atm_batch* B)
{
    static const int phases[] = {PH_S2, PH_TAU, PH_C, PH_S1, PH_N, PH_NF};
    atm_status st = enqueue_phases(B, phases, 6);
    if (st) return st;
    atm::batch::launch_decide(B->args_dev + (size_t)PH_NF * B->n, B->ctl_dev, B->hist_dev, kHistCap, B->n, false,
                              B->main);
    return check_launch();
}

uint64_t batch_key(const atm_batch* B)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t v) {
        for (int q = 0; q < 8; ++q) {
            h ^= (uint64_t)((v >> (8 * q)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    for (const Inst& in : B->inst) {
        mix(in.p.kind);
        mix(in.p.nx);
        mix(in.p.ny);
        mix(in.p.nt);
        mix(in.o.m);
        mix(in.o.k);
        mix(in.o.relax);
        mix(in.o.precision);
        mix(in.o.coarse_substeps);
    }
    return h;
}

bool cache_lookup(const atm_batch* B, uint64_t key, int& order, int& tiles)
{
    if (B->cache.empty()) return false;
    FILE* f = fopen(B->cache.c_str(), "r");
    if (!f) return false;
    unsigned long long k;
    int o, t;
    double ms;
    bool found = false;
    while (fscanf(f, "%llx %d %d %lf", &k, &o, &t, &ms) == 4)
        if (k == key) {
            order = o;
            tiles = t;
            found = true;
        }
    fclose(f);
    return found;
}

void cache_store(const atm_batch* B, uint64_t key, int order, int tiles, double ms)
{
    if (B->cache.empty()) return;
    FILE* f = fopen(B->cache.c_str(), "a");
    if (!f) return;
    fprintf(f, "%016llx %d %d %.4f\n", (unsigned long long)key, order, tiles, ms);
    fclose(f);
}

// Autotuner: time the window phase (it reads the iterate and writes only corrections, so it can be
// repeated) for every (task order, strip tile) choice; keep the fastest.  Needs the initial phase done.
atm_status autotune(atm_batch* B)
{
    const uint64_t key = batch_key(B);
    int order = 1, tiles = 1;
    if (cache_lookup(B, key, order, tiles)) {
        B->order = order;
        B->tiles = tiles;
        return upload_tables(B);
    }
    // the window phase reading the initial sweep's y (ya), so that its inputs are defined
    std::vector<atm::KArgs> probe(B->n);
    for (int i = 0; i < B->n; ++i) {
        ATM_HIP(hipMemcpy(&probe[i], B->args_dev + (size_t)PH_C * B->n + i, sizeof(atm::KArgs), hipMemcpyDeviceToHost));
        atm::KArgs k = probe[i];
        k.y = (double*)(B->ws + B->inst[i].off + B->inst[i].L.ya);
        probe[i] = k;
    }
    // a spare KArgs row: PH_TAU's slot is rewritten below and restored after
    std::vector<atm::KArgs> saved(B->n);
    ATM_HIP(hipMemcpy(saved.data(), B->args_dev + (size_t)PH_TAU * B->n, B->n * sizeof(atm::KArgs),
                      hipMemcpyDeviceToHost));
    // the timed windows add CG counts (and on stale data possibly a failure flag) to the headers:
    // keep the headers as the initial phase left them
    std::vector<atm::Header> hdrs(B->n);
    for (int i = 0; i < B->n; ++i)
        ATM_HIP(hipMemcpy(&hdrs[i], saved[i].hdr, sizeof(atm::Header), hipMemcpyDeviceToHost));
    hipEvent_t e0, e1;
    ATM_HIP(hipEventCreate(&e0));
    ATM_HIP(hipEventCreate(&e1));
    double best = 1e300;
    int best_o = 1, best_t = 1;
    const auto t_start = std::chrono::steady_clock::now();
    for (int o = 0; o < 2; ++o)
        for (int t = 0; t < 2; ++t) {
            B->order = o;
            B->tiles = t;
            atm_status st = upload_tables(B);
            if (st) return st;
            // run the window groups with the probe arguments placed in the PH_C row
            ATM_HIP(hipMemcpy(B->args_dev + (size_t)PH_C * B->n, probe.data(), B->n * sizeof(atm::KArgs),
                              hipMemcpyHostToDevice));
            double ms_min = 1e300;
            for (int rep = 0; rep < 2; ++rep) {
                static const int phases[] = {PH_C};
                ATM_HIP(hipEventRecord(e0, B->main));
                if ((st = enqueue_phases(B, phases, 1))) return st;
                ATM_HIP(hipEventRecord(e1, B->main));
                ATM_HIP(hipEventSynchronize(e1));
                float ms = 0.0f;
                ATM_HIP(hipEventElapsedTime(&ms, e0, e1));
                ms_min = std::min(ms_min, (double)ms);
            }
            if (ms_min < best) {
                best = ms_min;
                best_o = o;
                best_t = t;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // restore the cycle's window arguments
    std::vector<atm::KArgs> all((size_t)NPH * B->n);  // phase_args fills [phase][instance]
    for (int i = 0; i < B->n; ++i) {
        atm_status st = phase_args(B, i, all.data());
        if (st) return st;
    }
    ATM_HIP(hipMemcpy(B->args_dev + (size_t)PH_C * B->n, all.data() + (size_t)PH_C * B->n, B->n * sizeof(atm::KArgs),
                      hipMemcpyHostToDevice));
    ATM_HIP(hipMemcpy(B->args_dev + (size_t)PH_TAU * B->n, saved.data(), B->n * sizeof(atm::KArgs),
                      hipMemcpyHostToDevice));
    for (int i = 0; i < B->n; ++i)
        ATM_HIP(hipMemcpy(saved[i].hdr, &hdrs[i], sizeof(atm::Header), hipMemcpyHostToDevice));
    B->order = best_o;
    B->tiles = best_t;
    B->ms_tune = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    cache_store(B, key, best_o, best_t, best);
    return upload_tables(B);
}

}  // namespace batchhost

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

// ---------------------------------------------------------------------------
// the window phase without a workspace argument: its tables live in a static device array
// ---------------------------------------------------------------------------

namespace {

constexpr size_t kStaticScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

// One copy per GPU, held from the library's load until the process ends.  In host code the
// name stands for a host-side shadow, never for the device address: kernels get the address
// that hipGetSymbolAddress returns for the device in use.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device, looked up once per device
atm_status static_scratch(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(ATM_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(ATM_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return ATM_OK;
}

}  // namespace

size_t atm_static_scratch_bytes(void) { return kStaticScratchBytes; }

atm_status atm_coarse_solve_static(const atm_problem* prob, const atm_options* opts, const double* u, const double* y,
                                   double* e, void* stream)
{
    atm_status st = validate(prob, opts);
    if (st) return st;
    if (!u || !y || !e) return fail(ATM_ERR_INVALID_ARG, "null u, y or e");
    if (e == y) return fail(ATM_ERR_INVALID_ARG, "e and y must not alias");
    if (learned(opts) || three_level(opts))
        return fail(ATM_ERR_UNSUPPORTED, "the static window solve takes the two-level plain coarse propagator");
    if (large_grid(prob))
        return fail(ATM_ERR_UNSUPPORTED, "the static window solve takes grids of at most %d points per side",
                    atm::kMaxSide2D);
    if (prob->kind != ATM_HEAT1D && !spectral(prob, opts))
        return fail(ATM_ERR_UNSUPPORTED, "the static window solve takes Psi's direct solves only (coarse_solver 0 or 2)");
    const Layout L = coarse_layout(prob, opts);
    if (L.total > kStaticScratchBytes)
        return fail(ATM_ERR_WORKSPACE, "the window solve needs %zu bytes of scratch; the static scratch holds %zu",
                    L.total, kStaticScratchBytes);
    hipStream_t s = as_stream(stream);
    int dev = -1, sdev = -1;
    ATM_HIP(hipGetDevice(&dev));
    if (s) ATM_HIP(hipStreamGetDevice(s, &sdev));
    if (s && sdev != dev)
        return fail(ATM_ERR_INVALID_ARG, "stream of device %d while device %d is current", sdev, dev);
    void* ws = nullptr;
    if ((st = static_scratch(dev, &ws))) return st;
    atm::KArgs a;
    if ((st = make_args_in(prob, opts, ws, kStaticScratchBytes, L, a))) return st;
    atm::launch_reset(a.hdr, s);  // the header's counters start from zero in every call
    if ((st = check_launch())) return st;
    return do_coarse(a, (double*)u, (double*)y, e, s);
}

const char* atm_sweep_kernel(const atm_problem* prob, const atm_options* opts)
{
    if (validate(prob, opts) != ATM_OK) return "";
    if (prob->kind == ATM_HEAT1D) return "sweep1d_kernel";
    const bool mixed = opts->precision == 1;
    if (!large_grid(prob)) return mixed ? "sweep2d_mixed_kernel" : "sweep2d_kernel";
    if (!mixed) return "sweep_large_kernel";
    atm::KArgs a;
    memset(&a, 0, sizeof(a));
    a.large = 1;
    a.g.nx = prob->nx;
    a.g.ny = prob->ny;
    a.n = n_space(prob);
    a.NT = n_intervals(prob, opts);
    return atm::sweep_pair_pairs(a, sweep_tasks(prob, opts)) > 0 ? "sweep_pair_mixed_kernel" : "sweep_large_mixed_kernel";
}

const char* atm_coarse_kernel(const atm_problem* prob, const atm_options* opts)
{
    if (validate(prob, opts) != ATM_OK || opts->coarse_form == 3 || three_level(opts)) return "";
    if (prob->kind == ATM_HEAT1D) return "coarse1d_kernel";
    const int spec = spectral(prob, opts) ? (opts->coarse_solver == 2 ? 2 : 1) : 0;
    if (!large_grid(prob)) {
        if (spec == 2) return use_fas(prob, opts) ? "coarse2d_bf_fas_kernel" : "coarse2d_bf_kernel";
        return spec ? "coarse2d_spec_kernel" : "coarse2d_kernel";
    }
    atm::KArgs a;
    memset(&a, 0, sizeof(a));
    a.large = 1;
    a.spectral = spec;
    a.g.nx = prob->nx;
    a.g.ny = prob->ny;
    a.n = n_space(prob);
    a.NT = n_intervals(prob, opts);
    a.fas = use_fas(prob, opts) ? 1 : 0;
    a.substeps = opts->coarse_substeps;
    if (spec == 2) return atm::coarse_pair_pairs(a) > 0 ? "coarse_pair_bf_kernel" : "";
    return atm::coarse_pair_pairs(a) > 0 ? "coarse_pair_kernel" : "coarse_large_kernel";
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
    return header_status(h, a.maxit);
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
    const bool ml = three_level(opts);
    const atm::KArgs a1 = ml ? level1_args(a, prob, opts, L, base) : a;
    double* u1 = (double*)(base + L.u1);
    double* y1a = (double*)(base + L.y1a);
    double* y1b = (double*)(base + L.y1b);
    double* e2 = (double*)(base + L.e2);
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
    if (opts->nested == 1) {
        const auto t_setup = std::chrono::steady_clock::now();
        if ((st = nested_setup(a, a1, prob, opts, u, ya, e, u1, y1a, y1b, e2, s, S))) return st;
        ATM_HIP(hipStreamSynchronize(s));
        S.ms_setup = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_setup).count();
    }
    // the eigenbasis tables depend on the grid only: built once for every coarse solve below
    if ((a.spectral || a1.spectral) && !a.large) {
        atm::launch_spectral_tables(a.spectral ? a : a1, s);
        if ((st = check_launch())) return st;
    }
    // F-relax the initial guess, then its residual
    ATM_TIMED(kPhSweep, do_sweep(a, prob, opts, 0, u, nullptr, ya, s));
    if (st) return st;
    S.fine_steps += prob->nt;
    S.n_sweeps += 1;
    double res = 0.0;
    ATM_TIMED(kPhNorm, stop_norm(ya, &res));
    if (st == ATM_OK) st = T.collect();
    if (st == ATM_OK && hist && hist_cap > 0) hist[0] = res;
    // Buffers: the initial and every correction sweep write y_a (Phi of every last F-point); the
    // CF sweep reads y_a and writes y_b, which the windows then read.  The FP32 form's correction
    // sweep starts its y-steps from y_a's previous contents (y is in/out there).
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
        double* ycur = ya;
        if (opts->relax == 1) {
            // CF: C-points take Phi of their preceding F-point (held in y_a), then F-relax
            ycur = yb;
            ATM_TIMED(kPhSweep, do_sweep(a, prob, opts, 2, u, ya, yb, s, skip, ya));
            if (st) break;
            S.fine_steps += prob->nt;
            S.n_sweeps += 1;
        }
        if (use_learned) {
            ATM_TIMED(kPhCoarse, do_coarse_learned(a, L, ws, prob, opts, u, ycur, e, s));
            if (st) break;
            S.coarse_steps += window_psi_count(NT, opts->k) + NT;
            S.learned_cycles += 1;
        } else if (ml) {
            ATM_TIMED(kPhCoarse, do_lower_levels(a, a1, opts, u, ycur, u1, a.tau, y1a, y1b, e2, s, &S.coarse_steps));
            if (st) break;
        } else {
            ATM_TIMED(kPhCoarse, do_coarse(a, u, ycur, e, s, true));
            if (st) break;
            S.coarse_steps += window_psi_count(NT, opts->k) + (a.fas ? NT : 0);
        }
        // correction u_{pm} += e_p and F-interpolation; y_a receives Phi of every last F-point
        // (intervals that are skipped take theirs from y_b, the CF sweep's output)
        // (three levels: the fine C-points take level 1's values, i.e. u_{pm} += u1_p - v_p)
        if (ml)
            ATM_TIMED(kPhSweep, do_sweep(a, prob, opts, 2, u, u1, ya, s, skip, opts->relax == 1 ? yb : nullptr));
        else
            ATM_TIMED(kPhSweep, do_sweep(a, prob, opts, 1, u, e, ya, s, skip, opts->relax == 1 ? yb : nullptr));
        if (st) break;
        S.fine_steps += prob->nt;
        S.n_sweeps += 1;
        ++it;
        const double prev_res = res;
        ATM_TIMED(kPhNorm, stop_norm(ya, &res));
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
#undef ATM_TIMED
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

size_t atm_batch_workspace_bytes(int32_t n, const atm_problem* probs, const atm_options* opts)
{
    std::vector<batchhost::Inst> v;
    size_t total = 0;
    if (batchhost::describe(n, probs, opts, v, total) != ATM_OK) return 0;
    return total;
}

atm_status atm_batch_create(atm_batch** out, int32_t n, const atm_problem* probs, const atm_options* opts,
                            double* const* u, void* ws, size_t ws_bytes, const char* tune_cache)
{
    using namespace batchhost;
    if (!out) return fail(ATM_ERR_INVALID_ARG, "null out");
    *out = nullptr;
    std::vector<Inst> v;
    size_t total = 0;
    atm_status st = describe(n, probs, opts, v, total);
    if (st) return st;
    if (!u) return fail(ATM_ERR_INVALID_ARG, "null iterate array");
    for (int i = 0; i < n; ++i)
        if (!u[i]) return fail(ATM_ERR_INVALID_ARG, "instance %d: null iterate", i);
    if (!ws) return fail(ATM_ERR_INVALID_ARG, "null workspace");
    if (((uintptr_t)ws) % kAlign) return fail(ATM_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
    if (ws_bytes < total)
        return fail(ATM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, total);
    atm_batch* B = new atm_batch;
    B->n = n;
    B->inst = std::move(v);
    B->ws = (char*)ws;
    B->cache = tune_cache ? tune_cache : "";
    for (int i = 0; i < n; ++i) B->inst[i].u = u[i];
    size_t off = B->inst.back().off + align_up(B->inst.back().L.total);
    B->args_dev = (atm::KArgs*)(B->ws + off);
    off += align_up((size_t)NPH * n * sizeof(atm::KArgs));
    B->ctl_dev = (InstCtl*)(B->ws + off);
    off += align_up(n * sizeof(InstCtl));
    B->nchunk_dev = (int*)(B->ws + off);
    off += align_up(n * sizeof(int));
    B->hist_dev = (double*)(B->ws + off);
    off += align_up((size_t)n * kHistCap * sizeof(double));
    B->tasks_dev = (Task*)(B->ws + off);
    B->max_tasks = count_tasks(B->inst);
    auto cleanup = [&](atm_status s2) {
        delete B;
        return s2;
    };
    hipError_t he = hipStreamCreateWithFlags(&B->main, hipStreamNonBlocking);
    for (int c = 0; c < NCLS && he == hipSuccess; ++c) he = hipStreamCreateWithFlags(&B->br[c], hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&B->fork, hipEventDisableTiming);
    for (int c = 0; c < NCLS && he == hipSuccess; ++c) he = hipEventCreateWithFlags(&B->join[c], hipEventDisableTiming);
    if (he != hipSuccess) return cleanup(fail(ATM_ERR_DEVICE, "batch streams: %s", hipGetErrorString(he)));
    std::vector<atm::KArgs> args((size_t)NPH * n);
    std::vector<InstCtl> ctl(n);
    std::vector<int> nchunk(n);
    for (int i = 0; i < n; ++i) {
        if ((st = phase_args(B, i, args.data()))) return cleanup(st);
        ctl[i].active = 1;
        ctl[i].it = 0;
        ctl[i].status = ATM_NOT_CONVERGED;
        ctl[i].max_iter = B->inst[i].o.max_iter;
        ctl[i].tol = B->inst[i].o.tol;
        ctl[i].res = 0.0;
        nchunk[i] = B->inst[i].nchunk;
    }
    he = hipMemcpy(B->args_dev, args.data(), args.size() * sizeof(atm::KArgs), hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(B->ctl_dev, ctl.data(), n * sizeof(InstCtl), hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(B->nchunk_dev, nchunk.data(), n * sizeof(int), hipMemcpyHostToDevice);
    if (he != hipSuccess) return cleanup(fail(ATM_ERR_DEVICE, "batch arguments: %s", hipGetErrorString(he)));
    // eigenbasis tables of the instances whose Psi uses them (they depend on the grid only)
    for (int i = 0; i < n; ++i)
        if (args[(size_t)PH_C * n + i].spectral) atm::launch_spectral_tables(args[(size_t)PH_C * n + i], B->main);
    if ((st = check_launch())) return cleanup(st);
    if ((st = upload_tables(B))) return cleanup(st);
    *out = B;
    return ATM_OK;
}

atm_status atm_batch_run(atm_batch* B, int32_t use_graph, int32_t check_every, atm_status* status, atm_stats* stats,
                         double* hist, int32_t hist_cap, double* ms_solve, double* ms_tune, void* stream)
{
    using namespace batchhost;
    if (!B) return fail(ATM_ERR_INVALID_ARG, "null batch");
    if (check_every < 1) return fail(ATM_ERR_INVALID_ARG, "check_every must be >= 1");
    if (hist_cap < 0) return fail(ATM_ERR_INVALID_ARG, "hist_cap must be >= 0");
    atm_status st;
    hipStream_t caller = as_stream(stream);
    ATM_HIP(hipEventRecord(B->fork, caller));
    ATM_HIP(hipStreamWaitEvent(B->main, B->fork, 0));
    const auto t0 = std::chrono::steady_clock::now();
    // initial F-relaxation, its residual and the first decision
    atm::batch::launch_reset_headers(B->args_dev, B->ctl_dev, B->n, B->main);
    {
        static const int phases[] = {PH_S0, PH_N0, PH_NF0};
        if ((st = enqueue_phases(B, phases, 3))) return st;
        atm::batch::launch_decide(B->args_dev + (size_t)PH_NF0 * B->n, B->ctl_dev, B->hist_dev, kHistCap, B->n, true,
                                  B->main);
        if ((st = check_launch())) return st;
    }
    double tune = 0.0;
    if (!B->tuned) {
        ATM_HIP(hipStreamSynchronize(B->main));
        if ((st = autotune(B))) return st;
        B->tuned = true;
        tune = B->ms_tune;
    }
    if (use_graph && !B->exec) {
        ATM_HIP(hipStreamBeginCapture(B->main, hipStreamCaptureModeGlobal));
        st = enqueue_cycle(B);
        hipGraph_t g = nullptr;
        hipError_t he = hipStreamEndCapture(B->main, &g);
        if (st) return st;
        if (he != hipSuccess) return fail(ATM_ERR_DEVICE, "graph capture: %s", hipGetErrorString(he));
        B->graph = g;
        ATM_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    }
    int max_cycles = 0;
    for (const Inst& in : B->inst) max_cycles = std::max(max_cycles, in.o.max_iter);
    std::vector<InstCtl> ctl(B->n);
    int cycles = 0;
    for (;;) {
        ATM_HIP(hipMemcpyAsync(ctl.data(), B->ctl_dev, B->n * sizeof(InstCtl), hipMemcpyDeviceToHost, B->main));
        ATM_HIP(hipStreamSynchronize(B->main));
        bool any = false;
        for (const InstCtl& c : ctl) any = any || c.active;
        if (!any || cycles >= max_cycles) break;
        for (int r = 0; r < check_every && cycles < max_cycles; ++r, ++cycles) {
            if (use_graph) {
                ATM_HIP(hipGraphLaunch(B->exec, B->main));
            } else if ((st = enqueue_cycle(B))) {
                return st;
            }
        }
    }
    // paper-form residual of the precision-1 instances' results: every instance's pass is enqueued
    // (spread over the branch streams so that they overlap), then the headers are read
    std::vector<double> final_res(B->n);
    std::vector<int> pending;
    ATM_HIP(hipEventRecord(B->fork, B->main));
    for (int c = 0; c < NCLS; ++c) ATM_HIP(hipStreamWaitEvent(B->br[c], B->fork, 0));
    for (int i = 0; i < B->n; ++i) {
        final_res[i] = ctl[i].res;
        const Inst& in = B->inst[i];
        if (in.mixed && (ctl[i].status == ATM_OK || ctl[i].status == ATM_NOT_CONVERGED)) {
            atm::KArgs a;
            if ((st = make_args(&in.p, &in.o, B->ws + in.off, in.L.total, a))) return st;
            a.u = in.u;
            atm::launch_step_residual(a, sweep_tasks(&in.p, &in.o), B->br[pending.size() % NCLS]);
            pending.push_back(i);
        }
    }
    if ((st = check_launch())) return st;
    for (int c = 0; c < NCLS; ++c) {
        ATM_HIP(hipEventRecord(B->join[c], B->br[c]));
        ATM_HIP(hipStreamWaitEvent(B->main, B->join[c], 0));
    }
    ATM_HIP(hipStreamSynchronize(B->main));
    for (int i : pending) {
        const Inst& in = B->inst[i];
        atm::Header h;
        ATM_HIP(hipMemcpy(&h, B->ws + in.off + in.L.header, sizeof(h), hipMemcpyDeviceToHost));
        final_res[i] = sqrt(h.norm2);
        if (h.fail) ctl[i].status = ATM_ERR_INNER_SOLVE;
    }
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() - tune;
    atm_status worst = ATM_OK;
    for (int i = 0; i < B->n; ++i) {
        const Inst& in = B->inst[i];
        if (status) status[i] = ctl[i].status;
        if (ctl[i].status < 0) worst = ctl[i].status;
        else if (ctl[i].status == ATM_NOT_CONVERGED && worst == ATM_OK) worst = ATM_NOT_CONVERGED;
        if (stats) {
            atm::Header h;
            ATM_HIP(hipMemcpy(&h, B->ws + in.off + in.L.header, sizeof(h), hipMemcpyDeviceToHost));
            atm_stats S;
            memset(&S, 0, sizeof(S));
            S.iterations = ctl[i].it;
            S.final_residual = final_res[i];
            S.ms_total = ms;
            S.cg_fine = (int64_t)h.cg_fine;
            S.cg_coarse = (int64_t)h.cg_coarse;
            S.fine_steps_skipped = (int64_t)h.skipped;
            const int sweeps = 1 + ctl[i].it * (in.o.relax == 1 ? 2 : 1);
            S.n_sweeps = sweeps;
            S.fine_steps = (int64_t)sweeps * in.p.nt - S.fine_steps_skipped;
            S.coarse_steps = (int64_t)ctl[i].it * window_psi_count(n_intervals(&in.p, &in.o), in.o.k);
            stats[i] = S;
        }
        if (hist && hist_cap > 0) {
            const int cnt = std::min(std::min(hist_cap, kHistCap), ctl[i].it + 1);
            ATM_HIP(hipMemcpy(hist + (size_t)i * hist_cap, B->hist_dev + (size_t)i * kHistCap, cnt * sizeof(double),
                              hipMemcpyDeviceToHost));
        }
    }
    if (ms_solve) *ms_solve = ms;
    if (ms_tune) *ms_tune = tune;
    ATM_HIP(hipEventRecord(B->fork, B->main));
    ATM_HIP(hipStreamWaitEvent(caller, B->fork, 0));
    return worst;
}

int32_t atm_batch_tuning(const atm_batch* B, int32_t* order, int32_t* tiles)
{
    if (!B) return 0;
    if (order) *order = B->order;
    if (tiles) *tiles = B->tiles;
    return B->tuned ? 1 : 0;
}

void atm_batch_destroy(atm_batch* B) { delete B; }

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
