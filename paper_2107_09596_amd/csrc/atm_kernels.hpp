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
};

struct KArgs {
    // space-time data
    double* u;          // [nt+1][n]
    const double* aux;  // sweep modes 1 (e) and 2 (y of the previous sweep)
    double* y;          // sweep: out; coarse/tau/norm: in (Phi of the last F-point)
    double* e;          // coarse: out
    double* tau;        // FAS right-hand side, [N_T+1][n]
    double* partials;   // [N_T+1] norm partial sums
    Header* hdr;
    int* fail;
    unsigned long long* cg_count;
    // sizes
    int64_t nt, n, NT;
    int m, k, mode, fas, substeps, nx;
    int is1d, s_tmpl, exact;
    Grid2D g;
    StepCoef fine, coarse;
    double rtol2;         // squared CG tolerance of Phi
    double rtol2_coarse;  // squared CG tolerance of Psi
    int maxit;
};

void launch_reset(Header* h, hipStream_t s);
void launch_sweep(const KArgs& a, int64_t n_tasks, hipStream_t s);
void launch_tau(const KArgs& a, hipStream_t s);
void launch_coarse(const KArgs& a, hipStream_t s);
void launch_norm(const KArgs& a, hipStream_t s);
void launch_sequential(const KArgs& a, hipStream_t s);

}  // namespace atm
