// Batched AT-MGRIT: task records, per-instance control and the launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "atm_kernels.hpp"

namespace atm {
namespace batch {

enum { kStOk = 0, kStNotConverged = 1, kStDiverged = -4, kStInner = -5 };

// one task: instance and interval / window / norm piece
struct Task {
    int inst, idx;
};

struct InstCtl {
    int active;  // cycles continue while 1
    int it;      // cycles applied
    int status;  // ATM_* status once inactive
    int max_iter;
    double tol;
    double res;  // latest stopping norm
};

// a batched launch: the arguments of every instance for this phase, its task table and the controls
struct Launch {
    const KArgs* args;  // [n_inst]
    const Task* tasks;
    int ntasks;
    const InstCtl* ctl;
    const int* nchunk;  // implicit-residual pieces per instance (2D norm)
};

enum Body {
    kSweep1D,
    kSweep2D,    // FP32 defect-correction sweep (precision 1)
    kSweep2D64,  // FP64 sweep (precision 0)
    kCoarse1D,
    kCoarse2D,
    kTau2D,
    kNormC,      // C-point residual pieces (FP64 forms)
    kNormI,      // implicit residual pieces (precision 1)
    kNormFinalC,
    kNormFinalI,
    kCoarse2DSpec,  // windows with Psi in the eigenbasis
    kTau2DSpec,
    kCoarse2DBf,    // windows with Psi in the eigenbasis on the BF16 matrix cores (linear form)
    kCoarse2DBfFas, // the same in the FAS form (in terms of e = w - v)
};

// launch body over the task table with strip template S (2D), periodic flag and small flag (every
// instance of the table has at most 64 columns; used with S = 8)
void launch_tasks(Body body, int S, bool per, bool small, const Launch& l, hipStream_t s);
// decision after the norm of every instance: history, status, activity
void launch_decide(const KArgs* args, InstCtl* ctl, double* hist, int hist_cap, int n_inst, bool first, hipStream_t s);
void launch_reset_headers(const KArgs* args, InstCtl* ctl, int n_inst, hipStream_t s);

}  // namespace batch
}  // namespace atm
