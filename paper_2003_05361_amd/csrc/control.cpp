// What the host does after a persistent launch has ended for one right-hand
// side (no GPU code).
//
// Sec. 3.3.2: the asynchronous iteration stops on a detector that only sees
// local criteria and latest (mixed-time) residuals, so the global criterion
// ||b - A x|| < tol ||b|| is verified exactly once the kernel has returned; if
// it fails, the iteration resumes from the current x.  Limits (local-solve
// count, wall time) and a non-finite or overflowing residual end the solve
// with a warning or an error instead.
#include <cmath>

#include "../../include/ras.h"

extern "C" int32_t ras_async_next_step(int32_t kernel_stop, double verified_relres, double tol,
                                       int64_t min_local_solves, int64_t max_sweeps, double elapsed_seconds,
                                       double max_seconds, int32_t ordered) {
    // the kernel saw a non-finite or overflowing residual sum, or the exact check did
    if (kernel_stop == RAS_KSTOP_DIVERGED || !std::isfinite(verified_relres)) return RAS_STEP_DIVERGED;
    if (verified_relres < tol) return RAS_STEP_CONVERGED;
    const bool exhausted = min_local_solves >= max_sweeps;
    const bool timed = kernel_stop == RAS_KSTOP_TIME || (max_seconds > 0.0 && elapsed_seconds > max_seconds);
    // the ordered mode runs its fixed number of passes once
    if (exhausted || timed || ordered) return RAS_STEP_LIMIT;
    return RAS_STEP_RESUME;
}

extern "C" ras_status ras_final_status(int32_t step) {
    switch (step) {
        case RAS_STEP_CONVERGED: return RAS_OK;
        case RAS_STEP_DIVERGED: return RAS_E_DIVERGED;
        case RAS_STEP_LIMIT: return RAS_NOT_CONVERGED;
        default: return RAS_E_STATE;  // a resumed solve has no final status yet
    }
}
