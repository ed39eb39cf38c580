// woi_internal.h -- host-side helpers shared by the library's translation units (not part
// of the public C ABI).
#pragma once
#include <stdint.h>

#include "woi.h"
#include "woi_device.h"

namespace woi {

// Records the message returned by woi_last_error() and returns s.
woi_status set_error(woi_status s, const char* fmt, ...);
// Validation of one query for P points (the checks woi_estimate makes).
woi_status check_query(const woi_problem* p, int64_t P, const woi_query* q);
// The per-point estimate (plain or VR, batch_share 1) with its partial sums in a caller-given
// device buffer of partial_bytes bytes: the sample chunks are capped to fit it.  Allocates
// nothing: the problem must already be on the current device (INVALID_ARG otherwise).
woi_status estimate_into(const woi_problem* p, const double* points, int64_t P, const woi_query* q, double* mean,
                         double* se, double* grad, double* grad_se, double* partials, size_t partial_bytes,
                         uint64_t* counters, void* stream);
// Shared trajectories (batch_share > 1) of one validated query on an uploaded problem: per chunk
// the trajectory and evaluation launches, then the reduction, enqueued on `stream`.  seed_tab:
// device address of the Philox key (a cached graph refreshes it), or null for q->seed.
size_t shared_workspace_bytes(const woi_problem* p, int64_t P, const woi_query* q);
woi_status enqueue_shared(const woi_problem* p, const double* points, int64_t P, const woi_query* q, double* mean,
                          double* se, double* grad, double* grad_se, void* workspace, size_t workspace_bytes,
                          uint64_t* counters, const uint64_t* seed_tab, void* stream);
// Whether any interface of the problem is a triangle mesh (host state only).
bool problem_has_mesh(const woi_problem* p);

// A problem as the launch code sees it (uploading it to the current device if needed).
struct ProblemRef {
    const DevProblem* dev;     // device copy
    const DevProblem* host;    // host image of the same header
    int dim;
    uint64_t serial;           // unique per woi_problem_create in this process
};
woi_status problem_ref(woi_problem* p, ProblemRef* out);

}  // namespace woi
