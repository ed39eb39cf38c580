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
