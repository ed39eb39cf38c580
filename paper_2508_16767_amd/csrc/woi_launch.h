// woi_launch.h -- kernel parameter blocks and launchers (host <-> device boundary inside
// the library; not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "woi_device.h"

namespace woi {

// One estimation launch: grid.x covers points (one lane per point), grid.y covers
// chunks of `samples_per_thread` consecutive samples.
struct KParams {
    const DevProblem* dp;
    const double* points;          // [P*dim]
    int64_t P;
    uint64_t n_samples;            // samples per point (walkers, or walker pairs for VR)
    uint64_t first_sample;         // index of the first sample
    uint32_t samples_per_thread;
    uint32_t k0, k1;               // Philox key (seed)
    int M;
    int batch_share;
    int shared_sched;
    uint32_t instance;
    double* partials;              // [chunks][P][2 + 2 dim] or null
    double* traceF;                // per-walker values (trace mode) or null
    double* traceG;
    uint32_t* trace;
    uint64_t* counters;
};

struct RParams {
    const double* partials;
    int64_t P;
    int dim;
    int n_chunks;
    uint32_t samples_per_thread;
    uint64_t n_samples;
    double *mean, *se, *grad, *grad_se;
};

// Shared trajectories (batch_share B > 1).  Generation: lane = point group g < ng, grid.y
// splits the chunk's `ns` samples into runs of `spt`; trajectories go to `traj`
// (planes of ns * K * (M + 1) * ng elements, see StoreSink).  Evaluation: lane = point,
// grid.y = piece of `spt_e` samples; writes partials of piece (piece0 + blockIdx.y).
struct TParams {
    void* traj;                    // R-typed planes
    size_t plane;                  // elements per plane
    int ng;                        // point groups
    uint32_t ns;                   // samples in this chunk
    uint64_t chunk_first;          // first sample index of the chunk
    uint32_t spt;                  // generation: samples per thread
    uint32_t spt_e;                // evaluation: samples per piece
    int piece0;                    // global index of the chunk's first piece
};

hipError_t launch_traj(const KParams& kp, const TParams& tp, int dim, bool vr, bool fp32, unsigned lds_bytes,
                       hipStream_t s);
hipError_t launch_eval(const KParams& kp, const TParams& tp, int dim, bool vr, bool fp32, hipStream_t s);

// lds_bytes > 0 (dimension 2): polyline tables are staged in LDS; block must then be 512 threads
hipError_t launch_walk(const KParams& kp, int dim, bool vr, bool fp32, unsigned lds_bytes, dim3 grid, dim3 block,
                       hipStream_t s);
hipError_t launch_reduce(const RParams& rp, hipStream_t s);

}  // namespace woi
