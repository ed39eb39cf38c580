// woi_kernels_shared.hip -- the walk kernels' instantiations for queries that take the shared
// schedule (Alg. 3): the schedule's draws are then known to be wave-uniform at compile time.
#include "woi_walk_kernels.h"

namespace woi {

hipError_t launch_walk_shared(const KParams& kp, int dim, bool vr, bool fp32, unsigned lds_bytes, dim3 grid, dim3 block,
                              hipStream_t s) {
    return launch_walk_sched<true>(kp, dim, vr, fp32, lds_bytes, grid, block, s);
}

hipError_t launch_traj_shared(const KParams& kp, const TParams& tp, int dim, bool vr, bool fp32, unsigned lds_bytes,
                              hipStream_t s) {
    return launch_traj_sched<true>(kp, tp, dim, vr, fp32, lds_bytes, s);
}

}  // namespace woi
