// woi_batch_shared.hip -- the batch kernel's instantiations for launches whose instances all
// take the shared schedule (Alg. 3): the schedule's draws are then known to be wave-uniform
// at compile time.
#include "woi_batch_kernel.h"

namespace woi {

const void* pick_batch_shared(int dim, bool vr, bool fp32, bool count, int waves, bool lds) {
    return pick_batch<true>(dim, vr, fp32, count, waves, lds);
}

}  // namespace woi
