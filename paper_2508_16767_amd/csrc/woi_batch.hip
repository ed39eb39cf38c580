// woi_batch.hip -- many Walk-on-Interfaces instances in one persistent launch: the batch
// kernel's instantiations for independent schedules, the reduction, and the launchers.
#include "woi_batch_kernel.h"

namespace woi {

const void* pick_batch_indep(int dim, bool vr, bool fp32, bool count, int waves, bool lds) {
    return pick_batch<false>(dim, vr, fp32, count, waves, lds);
}

// One wave per (instance, point) of the flattened point list: lane l merges the point's
// chunk slots l, l + 64, ... in order, then the lanes' triples are combined in a fixed
// butterfly.  Deterministic.
__global__ __launch_bounds__(256) void batch_reduce_kernel(BRParams rp) {
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= rp.n_points) return;   // wave-uniform
    int lo = 0, hi = rp.n_inst - 1;           // last instance with out0 <= q
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rp.inst[mid].out0 <= q) lo = mid;
        else hi = mid - 1;
    }
    const BInst& in = rp.inst[lo];
    const int64_t p = q - in.out0;
    const int D = rp.dim, W = 2 + 2 * D;
    const uint64_t tile = (uint64_t)(p >> 6), pl = (uint64_t)(p & 63);
    Moments f{0, 0, 0}, g[WOI_MAX_DIM];
    for (int i = 0; i < D; ++i) g[i] = Moments{0, 0, 0};
    for (uint32_t c = (uint32_t)lane; c < in.n_chunks; c += 64) {
        const uint32_t len = rp.ctab[in.c0 + c + 1] - rp.ctab[in.c0 + c];
        const double* o = rp.partials + (in.slot0 + tile * in.n_chunks + c) * 64 * W + pl;
        double r[2 + 2 * WOI_MAX_DIM];
        for (int k = 0; k < W; ++k) r[k] = o[64 * k];
        merge_partial(f, g, D, (double)len, r);
    }
    for (int o = 1; o < 64; o <<= 1) {
        f.combine(shfl_xor_moments(f, o));
        for (int i = 0; i < D; ++i) g[i].combine(shfl_xor_moments(g[i], o));
    }
    if (lane == 0) store_moments(f, g, D, p, in.mean, in.se, in.grad, in.grad_se);
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static const void* pick(int dim, bool vr, bool fp32, bool shared, bool count, int waves, bool lds) {
    return shared ? pick_batch_shared(dim, vr, fp32, count, waves, lds) : pick_batch_indep(dim, vr, fp32, count, waves, lds);
}

hipError_t launch_batch(const BParams& bp, int dim, bool vr, bool fp32, bool shared, int waves, unsigned grid,
                        unsigned smem, hipStream_t s) {
    const bool lds = smem > 0;
    const void* fn = pick(dim, vr, fp32, shared, bp.counters != nullptr, waves, lds);
    if (!fn) return hipErrorInvalidValue;
    if (lds) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
    }
    BParams arg = bp;
    uint32_t* head = bp.head;
    double* wg = bp.wg_sums;
    double* part = bp.partials;
    uint64_t* cnt = bp.counters;
    void* args[] = {&arg, &head, &wg, &part, &cnt};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * waves), args, smem, s);
}

int batch_blocks_per_cu(int dim, bool vr, bool fp32, bool shared, int waves, unsigned smem) {
    const bool lds = smem > 0;
    const void* fn = pick(dim, vr, fp32, shared, false, waves, lds);
    if (!fn) return 0;
    if (lds && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64 * waves, smem) != hipSuccess) return 0;
    return nb;
}

hipError_t launch_batch_reduce(const BRParams& rp, hipStream_t s) {
    hipLaunchKernelGGL(batch_reduce_kernel, dim3((unsigned)((rp.n_points + 3) / 4)), dim3(256), 0, s, rp);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace woi
