// woi_walk_kernels.h -- the walk kernels of the per-point path (walk_kernel) and the
// shared-trajectory generation (traj_kernel) with their launchers, as templates.  The two
// translation units that include this file instantiate them for queries with independent
// schedules (woi_kernels.hip) and for the shared schedule (woi_kernels_shared.hip, Alg. 3),
// so that the two compile in parallel.
#pragma once
#include "woi_walk.h"

namespace woi {

// LDS: in 2D, the polylines are staged in LDS (512-thread workgroups); in 3D, the kernel
// handles triangle-mesh interfaces (their tables stay in global memory), which the other 3D
// kernels leave out so that quadric-only problems keep their register budget.  SH: the query
// takes the shared schedule (the kernel is compiled for it).
template <typename R, int D, bool VR, bool COUNT, bool LDS, bool SH>
__global__ __launch_bounds__(LDS ? 512 : 256, (walk_waves_per_simd<R, D>())) void walk_kernel(KParams kp) {
    const DevProblem* __restrict__ dp = kp.dp;
    const R* __restrict__ pay = Pay<R>::base(dp);
    if constexpr (LDS && D == 2) stage_polylines(dp);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = p < kp.P;
    const int64_t pc = active ? p : kp.P - 1;
    AccumSink<R, D> sink;
    sink.dp = dp;
    load_point<R, D>(kp.points, pc, sink.xh, sink.xl);
    const uint32_t group = (uint32_t)(pc / kp.batch_share);
    const uint64_t s0 = (uint64_t)blockIdx.y * kp.samples_per_thread;
    const uint64_t s1 = min(s0 + (uint64_t)kp.samples_per_thread, kp.n_samples);
    double S1 = 0, S2 = 0, G1[D], G2[D];
#pragma unroll
    for (int i = 0; i < D; ++i) { G1[i] = 0; G2[i] = 0; }
    Counts cnt{0, 0, 0, 0, 0, 0, 0, 0, 0};
    constexpr int K = VR ? 2 : 1;
    for (uint64_t s = s0; s < s1; ++s) {
        const uint32_t w = (uint32_t)(kp.first_sample + s);
        double F = 0, Gs[D];
#pragma unroll
        for (int i = 0; i < D; ++i) Gs[i] = 0;
        Start<R, D> st2[2];
        if constexpr (VR) vr_starts<R, D, LDS, SH>(dp, pay, kp, w, group, first_region<SH>(dp, kp, w, group), st2, cnt);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            uint32_t* tr = nullptr;
            const size_t idx = ((size_t)pc * kp.n_samples + s) * K + k;
            if (kp.trace && active) tr = kp.trace + idx * (kp.M + 1);
            walker<R, D, VR, LDS, AccumSink<R, D>, SH>(dp, pay, kp, w, group, k, sink, tr, cnt, VR ? &st2[k] : nullptr);
            const R Fk = sink.F * (R)dp->N;
            R Gk[D];
#pragma unroll
            for (int i = 0; i < D; ++i) Gk[i] = sink.G[i] * (R)dp->N;
            F += (double)Fk;
#pragma unroll
            for (int i = 0; i < D; ++i) Gs[i] += (double)Gk[i];
            if (kp.traceF && active) {
                kp.traceF[idx] = (double)Fk;
                if (kp.traceG)
#pragma unroll
                    for (int i = 0; i < D; ++i) kp.traceG[idx * D + i] = (double)Gk[i];
            }
        }
        S1 += F; S2 += F * F;
#pragma unroll
        for (int i = 0; i < D; ++i) { G1[i] += Gs[i]; G2[i] += Gs[i] * Gs[i]; }
    }
    if (active && kp.partials) {
        double* o = kp.partials + ((size_t)blockIdx.y * kp.P + p) * (2 + 2 * D);
        o[0] = S1; o[1] = S2;
#pragma unroll
        for (int i = 0; i < D; ++i) { o[2 + i] = G1[i]; o[2 + D + i] = G2[i]; }
    }
    if constexpr (COUNT) {
        const uint32_t v[WOI_COUNTERS] = {cnt.steps, cnt.redraws, cnt.rejections, cnt.caps,
                                          cnt.zero, cnt.nodes, cnt.segs, cnt.other, cnt.fb};
#pragma unroll
        for (int i = 0; i < WOI_COUNTERS; ++i) {
            const uint64_t s = wave_sum(active ? (uint64_t)v[i] : 0);
            if ((threadIdx.x & 63) == 0 && s) atomicAdd((unsigned long long*)&kp.counters[i], (unsigned long long)s);
        }
    }
}

// ----------------------------------------------------------------------------- shared trajectories
// Generation: lane = point group.  A workgroup row of tp.lg lanes (a multiple of 64, so a
// wave never leaves its row) walks one run of tp.spt consecutive samples; a workgroup holds
// blockDim.x / tp.lg rows.  All lanes of a wave share the walk index, so with the shared
// schedule the transition case and geometry record are wave-uniform.
template <typename R, int D, bool VR, bool LDS, bool SH>
__global__ __launch_bounds__(LDS ? 512 : 256, (walk_waves_per_simd<R, D>())) void traj_kernel(KParams kq, TParams tp) {
    KParams kp = kq;
    if (kq.seed_tab) {   // the key of a cached batch graph, refreshed before each launch
        const uint64_t key = *kq.seed_tab;
        kp.k0 = (uint32_t)key;
        kp.k1 = (uint32_t)(key >> 32);
    }
    const DevProblem* __restrict__ dp = kp.dp;
    const R* __restrict__ pay = Pay<R>::base(dp);
    if constexpr (LDS && D == 2) stage_polylines(dp);
    const int lg = tp.lg;
    const int row = __builtin_amdgcn_readfirstlane((int)threadIdx.x / lg);
    const int g = blockIdx.x * lg + (int)threadIdx.x % lg;
    const bool active = g < tp.ng;
    const int gc = active ? g : tp.ng - 1;
    constexpr int K = VR ? 2 : 1;
    R* planes = static_cast<R*>(tp.traj);
    const uint64_t first = ((uint64_t)blockIdx.y * (blockDim.x / lg) + row) * tp.spt;
    const uint32_t s0 = (uint32_t)min(first, (uint64_t)tp.ns), s1 = (uint32_t)min(first + tp.spt, (uint64_t)tp.ns);
    Counts cnt{0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t s = s0; s < s1; ++s) {
        const uint32_t w = (uint32_t)(kp.first_sample + tp.chunk_first + s);
        Start<R, D> st2[2];
        if constexpr (VR)
            vr_starts<R, D, LDS, SH>(dp, pay, kp, w, (uint32_t)gc, first_region<SH>(dp, kp, w, (uint32_t)gc), st2, cnt);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            StoreSink<R, D> sink;
            sink.base = planes + ((size_t)(s * K + k) * (kp.M + 1)) * tp.ng + gc;
            sink.plane = tp.plane;
            sink.ng = tp.ng;
            sink.M = kp.M;
            sink.on = active;
            walker<R, D, VR, LDS, StoreSink<R, D>, SH>(dp, pay, kp, w, (uint32_t)gc, k, sink, nullptr, cnt,
                                                       VR ? &st2[k] : nullptr);
        }
    }
}

// Lets `fn` take lds_budget() bytes of dynamic LDS on the current device (once per device and
// kernel; `done` is that kernel's per-device flag array).
static inline hipError_t allow_lds(const void* fn, bool* done) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (done[dev]) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_budget());
    if (e == hipSuccess) done[dev] = true;
    return e;
}

template <typename R, int D, bool VR, bool COUNT, bool LDS, bool SH>
static hipError_t launch_walk_t(const KParams& kp, dim3 grid, dim3 block, unsigned smem, hipStream_t s) {
    if constexpr (LDS && D == 2) {
        static bool done[64] = {};
        const hipError_t e = allow_lds(reinterpret_cast<const void*>(&walk_kernel<R, D, VR, COUNT, LDS, SH>), done);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((walk_kernel<R, D, VR, COUNT, LDS, SH>), grid, block, smem, s, kp);
    return hipGetLastError();
}

template <typename R, bool COUNT, bool SH>
static hipError_t launch_walk_c(const KParams& kp, int dim, bool vr, bool lds, dim3 grid, dim3 block, unsigned smem,
                                hipStream_t s) {
    if (dim == 3 && kp.mesh)   // the mesh-capable 3D kernel (no VR on meshes)
        return vr ? hipErrorInvalidValue : launch_walk_t<R, 3, false, COUNT, true, SH>(kp, grid, block, 0, s);
    if (lds) {
        if (dim != 2) return hipErrorInvalidValue;
        return vr ? launch_walk_t<R, 2, true, COUNT, true, SH>(kp, grid, block, smem, s)
                  : launch_walk_t<R, 2, false, COUNT, true, SH>(kp, grid, block, smem, s);
    }
    if (vr) {
        switch (dim) {
            case 2: return launch_walk_t<R, 2, true, COUNT, false, SH>(kp, grid, block, 0, s);
            case 3: return launch_walk_t<R, 3, true, COUNT, false, SH>(kp, grid, block, 0, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (dim) {
        case 2: return launch_walk_t<R, 2, false, COUNT, false, SH>(kp, grid, block, 0, s);
        case 3: return launch_walk_t<R, 3, false, COUNT, false, SH>(kp, grid, block, 0, s);
        case 4: return launch_walk_t<R, 4, false, COUNT, false, SH>(kp, grid, block, 0, s);
        case 5: return launch_walk_t<R, 5, false, COUNT, false, SH>(kp, grid, block, 0, s);
        case 6: return launch_walk_t<R, 6, false, COUNT, false, SH>(kp, grid, block, 0, s);
        case 7: return launch_walk_t<R, 7, false, COUNT, false, SH>(kp, grid, block, 0, s);
        case 8: return launch_walk_t<R, 8, false, COUNT, false, SH>(kp, grid, block, 0, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int D, bool VR, bool LDS, bool SH>
static hipError_t launch_traj_t(const KParams& kp, const TParams& tp, unsigned smem, hipStream_t s) {
    const int bs = LDS ? 512 : 256;
    if constexpr (LDS && D == 2) {
        static bool done[64] = {};
        const hipError_t e = allow_lds(reinterpret_cast<const void*>(&traj_kernel<R, D, VR, LDS, SH>), done);
        if (e != hipSuccess) return e;
    }
    if (tp.lg < 64 || tp.lg % 64 || bs % tp.lg) return hipErrorInvalidValue;
    const unsigned rows = (unsigned)(bs / tp.lg), runs = (unsigned)((tp.ns + tp.spt - 1) / tp.spt);
    const dim3 grid((unsigned)((tp.ng + tp.lg - 1) / tp.lg), (runs + rows - 1) / rows);
    hipLaunchKernelGGL((traj_kernel<R, D, VR, LDS, SH>), grid, dim3(bs), smem, s, kp, tp);
    return hipGetLastError();
}

template <typename R, bool SH>
static hipError_t launch_traj_r(const KParams& kp, const TParams& tp, int dim, bool vr, unsigned lds, hipStream_t s) {
    if (dim == 3 && kp.mesh) return vr ? hipErrorInvalidValue : launch_traj_t<R, 3, false, true, SH>(kp, tp, 0, s);
    if (lds && dim == 2) return vr ? launch_traj_t<R, 2, true, true, SH>(kp, tp, lds, s) : launch_traj_t<R, 2, false, true, SH>(kp, tp, lds, s);
    if (vr) {
        switch (dim) {
            case 2: return launch_traj_t<R, 2, true, false, SH>(kp, tp, 0, s);
            case 3: return launch_traj_t<R, 3, true, false, SH>(kp, tp, 0, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (dim) {
        case 2: return launch_traj_t<R, 2, false, false, SH>(kp, tp, 0, s);
        case 3: return launch_traj_t<R, 3, false, false, SH>(kp, tp, 0, s);
        case 4: return launch_traj_t<R, 4, false, false, SH>(kp, tp, 0, s);
        case 5: return launch_traj_t<R, 5, false, false, SH>(kp, tp, 0, s);
        case 6: return launch_traj_t<R, 6, false, false, SH>(kp, tp, 0, s);
        case 7: return launch_traj_t<R, 7, false, false, SH>(kp, tp, 0, s);
        case 8: return launch_traj_t<R, 8, false, false, SH>(kp, tp, 0, s);
        default: return hipErrorInvalidValue;
    }
}

template <bool SH>
static hipError_t launch_traj_sched(const KParams& kp, const TParams& tp, int dim, bool vr, bool fp32, unsigned lds_bytes,
                                    hipStream_t s) {
    return fp32 ? launch_traj_r<float, SH>(kp, tp, dim, vr, lds_bytes, s)
                : launch_traj_r<double, SH>(kp, tp, dim, vr, lds_bytes, s);
}

template <bool SH>
static hipError_t launch_walk_sched(const KParams& kp, int dim, bool vr, bool fp32, unsigned lds_bytes, dim3 grid,
                                    dim3 block, hipStream_t s) {
    const bool lds = lds_bytes > 0 && dim == 2;
    if (kp.counters) {
        return fp32 ? launch_walk_c<float, true, SH>(kp, dim, vr, lds, grid, block, lds_bytes, s)
                    : launch_walk_c<double, true, SH>(kp, dim, vr, lds, grid, block, lds_bytes, s);
    }
    return fp32 ? launch_walk_c<float, false, SH>(kp, dim, vr, lds, grid, block, lds_bytes, s)
                : launch_walk_c<double, false, SH>(kp, dim, vr, lds, grid, block, lds_bytes, s);
}

// Entry points of the two translation units: launch_walk / launch_traj for one schedule mode.
hipError_t launch_walk_indep(const KParams& kp, int dim, bool vr, bool fp32, unsigned lds_bytes, dim3 grid, dim3 block,
                             hipStream_t s);
hipError_t launch_walk_shared(const KParams& kp, int dim, bool vr, bool fp32, unsigned lds_bytes, dim3 grid, dim3 block,
                              hipStream_t s);
hipError_t launch_traj_indep(const KParams& kp, const TParams& tp, int dim, bool vr, bool fp32, unsigned lds_bytes,
                             hipStream_t s);
hipError_t launch_traj_shared(const KParams& kp, const TParams& tp, int dim, bool vr, bool fp32, unsigned lds_bytes,
                              hipStream_t s);

}  // namespace woi
