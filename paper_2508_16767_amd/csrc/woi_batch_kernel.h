// woi_batch_kernel.h -- the persistent batch kernel (a template), included by the two
// translation units that instantiate it: woi_batch.hip (samples with independent schedules)
// and woi_batch_shared.hip (one schedule per sample, shared by the wave's lanes: Alg. 3).
// Splitting the instantiations lets the two compile in parallel.
//
// The walks are those of the per-point kernel (Alg. 2, Alg. 3 with one schedule per
// sample, same Philox keys), so every sample of a batched instance equals the sample of
// a woi_estimate call with the same query.  What differs is the work distribution:
// uneven instances (N, P, W all vary) are cut into items (instance, 64-point tile,
// chunk of samples) listed largest-first, and a grid of resident workgroups pulls items
// from one atomic queue head until the list is exhausted.  The waves of a workgroup split
// an item's samples; their per-lane sums are added in wave order through the workgroup's
// own record in global memory (L2-resident, reused item after item; one turn per wave, each
// adding every field, where the few hundred bytes of LDS the staged polylines leave would
// need a turn per field) and written to the item's one partial slot, and the reduction merges
// the slots in chunk order, so the result does not depend on which workgroup ran which item.
#pragma once
#include "woi_walk.h"

namespace woi {

// SH: every instance of the launch takes the shared schedule, known at compile time.
// head, wg_sums, partials and counters are bp's, passed again as parameters the compiler may
// take as unaliased: the problem tables are then read with scalar loads where uniform.
template <typename R, int D, bool VR, bool COUNT, int WV, bool LDS, bool SH>
__global__ __launch_bounds__(64 * WV, (walk_waves_per_simd<R, D>())) void batch_kernel(
    BParams bp, uint32_t* __restrict__ head, double* __restrict__ wg_sums, double* __restrict__ partials,
    uint64_t* __restrict__ counters) {
    __shared__ uint32_t s_item;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int K = VR ? 2 : 1;
    uint32_t staged = 0xFFFFFFFFu;   // instance whose polylines are in LDS (workgroup-uniform)
    Counts tot{0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(head, 1u);
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();             // every wave has read s_item (and left the previous item)
        if (it >= bp.n_items) break;
        const BItem item = bp.items[it];
        const BInst& in = bp.inst[item.inst];
        const DevProblem* __restrict__ dp = uniform_global(in.dp);
        const R* __restrict__ pay = Pay<R>::base(dp);
        if constexpr (LDS) {
            if (in.lds && item.inst != staged) {
                stage_polylines(dp);
                staged = item.inst;
            }
        }
        KParams kp{};
        kp.dp = dp;
        const uint64_t key = bp.seeds[item.inst];
        kp.k0 = (uint32_t)key;
        kp.k1 = (uint32_t)(key >> 32);
        kp.M = in.M;
        kp.batch_share = 1;
        kp.shared_sched = in.shared_sched;
        kp.instance = in.instance;
        // this wave's share of the chunk
        const uint32_t a = bp.ctab[in.c0 + item.chunk], len = bp.ctab[in.c0 + item.chunk + 1] - a;
        const uint32_t s0 = a + (uint32_t)(((uint64_t)len * wv) / WV);
        const uint32_t s1 = a + (uint32_t)(((uint64_t)len * (wv + 1)) / WV);
        const int64_t p = (int64_t)item.tile * 64 + lane;
        const bool active = p < in.P;
        const int64_t pc = active ? p : in.P - 1;
        AccumSink<R, D> sink;
        sink.dp = dp;
        load_point<R, D>(in.points, pc, sink.xh, sink.xl);
        double S1 = 0, S2 = 0, G1[D], G2[D];
#pragma unroll
        for (int i = 0; i < D; ++i) { G1[i] = 0; G2[i] = 0; }
        Counts cnt{0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (uint32_t s = s0; s < s1; ++s) {
            const uint32_t w = (uint32_t)(in.first_sample + s);
            double F = 0, Gs[D];
#pragma unroll
            for (int i = 0; i < D; ++i) Gs[i] = 0;
            Start<R, D> st2[2];
            if constexpr (VR)
                vr_starts<R, D, LDS, SH>(dp, pay, kp, w, (uint32_t)pc, first_region<SH>(dp, kp, w, (uint32_t)pc), st2, cnt);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                walker<R, D, VR, LDS, AccumSink<R, D>, SH>(dp, pay, kp, w, (uint32_t)pc, k, sink, nullptr, cnt,
                                                         VR ? &st2[k] : nullptr);
                F += (double)(sink.F * (R)dp->N);
#pragma unroll
                for (int i = 0; i < D; ++i) Gs[i] += (double)(sink.G[i] * (R)dp->N);
            }
            S1 += F; S2 += F * F;
#pragma unroll
            for (int i = 0; i < D; ++i) { G1[i] += Gs[i]; G2[i] += Gs[i] * Gs[i]; }
        }
        // the waves' sums, added in wave order: wave r adds its own to the running record of
        // waves 0..r-1; the last wave writes the item's slot (fields of one lane 64 apart)
        {
            constexpr int NF = 2 + 2 * D;
            double v[NF];
            v[0] = S1; v[1] = S2;
#pragma unroll
            for (int i = 0; i < D; ++i) { v[2 + i] = G1[i]; v[2 + D + i] = G2[i]; }
            double* acc = wg_sums + (size_t)blockIdx.x * 64 * NF + lane;
            const uint64_t slot = in.slot0 + (uint64_t)item.tile * in.n_chunks + item.chunk;
            double* o = partials + slot * 64 * NF + lane;
            for (int r = 0; r < WV; ++r) {
                if (wv == r) {
                    if (r > 0) {
#pragma unroll
                        for (int f = 0; f < NF; ++f) v[f] = acc[64 * f] + v[f];
                    }
                    if (r < WV - 1) {
#pragma unroll
                        for (int f = 0; f < NF; ++f) acc[64 * f] = v[f];
                    } else if (active) {
#pragma unroll
                        for (int f = 0; f < NF; ++f) o[64 * f] = v[f];
                    }
                }
                if (r < WV - 1) __syncthreads();
            }
        }
        if (COUNT && active) {   // idle lanes of a ragged tile walk too, but are not counted
            tot.steps += cnt.steps; tot.redraws += cnt.redraws; tot.rejections += cnt.rejections;
            tot.caps += cnt.caps; tot.zero += cnt.zero; tot.nodes += cnt.nodes; tot.segs += cnt.segs;
            tot.other += cnt.other; tot.fb += cnt.fb;
        }
    }
    if constexpr (COUNT) {
        const uint32_t v[WOI_COUNTERS] = {tot.steps, tot.redraws, tot.rejections, tot.caps,
                                          tot.zero, tot.nodes, tot.segs, tot.other, tot.fb};
#pragma unroll
        for (int i = 0; i < WOI_COUNTERS; ++i) {
            const uint64_t s = wave_sum((uint64_t)v[i]);
            if (lane == 0 && s) atomicAdd((unsigned long long*)&counters[i], (unsigned long long)s);
        }
    }
}

// Function pointer of the instantiation for (dim, vr, fp32, count, waves, lds); null if none.
template <typename R, int D, bool VR, bool COUNT, int WV, bool LDS, bool SH>
static const void* batch_fn() {
    return reinterpret_cast<const void*>(&batch_kernel<R, D, VR, COUNT, WV, LDS, SH>);
}

template <typename R, bool COUNT, int WV, bool SH>
static const void* pick_r(int dim, bool vr, bool lds) {
    if (lds) {
        if (dim != 2) return nullptr;
        return vr ? batch_fn<R, 2, true, COUNT, WV, true, SH>() : batch_fn<R, 2, false, COUNT, WV, true, SH>();
    }
    if (vr) {
        switch (dim) {
            case 2: return batch_fn<R, 2, true, COUNT, WV, false, SH>();
            case 3: return batch_fn<R, 3, true, COUNT, WV, false, SH>();
            default: return nullptr;
        }
    }
    switch (dim) {
        case 2: return batch_fn<R, 2, false, COUNT, WV, false, SH>();
        case 3: return batch_fn<R, 3, false, COUNT, WV, false, SH>();
        case 4: return batch_fn<R, 4, false, COUNT, WV, false, SH>();
        case 5: return batch_fn<R, 5, false, COUNT, WV, false, SH>();
        case 6: return batch_fn<R, 6, false, COUNT, WV, false, SH>();
        case 7: return batch_fn<R, 7, false, COUNT, WV, false, SH>();
        case 8: return batch_fn<R, 8, false, COUNT, WV, false, SH>();
        default: return nullptr;
    }
}

template <bool COUNT, bool SH>
static const void* pick_c(int dim, bool vr, bool fp32, int waves, bool lds) {
    if (waves == 4) return fp32 ? pick_r<float, COUNT, 4, SH>(dim, vr, lds) : pick_r<double, COUNT, 4, SH>(dim, vr, lds);
    if (waves == 8) return fp32 ? pick_r<float, COUNT, 8, SH>(dim, vr, lds) : pick_r<double, COUNT, 8, SH>(dim, vr, lds);
    return nullptr;
}

template <bool SH>
static const void* pick_batch(int dim, bool vr, bool fp32, bool count, int waves, bool lds) {
    return count ? pick_c<true, SH>(dim, vr, fp32, waves, lds) : pick_c<false, SH>(dim, vr, fp32, waves, lds);
}

// Entry points of the two translation units.
const void* pick_batch_indep(int dim, bool vr, bool fp32, bool count, int waves, bool lds);
const void* pick_batch_shared(int dim, bool vr, bool fp32, bool count, int waves, bool lds);

}  // namespace woi
