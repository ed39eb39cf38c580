// woi_kernels.hip -- gfx950 kernels of the Walk-on-Interfaces estimator.
//
// Kernels of the per-point path (walk_kernel), the shared-trajectory path (traj_kernel,
// eval_kernel) and the per-point reduction; the walker itself is in woi_walk.h.
#include "woi_walk.h"

namespace woi {

// LDS: in 2D, the polylines are staged in LDS (512-thread workgroups); in 3D, the kernel
// handles triangle-mesh interfaces (their tables stay in global memory), which the other 3D
// kernels leave out so that quadric-only problems keep their register budget.
template <typename R, int D, bool VR, bool COUNT, bool LDS>
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
        if constexpr (VR) vr_starts<R, D, LDS>(dp, pay, kp, w, group, first_region(dp, kp, w, group), st2, cnt);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            uint32_t* tr = nullptr;
            const size_t idx = ((size_t)pc * kp.n_samples + s) * K + k;
            if (kp.trace && active) tr = kp.trace + idx * (kp.M + 1);
            walker<R, D, VR, LDS>(dp, pay, kp, w, group, k, sink, tr, cnt, VR ? &st2[k] : nullptr);
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
template <typename R, int D, bool VR, bool LDS>
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
        if constexpr (VR) vr_starts<R, D, LDS>(dp, pay, kp, w, (uint32_t)gc, first_region(dp, kp, w, (uint32_t)gc), st2, cnt);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            StoreSink<R, D> sink;
            sink.base = planes + ((size_t)(s * K + k) * (kp.M + 1)) * tp.ng + gc;
            sink.plane = tp.plane;
            sink.ng = tp.ng;
            sink.M = kp.M;
            sink.on = active;
            walker<R, D, VR, LDS, StoreSink<R, D>>(dp, pay, kp, w, (uint32_t)gc, k, sink, nullptr, cnt,
                                                   VR ? &st2[k] : nullptr);
        }
    }
}

// Natural log scaled: lnk(x) * ln_scale = ln x.  FP32 uses the hardware log2.
template <typename R> struct LnK;
template <> struct LnK<double> {
    static __device__ __forceinline__ double lnk(double x) { return log(x); }
    static constexpr double scale = 1.0;
};
template <> struct LnK<float> {
    static __device__ __forceinline__ float lnk(float x) { return __log2f(x); }
    static constexpr float scale = 0.693147180559945309417232121458f;
};

// Evaluation: lane = point, workgroup = 256 consecutive points (groups g_lo..g_hi).  The
// workgroup's piece of tp.spt_e samples is a sequence of rows (sample, walker, step); tiles
// of tp.tile_rows rows are copied into LDS as records {c_F, c_G, y_0 .. y_{m-1}} per group,
// with c_F = N c times the Phi prefactor and c_G = -N c / |S^{m-1}|, and every lane then
// forms F = sum_i c_F phi_i and G = sum_i c_G (x - y_i) / r_i^m from LDS (records of one
// group are read by all its lanes at once).  Per-sample sums and squares are FP64.
template <typename R, int D, bool VR>
__global__ __launch_bounds__(256) void eval_kernel(KParams kp, TParams tp) {
    constexpr int K = VR ? 2 : 1;
    constexpr int S = (D + 2 + 3) & ~3;                 // record stride (elements)
    const DevProblem* __restrict__ dp = kp.dp;
    const int64_t p0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t p = p0 + threadIdx.x;
    const bool active = p < kp.P;
    const int64_t pc = active ? p : kp.P - 1;
    const int B = kp.batch_share;
    const int g_lo = (int)(p0 / B);
    const int nb = (int)((min(p0 + (int64_t)blockDim.x, kp.P) - 1) / B) - g_lo + 1;
    const int gl = (int)(pc / B) - g_lo;
    R xh[D], xl[D];
    load_point<R, D>(kp.points, pc, xh, xl);
    const int M1 = kp.M + 1;
    const R* __restrict__ planes = static_cast<const R*>(tp.traj);
    R* rec = reinterpret_cast<R*>(woi_smem);
    const R N = (R)dp->N;
    const R cf = (D == 2 ? R(-0.0795774715459476678844418816863) * LnK<R>::scale : Pay<R>::pc(dp)) * N;
    const R cg = -N / Pay<R>::ua(dp);
    const uint32_t s0 = blockIdx.y * tp.spt_e, s1 = min(s0 + tp.spt_e, tp.ns);
    const int rows = (int)(s1 - s0) * K * M1;
    const size_t row0 = (size_t)s0 * K * M1;           // first row of the piece in the planes
    double S1 = 0, S2 = 0, G1[D], G2[D], F = 0, Gs[D];
    R Fk = 0, Gk[D];
#pragma unroll
    for (int i = 0; i < D; ++i) { G1[i] = 0; G2[i] = 0; Gs[i] = 0; Gk[i] = 0; }
    int step = 0, walker = 0;                          // position of the current row
    for (int r0 = 0; r0 < rows; r0 += tp.tile_rows) {
        const int rn = min(tp.tile_rows, rows - r0);
        __syncthreads();                                // the previous tile is consumed
        // record e = r nb + gg; (r, gg) advance by (step_r, step_g) per stride of blockDim.x
        int r = (int)threadIdx.x / nb, gg = (int)threadIdx.x - r * nb;
        const int step_r = (int)blockDim.x / nb, step_g = (int)blockDim.x - step_r * nb;
        for (int e = threadIdx.x; e < rn * nb; e += blockDim.x) {
            const size_t src = (row0 + r0 + r) * tp.ng + g_lo + gg;
            const R c = planes[src];
            R* o = rec + (size_t)e * S;
            o[0] = c * cf;
            o[1] = c * cg;
#pragma unroll
            for (int d = 0; d < D; ++d) o[2 + d] = planes[(d + 1) * tp.plane + src];
            r += step_r;
            gg += step_g;
            if (gg >= nb) { gg -= nb; ++r; }
        }
        __syncthreads();
        const R* q = rec + (size_t)gl * S;
        for (int r = 0; r < rn; ++r, q += (size_t)nb * S) {
            R dv[D], r2 = 0;
#pragma unroll
            for (int d = 0; d < D; ++d) { dv[d] = (xh[d] - q[2 + d]) + xl[d]; r2 += dv[d] * dv[d]; }
            // |x - y| = 0: the term is skipped (its kernel powers are taken as 0, one select)
            const bool nz = r2 > R(0);
            R tg;
            if constexpr (D == 2) {
                const R lg = nz ? LnK<R>::lnk(r2) : R(0), rc = nz ? RO<R>::rcp(r2) : R(0);
                Fk = fma(q[0], lg, Fk);
                tg = q[1] * rc;
            } else {
                const R ir = nz ? RO<R>::rsq(r2) : R(0);
                const R ir2 = ir * ir;
                R pw = R(1);
#pragma unroll
                for (int i = 0; i < (D - 2) / 2; ++i) pw *= ir2;
                if constexpr (D % 2) pw *= ir;          // r^{2-m}
                Fk = fma(q[0], pw, Fk);
                tg = q[1] * pw * ir2;
            }
#pragma unroll
            for (int d = 0; d < D; ++d) Gk[d] = fma(tg, dv[d], Gk[d]);
            if (++step == M1) {                         // walker done (uniform branch)
                step = 0;
                F += (double)Fk;
                Fk = 0;
#pragma unroll
                for (int d = 0; d < D; ++d) { Gs[d] += (double)Gk[d]; Gk[d] = 0; }
                if (++walker == K) {                    // sample done
                    walker = 0;
                    S1 += F; S2 += F * F;
#pragma unroll
                    for (int d = 0; d < D; ++d) { G1[d] += Gs[d]; G2[d] += Gs[d] * Gs[d]; Gs[d] = 0; }
                    F = 0;
                }
            }
        }
    }
    if (active) {   // slot blockIdx.y: the same piece of every chunk, summed in chunk order
        double* o = kp.partials + ((size_t)blockIdx.y * kp.P + p) * (2 + 2 * D);
        if (tp.accumulate) {
            o[0] += S1; o[1] += S2;
#pragma unroll
            for (int i = 0; i < D; ++i) { o[2 + i] += G1[i]; o[2 + D + i] += G2[i]; }
        } else {
            o[0] = S1; o[1] = S2;
#pragma unroll
            for (int i = 0; i < D; ++i) { o[2 + i] = G1[i]; o[2 + D + i] = G2[i]; }
        }
    }
}

// Per-point merge of the slot partials: one wave per point; lane l merges slots l, l + 64, ...
// in order, then the lanes' triples are combined in a fixed butterfly.  Deterministic.
// Slot c holds full + min(spt, max(0, tail - c spt)) samples.
__global__ __launch_bounds__(256) void reduce_kernel(RParams rp) {
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= rp.P) return;
    const int D = rp.dim, W = 2 + 2 * D;
    Moments f{0, 0, 0}, g[WOI_MAX_DIM];
    for (int i = 0; i < D; ++i) g[i] = Moments{0, 0, 0};
    for (int c = lane; c < rp.n_chunks; c += 64) {
        const uint64_t lo = (uint64_t)c * rp.samples_per_thread;
        const uint64_t own = lo < rp.tail ? min((uint64_t)rp.samples_per_thread, rp.tail - lo) : 0;
        const uint64_t nc = rp.full + own;
        if (nc == 0) continue;
        merge_partial(f, g, D, (double)nc, rp.partials + ((size_t)c * rp.P + p) * W);
    }
    for (int o = 1; o < 64; o <<= 1) {
        f.combine(shfl_xor_moments(f, o));
        for (int i = 0; i < D; ++i) g[i].combine(shfl_xor_moments(g[i], o));
    }
    if (lane == 0) store_moments(f, g, D, p, rp.mean, rp.se, rp.grad, rp.grad_se);
}

// ----------------------------------------------------------------------------- launchers
// Lets `fn` take lds_budget() bytes of dynamic LDS on the current device (once per device and
// kernel; `done` is that kernel's per-device flag array).
static hipError_t allow_lds(const void* fn, bool* done) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (done[dev]) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_budget());
    if (e == hipSuccess) done[dev] = true;
    return e;
}

template <typename R, int D, bool VR, bool COUNT, bool LDS>
static hipError_t launch_walk_t(const KParams& kp, dim3 grid, dim3 block, unsigned smem, hipStream_t s) {
    if constexpr (LDS && D == 2) {
        static bool done[64] = {};
        const hipError_t e = allow_lds(reinterpret_cast<const void*>(&walk_kernel<R, D, VR, COUNT, LDS>), done);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((walk_kernel<R, D, VR, COUNT, LDS>), grid, block, smem, s, kp);
    return hipGetLastError();
}

template <typename R, bool COUNT>
static hipError_t launch_walk_c(const KParams& kp, int dim, bool vr, bool lds, dim3 grid, dim3 block, unsigned smem,
                                hipStream_t s) {
    if (dim == 3 && kp.mesh)   // the mesh-capable 3D kernel (no VR on meshes)
        return vr ? hipErrorInvalidValue : launch_walk_t<R, 3, false, COUNT, true>(kp, grid, block, 0, s);
    if (lds) {
        if (dim != 2) return hipErrorInvalidValue;
        return vr ? launch_walk_t<R, 2, true, COUNT, true>(kp, grid, block, smem, s)
                  : launch_walk_t<R, 2, false, COUNT, true>(kp, grid, block, smem, s);
    }
    if (vr) {
        switch (dim) {
            case 2: return launch_walk_t<R, 2, true, COUNT, false>(kp, grid, block, 0, s);
            case 3: return launch_walk_t<R, 3, true, COUNT, false>(kp, grid, block, 0, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (dim) {
        case 2: return launch_walk_t<R, 2, false, COUNT, false>(kp, grid, block, 0, s);
        case 3: return launch_walk_t<R, 3, false, COUNT, false>(kp, grid, block, 0, s);
        case 4: return launch_walk_t<R, 4, false, COUNT, false>(kp, grid, block, 0, s);
        case 5: return launch_walk_t<R, 5, false, COUNT, false>(kp, grid, block, 0, s);
        case 6: return launch_walk_t<R, 6, false, COUNT, false>(kp, grid, block, 0, s);
        case 7: return launch_walk_t<R, 7, false, COUNT, false>(kp, grid, block, 0, s);
        case 8: return launch_walk_t<R, 8, false, COUNT, false>(kp, grid, block, 0, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int D, bool VR, bool LDS>
static hipError_t launch_traj_t(const KParams& kp, const TParams& tp, unsigned smem, hipStream_t s) {
    const int bs = LDS ? 512 : 256;
    if constexpr (LDS && D == 2) {
        static bool done[64] = {};
        const hipError_t e = allow_lds(reinterpret_cast<const void*>(&traj_kernel<R, D, VR, LDS>), done);
        if (e != hipSuccess) return e;
    }
    if (tp.lg < 64 || tp.lg % 64 || bs % tp.lg) return hipErrorInvalidValue;
    const unsigned rows = (unsigned)(bs / tp.lg), runs = (unsigned)((tp.ns + tp.spt - 1) / tp.spt);
    const dim3 grid((unsigned)((tp.ng + tp.lg - 1) / tp.lg), (runs + rows - 1) / rows);
    hipLaunchKernelGGL((traj_kernel<R, D, VR, LDS>), grid, dim3(bs), smem, s, kp, tp);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_traj_r(const KParams& kp, const TParams& tp, int dim, bool vr, unsigned lds, hipStream_t s) {
    if (dim == 3 && kp.mesh) return vr ? hipErrorInvalidValue : launch_traj_t<R, 3, false, true>(kp, tp, 0, s);
    if (lds && dim == 2) return vr ? launch_traj_t<R, 2, true, true>(kp, tp, lds, s) : launch_traj_t<R, 2, false, true>(kp, tp, lds, s);
    if (vr) {
        switch (dim) {
            case 2: return launch_traj_t<R, 2, true, false>(kp, tp, 0, s);
            case 3: return launch_traj_t<R, 3, true, false>(kp, tp, 0, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (dim) {
        case 2: return launch_traj_t<R, 2, false, false>(kp, tp, 0, s);
        case 3: return launch_traj_t<R, 3, false, false>(kp, tp, 0, s);
        case 4: return launch_traj_t<R, 4, false, false>(kp, tp, 0, s);
        case 5: return launch_traj_t<R, 5, false, false>(kp, tp, 0, s);
        case 6: return launch_traj_t<R, 6, false, false>(kp, tp, 0, s);
        case 7: return launch_traj_t<R, 7, false, false>(kp, tp, 0, s);
        case 8: return launch_traj_t<R, 8, false, false>(kp, tp, 0, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_traj(const KParams& kp, const TParams& tp, int dim, bool vr, bool fp32, unsigned lds_bytes,
                       hipStream_t s) {
    return fp32 ? launch_traj_r<float>(kp, tp, dim, vr, lds_bytes, s) : launch_traj_r<double>(kp, tp, dim, vr, lds_bytes, s);
}

template <typename R, int D, bool VR>
static hipError_t launch_eval_t(const KParams& kp, const TParams& tp, hipStream_t s) {
    const int bs = EVAL_BLOCK;
    const dim3 grid((unsigned)((kp.P + bs - 1) / bs), (unsigned)((tp.ns + tp.spt_e - 1) / tp.spt_e));
    const unsigned smem = (unsigned)eval_lds_bytes(kp.batch_share, kp.P, D, tp.tile_rows, sizeof(R));
    if (smem > (unsigned)EVAL_LDS) return hipErrorInvalidValue;
    hipLaunchKernelGGL((eval_kernel<R, D, VR>), grid, dim3(bs), smem, s, kp, tp);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_eval_r(const KParams& kp, const TParams& tp, int dim, bool vr, hipStream_t s) {
    if (vr) {
        switch (dim) {
            case 2: return launch_eval_t<R, 2, true>(kp, tp, s);
            case 3: return launch_eval_t<R, 3, true>(kp, tp, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (dim) {
        case 2: return launch_eval_t<R, 2, false>(kp, tp, s);
        case 3: return launch_eval_t<R, 3, false>(kp, tp, s);
        case 4: return launch_eval_t<R, 4, false>(kp, tp, s);
        case 5: return launch_eval_t<R, 5, false>(kp, tp, s);
        case 6: return launch_eval_t<R, 6, false>(kp, tp, s);
        case 7: return launch_eval_t<R, 7, false>(kp, tp, s);
        case 8: return launch_eval_t<R, 8, false>(kp, tp, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_eval(const KParams& kp, const TParams& tp, int dim, bool vr, bool fp32, hipStream_t s) {
    return fp32 ? launch_eval_r<float>(kp, tp, dim, vr, s) : launch_eval_r<double>(kp, tp, dim, vr, s);
}

hipError_t launch_walk(const KParams& kp, int dim, bool vr, bool fp32, unsigned lds_bytes, dim3 grid, dim3 block,
                       hipStream_t s) {
    const bool lds = lds_bytes > 0 && dim == 2;
    if (kp.counters) {
        return fp32 ? launch_walk_c<float, true>(kp, dim, vr, lds, grid, block, lds_bytes, s)
                    : launch_walk_c<double, true>(kp, dim, vr, lds, grid, block, lds_bytes, s);
    }
    return fp32 ? launch_walk_c<float, false>(kp, dim, vr, lds, grid, block, lds_bytes, s)
                : launch_walk_c<double, false>(kp, dim, vr, lds, grid, block, lds_bytes, s);
}

int lds_budget() {
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
    if (!cache[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 64 * 1024;
        cache[dev] = v < LDS_BUDGET_MAX ? v : LDS_BUDGET_MAX;
    }
    return cache[dev];
}

hipError_t launch_reduce(const RParams& rp, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)((rp.P + 3) / 4)), dim3(256), 0, s, rp);
    return hipGetLastError();
}

}  // namespace woi
