// woi_kernels.hip -- gfx950 kernels of the Walk-on-Interfaces estimator.
//
// Kernels of the shared-trajectory evaluation (eval_kernel) and the per-point reduction, the
// walk kernels' instantiations for independent schedules (the templates are in
// woi_walk_kernels.h, the walker in woi_walk.h), and the launchers.
#include "woi_walk_kernels.h"

namespace woi {

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
hipError_t launch_walk_indep(const KParams& kp, int dim, bool vr, bool fp32, unsigned lds_bytes, dim3 grid, dim3 block,
                             hipStream_t s) {
    return launch_walk_sched<false>(kp, dim, vr, fp32, lds_bytes, grid, block, s);
}

hipError_t launch_traj_indep(const KParams& kp, const TParams& tp, int dim, bool vr, bool fp32, unsigned lds_bytes,
                             hipStream_t s) {
    return launch_traj_sched<false>(kp, tp, dim, vr, fp32, lds_bytes, s);
}

hipError_t launch_traj(const KParams& kp, const TParams& tp, int dim, bool vr, bool fp32, unsigned lds_bytes,
                       hipStream_t s) {
    return kp.shared_sched ? launch_traj_shared(kp, tp, dim, vr, fp32, lds_bytes, s)
                           : launch_traj_indep(kp, tp, dim, vr, fp32, lds_bytes, s);
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
    return kp.shared_sched ? launch_walk_shared(kp, dim, vr, fp32, lds_bytes, grid, block, s)
                           : launch_walk_indep(kp, dim, vr, fp32, lds_bytes, grid, block, s);
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
