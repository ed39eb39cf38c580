// woi_naive.hip -- the naive Walk-on-Interfaces estimator (Markov trees, Sec. 4.2) on gfx950.
//
// One observation is a Markov tree (Eq. naive_woi_estimator): roots y_(h0), uniform on every
// interface h0 (Eq. naive_woi_p0), and below every node (h0..hi), i < M, one child per next
// interface h_{i+1}, drawn from the node by the transition of Eq. naive_woi_p.  The tree's value
// is the sum over its nodes of w_i (prod_{m=1}^{i} alpha_{h_m}) Q T Phi(x, y), with Q, T of
// Eqs. naive_woi_Q and naive_woi_T and w_i = 1 - delta_{iM}/2.  The cost per tree is
// sum_{i=0}^{M} N^{i+1} interface points, which is what the scheduled estimator avoids.
//
// GPU mapping: wave = (point, chunk of trees); lane = leaf.  A leaf is a tuple (h0..hM), its
// index the base-N number with digits h0..hM (h0 most significant).  A lane walks its leaf's
// branch from the root; node (h0..hi) draws from the Philox counter
// (tree, point, NAIVE_TAG | id, step i), id = the base-(N+1) number with digits h0+1..hi+1,
// so the lanes sharing a prefix draw the same points: the branch reuse of the Markov tree,
// without a stack.  The node's term (and its counters) is taken by the one lane whose digits
// below h_i are all 0 (leaf index divisible by N^(M-i)); the wave then sums its lanes in a fixed
// butterfly, so results do not depend on scheduling.  Cost: (M + 1) N^(M+1) node draws per tree
// against the tree's N (N^(M+1) - 1) / (N - 1) nodes, i.e. at most a factor (M + 1)(N - 1)/N.
#include "woi_walk.h"

namespace woi {

constexpr uint32_t NAIVE_TAG = 0x80000000u;

__device__ __forceinline__ void add_counts(Counts& a, const Counts& b) {
    a.steps += b.steps; a.redraws += b.redraws; a.rejections += b.rejections; a.caps += b.caps;
    a.zero += b.zero; a.nodes += b.nodes; a.segs += b.segs; a.other += b.other; a.fb += b.fb;
}

// R: FP64, or FP32 walks (each node's term c Phi, c grad Phi in FP32, converted to FP64 before it
// joins the lane's sum; the tree's lane sum and the moments in FP64).  LDS: in 3D, the mesh-capable instantiation (nothing is staged in LDS by this kernel).
template <typename R, int D, bool LDS, bool COUNT>
__global__ __launch_bounds__(256, (walk_waves_per_simd<R, D>())) void naive_kernel(KParams kp, NParams np) {
    const DevProblem* __restrict__ dp = kp.dp;
    const R* __restrict__ pay = Pay<R>::base(dp);
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    if (p >= kp.P) return;   // wave-uniform: the kernel has no workgroup barrier
    const int M = kp.M;
    const uint32_t N = (uint32_t)dp->N;
    R xh[D], xl[D];
    load_point<R, D>(kp.points, p, xh, xl);
    const uint64_t s0 = (uint64_t)blockIdx.y * kp.samples_per_thread;
    const uint64_t s1 = min(s0 + (uint64_t)kp.samples_per_thread, kp.n_samples);
    double S1 = 0, S2 = 0, G1[D], G2[D];
#pragma unroll
    for (int i = 0; i < D; ++i) { G1[i] = 0; G2[i] = 0; }
    Counts cnt{0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t s = s0; s < s1; ++s) {
        const uint32_t w = (uint32_t)(kp.first_sample + s);
        double Fl = 0, Gl[D];
#pragma unroll
        for (int i = 0; i < D; ++i) Gl[i] = 0;
        for (uint32_t leaf = lane; leaf < np.leaves; leaf += 64) {
            uint32_t span = np.span0, id = 0;
            int hp = 0, seg = 0;
            R y[D], Q = 0, T = 1, A = 1;
#pragma unroll
            for (int i = 0; i < D; ++i) y[i] = 0;
            for (int i = 0; i <= M; ++i) {
                const uint32_t pre = leaf / span;          // digits h0..hi
                const int h = (int)(pre % N);
                const bool counted = leaf == pre * span;   // digits below h_i all 0
                id = id * (N + 1) + (uint32_t)(h + 1);
                const Stream st{kp.k0, kp.k1, w, (uint32_t)p, NAIVE_TAG | id};
                const DevRegion* g = &dp->reg[h];
                Counts c{0, 0, 0, 0, 0, 0, 0, 0, 0};
                bool alive = true;
                if (i == 0) {   // y_0 uniform on dOmega_{h0}: Q = beta(y_0) |dOmega_{h0}|
                    int att;
                    for (att = 0; att < WOI_ATTEMPT_CAP; ++att) {
                        if (surf_attempt<R, D, LDS>(dp, *g, pay, st, 0u, att, y, seg)) break;
                        c.rejections++;
                    }
                    if (att == WOI_ATTEMPT_CAP) c.caps++;
                    Q = Pay<R>::s(*g) * data_b<R, D, LDS>(dp, *g, pay, y, seg) * Pay<R>::area(*g);
                } else {
                    R yn[D];
                    int segn = 0, qn = 1, pick = 0, att = 0;
                    const R tf = transition<R, D, LDS>(dp, pay, g, dp->rel[hp][h], st, (uint32_t)i, y, seg, yn, segn,
                                                       Q, qn, pick, att, c);
                    if (tf == R(0)) {
                        alive = false;   // no hit within the attempt cap: the subtree contributes nothing
                    } else {
                        T *= tf;
                        A *= (R)g->alpha;
#pragma unroll
                        for (int j = 0; j < D; ++j) y[j] = yn[j];
                        seg = segn;
                    }
                }
                if (counted) {
                    if (alive) {
                        R Fn = 0, Gn[D];
#pragma unroll
                        for (int j = 0; j < D; ++j) Gn[j] = 0;
                        add_term<R, D>(dp, xh, xl, y, (i == M ? R(0.5) : R(1)) * A * Q * T, Fn, Gn, c);
                        Fl += (double)Fn;
#pragma unroll
                        for (int j = 0; j < D; ++j) Gl[j] += (double)Gn[j];
                        c.steps++;
                    }
                    if constexpr (COUNT) add_counts(cnt, c);
                }
                if (!alive) break;
                hp = h;
                span /= N;
            }
        }
        // the tree's value: lanes summed in FP64 in a fixed butterfly (every lane ends with the same sum)
        double F = Fl, G[D];
#pragma unroll
        for (int i = 0; i < D; ++i) G[i] = Gl[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            F += __shfl_xor(F, o, 64);
#pragma unroll
            for (int i = 0; i < D; ++i) G[i] += __shfl_xor(G[i], o, 64);
        }
        if (kp.traceF && lane == 0) {
            const size_t idx = (size_t)p * kp.n_samples + s;
            kp.traceF[idx] = F;
            if (kp.traceG)
#pragma unroll
                for (int i = 0; i < D; ++i) kp.traceG[idx * D + i] = G[i];
        }
        S1 += F; S2 += F * F;
#pragma unroll
        for (int i = 0; i < D; ++i) { G1[i] += G[i]; G2[i] += G[i] * G[i]; }
    }
    if (kp.partials && lane == 0) {
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
            const uint64_t t = wave_sum((uint64_t)v[i]);
            if (lane == 0 && t) atomicAdd((unsigned long long*)&kp.counters[i], (unsigned long long)t);
        }
    }
}

template <typename R, int D, bool LDS, bool COUNT>
static hipError_t launch_naive_t(const KParams& kp, const NParams& np, dim3 grid, hipStream_t s) {
    hipLaunchKernelGGL((naive_kernel<R, D, LDS, COUNT>), grid, dim3(256), 0, s, kp, np);
    return hipGetLastError();
}

template <typename R, bool COUNT>
static hipError_t launch_naive_c(const KParams& kp, const NParams& np, int dim, dim3 grid, hipStream_t s) {
    if (dim == 3 && kp.mesh) return launch_naive_t<R, 3, true, COUNT>(kp, np, grid, s);
    switch (dim) {
        case 2: return launch_naive_t<R, 2, false, COUNT>(kp, np, grid, s);
        case 3: return launch_naive_t<R, 3, false, COUNT>(kp, np, grid, s);
        case 4: return launch_naive_t<R, 4, false, COUNT>(kp, np, grid, s);
        case 5: return launch_naive_t<R, 5, false, COUNT>(kp, np, grid, s);
        case 6: return launch_naive_t<R, 6, false, COUNT>(kp, np, grid, s);
        case 7: return launch_naive_t<R, 7, false, COUNT>(kp, np, grid, s);
        case 8: return launch_naive_t<R, 8, false, COUNT>(kp, np, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_naive(const KParams& kp, const NParams& np, int dim, bool fp32, dim3 grid, hipStream_t s) {
    if (fp32)
        return kp.counters ? launch_naive_c<float, true>(kp, np, dim, grid, s) : launch_naive_c<float, false>(kp, np, dim, grid, s);
    return kp.counters ? launch_naive_c<double, true>(kp, np, dim, grid, s) : launch_naive_c<double, false>(kp, np, dim, grid, s);
}

}  // namespace woi
