// woi_walk.h -- device code of one Walk-on-Interfaces walker (Philox streams, geometry,
// transitions, kernel evaluation), shared by the kernel translation units.
//
// Paper: Ding & Stinchcombe, "Walk-on-Interfaces", arXiv 2508.16767.
//   schedule H_0 ~ U{1..N}, H_i ~ |alpha|/||alpha||_1      Theorem 2, Eq. scheduled_interface_pdf
//   transitions (line / ray / uniform) and Q, T factors    Sec. 4.2.1-4.2.3, Eqs. naive_woi_p, _Q, _T
//   accumulation of w_i ||alpha||^i prod sign Q T Phi      Eq. woi_estimator, Alg. 2
//   two walkers on {beta >= 0} / {beta < 0}               Sec. 4.4, Alg. 3
//   gradient by grad_x Phi on the same walks               Sec. 4.5
//
// Mapping: one lane = one evaluation point, a thread loops over a chunk of samples
// (walk indices).  With the shared schedule the walk index -- and so the scheduled
// interface and the transition case -- is the same for all 64 lanes of a wave, so
// the case branch and the geometry record are wave-uniform (scalar loads/branches);
// only positions differ.  Every lane draws its own Philox4x32-10 counters keyed by
// (walk, point group, instance|walker|purpose, step|draw), so results do not depend
// on the launch shape.  Per-point sums are FP64 in every precision.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "woi_device.h"
#include "woi_launch.h"

namespace woi {

#define WOI_ATTEMPT_CAP 256

// ----------------------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw (SC'11): 10 rounds, multipliers 0xD2511F53 / 0xCD9E8D57,
// Weyl key increments 0x9E3779B9 / 0xBB67AE85.
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                       (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
    }
    return c;
}

// p, known to address global memory and to be the same in every lane, as the compiler should
// see it: loads through the result are global-memory loads from a scalar base (scalar loads
// where the address is uniform and no store of the kernel may alias them).
template <typename T>
__device__ __forceinline__ const T* uniform_global(const T* p) {
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (const T*)reinterpret_cast<const __attribute__((address_space(1))) T*>(((uint64_t)hi << 32) | lo);
}

struct Stream {
    uint32_t k0, k1, c0, c1, c2;
    __device__ __forceinline__ uint4 block(uint32_t step, uint32_t draw) const {
        return philox(make_uint4(c0, c1, c2, (step << 16) | (draw & 0xFFFFu)), k0, k1);
    }
};

// NW consecutive words of draws [first, ...): registers only (fully unrolled).
template <int NW>
struct Words {
    uint32_t w[NW];
    __device__ __forceinline__ void fill(const Stream& s, uint32_t step, uint32_t first) {
#pragma unroll
        for (int b = 0; b < (NW + 3) / 4; ++b) {
            const uint4 v = s.block(step, first + b);
            if (4 * b + 0 < NW) w[4 * b + 0] = v.x;
            if (4 * b + 1 < NW) w[4 * b + 1] = v.y;
            if (4 * b + 2 < NW) w[4 * b + 2] = v.z;
            if (4 * b + 3 < NW) w[4 * b + 3] = v.w;
        }
    }
    // Attempt words: the two words pre-drawn for the first attempt (2D transitions: one block
    // serves steps 2k+1 and 2k+2, counter word 3 = (0x8000 | k) << 16), else draws from `first`.
    __device__ __forceinline__ void take(const Stream& s, uint32_t step, uint32_t first, const uint32_t* pre) {
        if (pre && first == 0 && NW <= 2) {
#pragma unroll
            for (int i = 0; i < NW && i < 2; ++i) w[i] = pre[i];
        } else {
            fill(s, step, first);
        }
    }
};

// ----------------------------------------------------------------------------- precision
template <typename R> struct RO;
template <> struct RO<double> {
    static __device__ __forceinline__ double u(uint32_t v) { return ((double)v + 0.5) * 0x1p-32; }
    static __device__ __forceinline__ void sc2pi(double u, double& s, double& c) { sincospi(2.0 * u, &s, &c); }
    static __device__ __forceinline__ double lg(double x) { return log(x); }
    static __device__ __forceinline__ double sq(double x) { return sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
    static constexpr double line_eps = 1e-12;   // |t| below which a polyline hit is y itself
    static constexpr double ray_eps = 0.0;
};
template <> struct RO<float> {
    static __device__ __forceinline__ float u(uint32_t v) { return (float)((v >> 8) | 1u) * 0x1p-24f; }
    // v_sin_f32 / v_cos_f32 take their argument in revolutions
    static __device__ __forceinline__ void sc2pi(float u, float& s, float& c) {
        s = __builtin_amdgcn_sinf(u); c = __builtin_amdgcn_cosf(u);
    }
    // natural log from the hardware log2 (one instruction; __logf adds ten for denormal inputs and
    // an extended-precision ln 2).  FP32 walks take it of uniforms >= 2^-24 and of squared
    // distances, whose reciprocal they also form: below FLT_MIN that overflows either way.
    static __device__ __forceinline__ float lg(float x) { return __log2f(x) * 0.693147180559945309f; }
    // hardware square root (about 1 ulp; sqrtf adds a correctly rounded refinement, 17 instructions)
    static __device__ __forceinline__ float sq(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    // a / b to about 2 ulp (hardware reciprocal), for the FP32 walks
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
    static constexpr float line_eps = 1e-5f;   // FP32 line hits with |t| < POLY_T_BAND are decided in FP64
    static constexpr float ray_eps = 0.0f;
};

template <typename R> struct Pay;
template <> struct Pay<double> {
    static __device__ __forceinline__ const double* base(const DevProblem* dp) {
        return reinterpret_cast<const double*>(reinterpret_cast<const char*>(dp) + dp->off64);
    }
    static __device__ __forceinline__ int g(const DevRegion& r) { return r.g64; }
    static __device__ __forceinline__ int len(const DevRegion& r) { return r.len64; }
    static __device__ __forceinline__ int cum(const DevRegion& r) { return r.cum64; }
    static __device__ __forceinline__ int nrm(const DevRegion& r) { return r.nrm64; }
    static __device__ __forceinline__ int dat(const DevRegion& r) { return r.d64; }
    static __device__ __forceinline__ int brk(const DevRegion& r) { return r.b64; }
    static __device__ __forceinline__ double area(const DevRegion& r) { return r.area; }
    static __device__ __forceinline__ double meas(const DevRegion& r, int k) { return r.meas[k]; }
    static __device__ __forceinline__ double total(const DevRegion& r) { return r.total; }
    static __device__ __forceinline__ double gscale(const DevRegion& r) { return r.gscale; }
    static __device__ __forceinline__ double s(const DevRegion& r) { return r.s; }
    static __device__ __forceinline__ double sgn(const DevRegion& r) { return r.sgn; }
    static __device__ __forceinline__ double l1(const DevProblem* dp) { return dp->alpha_l1; }
    static __device__ __forceinline__ double ua(const DevProblem* dp) { return dp->unit_area; }
    static __device__ __forceinline__ double pc(const DevProblem* dp) { return dp->phi_c; }
};
template <> struct Pay<float> {
    static __device__ __forceinline__ const float* base(const DevProblem* dp) {
        return reinterpret_cast<const float*>(reinterpret_cast<const char*>(dp) + dp->off32);
    }
    static __device__ __forceinline__ int g(const DevRegion& r) { return r.g32; }
    static __device__ __forceinline__ int len(const DevRegion& r) { return r.len32; }
    static __device__ __forceinline__ int cum(const DevRegion& r) { return r.cum32; }
    static __device__ __forceinline__ int nrm(const DevRegion& r) { return r.nrm32; }
    static __device__ __forceinline__ int dat(const DevRegion& r) { return r.d32; }
    static __device__ __forceinline__ int brk(const DevRegion& r) { return r.b32; }
    static __device__ __forceinline__ float area(const DevRegion& r) { return r.area_f; }
    static __device__ __forceinline__ float meas(const DevRegion& r, int k) { return r.meas_f[k]; }
    static __device__ __forceinline__ float total(const DevRegion& r) { return r.total_f; }
    static __device__ __forceinline__ float gscale(const DevRegion& r) { return r.gscale_f; }
    static __device__ __forceinline__ float s(const DevRegion& r) { return r.s_f; }
    static __device__ __forceinline__ float sgn(const DevRegion& r) { return r.sgn_f; }
    static __device__ __forceinline__ float l1(const DevProblem* dp) { return dp->alpha_l1_f; }
    static __device__ __forceinline__ float ua(const DevProblem* dp) { return dp->unit_area_f; }
    static __device__ __forceinline__ float pc(const DevProblem* dp) { return dp->phi_c_f; }
};

struct Counts {
    uint32_t steps, redraws, rejections, caps, zero, nodes, segs, other, fb;
};

// Polyline tables staged by the workgroup (FP32 vertices, FP16 block bounds).
extern __shared__ __align__(16) char woi_smem[];

// Vertices of a polyline in precision R: the LDS copy when the kernel staged the polylines
// (FP32 only: the staged copy is the FP32 array itself), else the payload in global memory.
template <typename R, bool LDS>
__device__ __forceinline__ const R* poly_xy(const DevRegion& g, const R* __restrict__ pay) {
    if constexpr (LDS && std::is_same<R, float>::value) return reinterpret_cast<const R*>(woi_smem + g.lds_v);
    else return pay + Pay<R>::g(g);
}

constexpr int dir_words(int D) { return D == 2 ? 1 : (D == 3 ? 2 : 2 * ((D + 1) / 2)); }

// Resident waves per SIMD that the FP32 walk kernels keep (the register budget they are
// compiled to: 128 VGPRs for 4 waves): the FP64 recheck paths, rarely taken, would otherwise
// raise the allocation and cost a wave per SIMD.  FP64 kernels are left to the compiler.
template <typename R, int D>
constexpr int walk_waves_per_simd() { return std::is_same<R, float>::value ? (D <= 4 ? 4 : D <= 6 ? 3 : 2) : 1; }

// ----------------------------------------------------------------------------- directions
// Uniform direction on S^{D-1} from the first dir_words(D) words.
template <typename R, int D, int NW>
__device__ __forceinline__ void unit_dir(const Words<NW>& W, R d[D]) {
    if constexpr (D == 2) {
        RO<R>::sc2pi(RO<R>::u(W.w[0]), d[1], d[0]);
    } else if constexpr (D == 3) {
        const R z = R(2) * RO<R>::u(W.w[0]) - R(1);
        R s, c;
        RO<R>::sc2pi(RO<R>::u(W.w[1]), s, c);
        const R r = RO<R>::sq(fmax(R(0), R(1) - z * z));
        d[0] = r * c; d[1] = r * s; d[2] = z;
    } else {
        R g[2 * ((D + 1) / 2)];
#pragma unroll
        for (int j = 0; j < (D + 1) / 2; ++j) {
            const R rr = RO<R>::sq(R(-2) * RO<R>::lg(RO<R>::u(W.w[2 * j])));
            R s, c;
            RO<R>::sc2pi(RO<R>::u(W.w[2 * j + 1]), s, c);
            g[2 * j] = rr * c; g[2 * j + 1] = rr * s;
        }
        R n2 = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) n2 += g[i] * g[i];
        const R inv = RO<R>::rsq(n2);
#pragma unroll
        for (int i = 0; i < D; ++i) d[i] = g[i] * inv;
    }
}

// ----------------------------------------------------------------------------- geometry
template <typename R, int D, bool LDS = false>
__device__ __forceinline__ void normal_at(const DevRegion& g, const R* __restrict__ pay, const R y[D], int seg, R n[D]) {
    const R* q = pay + Pay<R>::g(g);
    if (g.kind == WOI_SHAPE_SPHERE) {
        const R iR = RO<R>::rcp(q[D]);   // FP64: exact division
#pragma unroll
        for (int i = 0; i < D; ++i) n[i] = (y[i] - q[i]) * iR;
    } else if (g.kind == WOI_SHAPE_ELLIPSOID) {
        R s = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            R t = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) t += q[D + i * D + j] * (y[j] - q[j]);
            n[i] = t; s += t * t;
        }
        const R inv = RO<R>::rsq(s);     // FP64: 1 / sqrt
#pragma unroll
        for (int i = 0; i < D; ++i) n[i] *= inv;
    } else if (D == 3 && LDS && g.kind == WOI_SHAPE_MESH3D) {
        const R* nr = pay + Pay<R>::nrm(g) + 3 * seg;
#pragma unroll
        for (int i = 0; i < D && i < 3; ++i) n[i] = nr[i];
    } else {
        if constexpr (D == 2) {
            if constexpr (LDS && std::is_same<R, float>::value) {
                // FP32 with staged vertices: the segment's normal from its LDS endpoints
                const float* v = poly_xy<R, LDS>(g, pay) + 2 * seg;
                const float ex = v[2] - v[0], ey = v[3] - v[1], il = RO<float>::rsq(ex * ex + ey * ey);
                n[0] = ey * il; n[1] = -ex * il;
            } else {
                const R* nr = pay + Pay<R>::nrm(g) + 2 * seg;
                n[0] = nr[0]; n[1] = nr[1];
            }
        }
    }
}

// Fourier series of a 2D datum in the direction e with NT modes (NT fixed: every coefficient is
// loaded before the sum starts); the same sum as the general loop in data_b.
template <typename R, int NT>
__device__ __forceinline__ R fourier_fixed(const R* __restrict__ cf, const R e[2]) {
    R c[2 * NT + 1];
#pragma unroll
    for (int k = 0; k <= 2 * NT; ++k) c[k] = cf[k];
    R b = c[0], zr = 1, zi = 0;
#pragma unroll
    for (int k = 1; k <= NT; ++k) {
        const R nr = zr * e[0] - zi * e[1], ni = zr * e[1] + zi * e[0];
        zr = nr; zi = ni;
        b += c[2 * k - 1] * zr + c[2 * k] * zi;
    }
    return b;
}

// Nested Horner sum of a 3D directional polynomial of degree NT over its dense triangular
// coefficient table (NT fixed: every coefficient is loaded before the sum starts); the same sum
// as the general loop in data_b.
template <typename R, int NT>
__device__ __forceinline__ R horner3_fixed(const R* __restrict__ cf, const R e[3]) {
    constexpr int NC = (NT + 1) * (NT + 2) * (NT + 3) / 6;
    R c[NC];
#pragma unroll
    for (int t = 0; t < NC; ++t) c[t] = cf[t];
    int q = 0;
    R b0 = 0;
#pragma unroll
    for (int i = NT; i >= 0; --i) {
        R b1 = 0;
#pragma unroll
        for (int j = NT - i; j >= 0; --j) {
            R b2 = 0;
#pragma unroll
            for (int k = NT - i - j; k >= 0; --k) b2 = b2 * e[2] + c[q++];
            b1 = b1 * e[1] + b2;
        }
        b0 = b0 * e[0] + b1;
    }
    return b0;
}

// b_i(y) (Eq. interface_problem data).
template <typename R, int D, bool LDS = false>
__device__ __forceinline__ R data_b(const DevProblem* dp, const DevRegion& g, const R* __restrict__ pay,
                                    const R y[D], int seg) {
    const R* cf = pay + Pay<R>::dat(g);
    if (g.dkind == WOI_DATA_ZERO) return R(0);
    if (g.dkind == WOI_DATA_FIELD_FLUX || g.dkind == WOI_DATA_SOURCE_FLUX) {
        R n[D];
        normal_at<R, D, LDS>(g, pay, y, seg, n);
        if (g.dkind == WOI_DATA_FIELD_FLUX) {
            R b = 0;
#pragma unroll
            for (int i = 0; i < D; ++i) b += cf[i] * n[i];
            return b;
        }
        R dn = 0, r2 = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) { const R e = y[i] - cf[1 + i]; dn += e * n[i]; r2 += e * e; }
        R rm = R(1);
#pragma unroll
        for (int i = 0; i < D / 2; ++i) rm *= r2;
        if constexpr (D % 2) rm *= RO<R>::sq(r2);
        return RO<R>::div(cf[0] * dn, rm);
    }
    // direction-based data: e = (y - c)/|y - c|, c stored after the coefficients
    int ncoef = g.dkind == WOI_DATA_FOURIER2D ? 2 * g.nt + 1 : g.nt;
    if (D <= 3 && g.dkind == DK_DIRPOLY_HORNER) {
        const int n = g.nt;
        ncoef = D == 2 ? (n + 1) * (n + 2) / 2 : (n + 1) * (n + 2) * (n + 3) / 6;
    }
    const R* c = cf + ncoef;
    R e[D], r2 = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) { e[i] = y[i] - c[i]; r2 += e[i] * e[i]; }
    const R ir = RO<R>::rsq(r2);
#pragma unroll
    for (int i = 0; i < D; ++i) e[i] *= ir;
    if (g.dkind == WOI_DATA_FOURIER2D) {
        switch (g.nt) {   // the common mode counts, with their coefficients loaded up front
            case 1: return fourier_fixed<R, 1>(cf, e);
            case 2: return fourier_fixed<R, 2>(cf, e);
            case 3: return fourier_fixed<R, 3>(cf, e);
            case 4: return fourier_fixed<R, 4>(cf, e);
            case 5: return fourier_fixed<R, 5>(cf, e);
            case 6: return fourier_fixed<R, 6>(cf, e);
            default: break;
        }
        // cos(k th) + i sin(k th) = (e_x + i e_y)^k
        R b = cf[0], zr = 1, zi = 0;
        for (int k = 1; k <= g.nt; ++k) {
            const R nr = zr * e[0] - zi * e[1], ni = zr * e[1] + zi * e[0];
            zr = nr; zi = ni;
            b += cf[2 * k - 1] * zr + cf[2 * k] * zi;
        }
        return b;
    }
    if constexpr (D <= 3) {
        if (g.dkind == DK_DIRPOLY_HORNER) {   // nested Horner over the dense triangular table
            if constexpr (D == 3) {
                switch (g.nt) {   // the common degrees, with their coefficients loaded up front
                    case 1: return horner3_fixed<R, 1>(cf, e);
                    case 2: return horner3_fixed<R, 2>(cf, e);
                    case 3: return horner3_fixed<R, 3>(cf, e);
                    case 4: return horner3_fixed<R, 4>(cf, e);
                    default: break;
                }
            }
            const int n = g.nt;
            const R* q = cf;
            R b0 = 0;
            for (int i = n; i >= 0; --i) {
                R b1 = 0;
                for (int j = n - i; j >= 0; --j) {
                    if constexpr (D == 3) {
                        R b2 = 0;
                        for (int k = n - i - j; k >= 0; --k) b2 = b2 * e[2] + *q++;
                        b1 = b1 * e[1] + b2;
                    } else {
                        b1 = b1 * e[1] + *q++;
                    }
                }
                b0 = b0 * e[0] + b1;
            }
            return b0;
        }
    }
    // term list: the exponents of term t are the bytes of one 8-byte word (dimension i in byte i)
    const uint64_t* ex = reinterpret_cast<const uint64_t*>(reinterpret_cast<const char*>(dp) + dp->offb + g.dexp);
    R b = 0;
    for (int t = 0; t < g.nt; ++t) {
        R term = cf[t];
        const uint64_t xb = ex[t];
#pragma unroll
        for (int i = 0; i < D; ++i)
            for (int p = (int)((xb >> (8 * i)) & 0xFFu); p > 0; --p) term *= e[i];
        b += term;
    }
    return b;
}

// ---- uniform surface sample, one attempt: returns false when rejected
__device__ __forceinline__ const int* int_payload(const DevProblem* dp) {
    return reinterpret_cast<const int*>(reinterpret_cast<const char*>(dp) + dp->offi);
}

// Point at arclength s on a polyline: the segment is the largest j with cum[j] <= s, found
// from the guide table entry for s in O(1) expected probes (inlined in every kernel: no call
// frame, no scratch).
template <typename R, int D, bool LDS>
__device__ __forceinline__ bool polyline_at(const DevProblem* dp, const DevRegion& g, const R* __restrict__ pay, R s,
                                            R y[D], int& seg) {
    if constexpr (D == 2) {
        // FP32: cum and 1/len interleaved (stride 2); FP64: cum, and len in its own table
        constexpr bool F32 = std::is_same<R, float>::value;
        constexpr int CS = F32 ? 2 : 1;
        const int n = g.nv;
        int k = (int)(s * Pay<R>::gscale(g));   // guide hint; the probes below find the exact j
        k = min(max(k, 0), n - 1);
        auto locate = [&](const R* cum, const int* guide) {
            int j = guide[k];
            while (j < n - 1 && cum[CS * (j + 1)] <= s) ++j;
            while (j > 0 && cum[CS * j] > s) --j;
            const R* v = poly_xy<R, LDS>(g, pay) + 2 * j;
            R f;
            if constexpr (F32) f = (s - cum[2 * j]) * cum[2 * j + 1];
            else f = (s - cum[j]) / pay[Pay<R>::len(g) + j];
            y[0] = v[0] + f * (v[2] - v[0]); y[1] = v[1] + f * (v[3] - v[1]);
            seg = j;
        };
        // the staged copies where the layout has them (region-uniform branch), else global memory
        if (LDS && F32 && g.lds_c >= 0)
            locate(reinterpret_cast<const R*>(woi_smem + g.lds_c), reinterpret_cast<const int*>(woi_smem + g.lds_g));
        else
            locate(pay + Pay<R>::cum(g), int_payload(dp) + g.guide);
    }
    return true;
}

template <typename R, int D>
__device__ __forceinline__ int surf_words(const DevRegion& g) {
    return g.kind == WOI_SHAPE_POLYLINE2D ? 1 : g.kind == WOI_SHAPE_MESH3D ? 3
         : dir_words(D) + (g.kind == WOI_SHAPE_ELLIPSOID ? 1 : 0);
}

// Triangle mesh (3D): the triangle j with cum[j] <= s < cum[j + 1] (cumulative areas; guide
// table and probes as for polylines), then the uniform point a + r (1 - u) e1 + r u e2 with
// r = sqrt(u1), from the per-triangle record (a, e1 = b - a, e2 = c - a).
template <typename R>
__device__ __forceinline__ int mesh_triangle(const DevProblem* dp, const DevRegion& g, const R* __restrict__ pay, R s) {
    constexpr int CS = std::is_same<R, float>::value ? 2 : 1;
    const R* cum = pay + Pay<R>::cum(g);
    const int n = g.nv;
    int k = (int)(s * Pay<R>::gscale(g));
    k = min(max(k, 0), n - 1);
    int j = int_payload(dp)[g.guide + k];
    while (j < n - 1 && cum[CS * (j + 1)] <= s) ++j;
    while (j > 0 && cum[CS * j] > s) --j;
    return j;
}

template <typename R, int D, bool LDS>
__device__ __forceinline__ bool surf_attempt(const DevProblem* dp, const DevRegion& g, const R* __restrict__ pay,
                                             const Stream& st, uint32_t step, int att, R y[D], int& seg,
                                             const uint32_t* pre = nullptr) {
    seg = 0;
    if (D == 3 && LDS && g.kind == WOI_SHAPE_MESH3D) {
        if constexpr (D == 3) {
            Words<3> W; W.fill(st, step, (uint32_t)att);
            const int j = mesh_triangle<R>(dp, g, pay, RO<R>::u(W.w[0]) * Pay<R>::total(g));
            const R r = RO<R>::sq(RO<R>::u(W.w[1])), u2 = RO<R>::u(W.w[2]);
            const R* T = pay + Pay<R>::g(g) + 9 * j;
            const R f1 = r * (R(1) - u2), f2 = r * u2;
#pragma unroll
            for (int i = 0; i < 3; ++i) y[i] = T[i] + f1 * T[3 + i] + f2 * T[6 + i];
            seg = j;
        }
        return true;
    }
    if (g.kind == WOI_SHAPE_POLYLINE2D) {
        Words<1> W; W.take(st, step, (uint32_t)att, pre);
        return polyline_at<R, D, LDS>(dp, g, pay, RO<R>::u(W.w[0]) * Pay<R>::total(g), y, seg);
    }
    const R* q = pay + Pay<R>::g(g);
    if (g.kind == WOI_SHAPE_SPHERE) {
        constexpr int NW = dir_words(D), NB = (NW + 3) / 4;
        Words<NW> W; W.take(st, step, (uint32_t)(att * NB), pre);
        R u[D];
        unit_dir<R, D>(W, u);
#pragma unroll
        for (int i = 0; i < D; ++i) y[i] = q[i] + q[D] * u[i];
        return true;
    }
    // ellipsoid: y = c + A^{-1/2} u, accept with probability |A^{1/2} u| / sqrt(lambda_max)
    constexpr int NW = dir_words(D) + 1, NB = (NW + 3) / 4;
    Words<NW> W; W.take(st, step, (uint32_t)(att * NB), pre);
    R u[D];
    unit_dir<R, D>(W, u);
    const R acc = RO<R>::u(W.w[NW - 1]);
    R uAu = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        R t = 0, l = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) { t += q[D + i * D + j] * u[j]; l += q[D + D * D + i * D + j] * u[j]; }
        uAu += u[i] * t;
        y[i] = q[i] + l;
    }
    return acc < RO<R>::sq(uAu * q[D + 2 * D * D]);
}

// point at arclength s on a closed 2D curve (circle or polyline)
template <typename R, int D, bool LDS>
__device__ __forceinline__ void curve_at(const DevProblem* dp, const DevRegion& g, const R* __restrict__ pay, R s,
                                         R y[D], int& seg) {
    if constexpr (D == 2) {
        if (g.kind == WOI_SHAPE_POLYLINE2D) { polyline_at<R, D, LDS>(dp, g, pay, s, y, seg); return; }
        const R* q = pay + Pay<R>::g(g);
        R sn, cs;
        RO<R>::sc2pi(RO<R>::div(s, R(2) * R(3.14159265358979323846) * q[2]), sn, cs);
        y[0] = q[0] + q[2] * cs; y[1] = q[1] + q[2] * sn; seg = 0;
    }
}

// one attempt of a uniform sample on the VR half `cls` of region h
template <typename R, int D, bool LDS>
__device__ __forceinline__ bool vr_attempt(const DevProblem* dp, const DevRegion& g, const R* __restrict__ pay,
                                           int cls, const Stream& st, int att, R y[D], int& seg) {
    if constexpr (D == 2) {
        Words<1> W; W.fill(st, 0, (uint32_t)att);
        const R t = RO<R>::u(W.w[0]) * Pay<R>::meas(g, cls);
        const R* br = pay + Pay<R>::brk(g);
        R start = 0, acc = 0;
        int c = g.class0;
        for (int p = 0; p <= g.nbrk; ++p) {
            const R end = p < g.nbrk ? br[p] : Pay<R>::total(g);
            if (c == cls) {
                const R l = end - start;
                if (t < acc + l || p == g.nbrk) {
                    curve_at<R, D, LDS>(dp, g, pay, fmin(start + (t - acc), end), y, seg);
                    return true;
                }
                acc += l;
            }
            start = end; c ^= 1;
        }
        curve_at<R, D, LDS>(dp, g, pay, start, y, seg);
        return true;
    } else {
        if (!surf_attempt<R, D, LDS>(dp, g, pay, st, 0, att, y, seg)) return false;
        return (Pay<R>::s(g) * data_b<R, D, LDS>(dp, g, pay, y, seg) >= R(0)) == (cls == 0);
    }
}

// ---- wave-cooperative rejection sampling
// Lane l needs the first attempt a >= 0 whose proposal try_at(c0_l, c1_l, a, y, seg) accepts,
// or the proposal of attempt WOI_ATTEMPT_CAP - 1 when none does (rejection sampling on an
// ellipsoid, or on a half {beta >= 0} / {beta < 0}).  Every proposal is a function of the lane's
// stream words (c0, c1) and a alone, so after each lane's own attempt 0 the whole wave serves the
// lanes still pending: with np pending, the lane of rank r among them gets its next 64 / np
// attempts from the lanes r, r + np, r + 2 np, ... and takes the first accepted one in attempt
// order.  Points, attempt numbers and rejection / cap counts are those of each lane's sequential
// loop; a wave waits for about two rounds instead of its unluckiest lane.  Requires all 64 lanes
// active on the same interface (a shared schedule); try_at must hold no wave-wide operation.
// Returns the attempt taken (WOI_ATTEMPT_CAP on a cap hit).
template <typename R, int D, class Try>
__device__ __forceinline__ int coop_first_accept(const Try& try_at, uint32_t c0, uint32_t c1, R y[D], int& seg,
                                                 Counts& cnt) {
    int att = 0, next = 1;
    bool pend = !try_at(c0, c1, 0, y, seg);
    if (pend) cnt.rejections++;
    uint64_t pm = __ballot(pend);
    const int lane = (int)__lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    while (pm) {
        const int np = __popcll(pm), per = 64 / np;
        // lane id of every pending rank (ds_permute by a permutation of the lanes: pending lanes to
        // their rank, the others after them in lane order)
        const int rk = __popcll(pm & below);
        const int dst = pend ? rk : np + (lane - rk);
        const int who = __builtin_amdgcn_ds_permute(dst << 2, lane);
        // this lane evaluates attempt next_t + k of the pending lane t of rank r = lane mod np
        const int r = lane % np, k = lane / np;
        const int t = __shfl(who, r);
        const uint32_t tc0 = __shfl(c0, t), tc1 = __shfl(c1, t);
        const int a = __shfl(next, t) + k;
        R yc[D];
        int sc = 0;
        bool okc = false, fin = false;
#pragma unroll
        for (int j = 0; j < D; ++j) yc[j] = R(0);
        if ((k < per) & (a < WOI_ATTEMPT_CAP)) {
            okc = try_at(tc0, tc1, a, yc, sc);
            fin = okc | (a == WOI_ATTEMPT_CAP - 1);
        }
        const uint64_t fm = __ballot(fin);
        // pending lanes: the first finished helper in attempt order
        int h = lane, kk = 0;
        bool got = false;
        if (pend) {
            for (kk = 0; kk < per && next + kk < WOI_ATTEMPT_CAP; ++kk)
                if ((fm >> (rk + kk * np)) & 1ull) { got = true; break; }
            if (got) h = rk + kk * np;
        }
        R yh[D];
#pragma unroll
        for (int j = 0; j < D; ++j) yh[j] = __shfl(yc[j], h);
        const int sh = __shfl(sc, h);
        const bool okh = __shfl((int)okc, h) != 0;
        if (pend) {
            if (got) {
#pragma unroll
                for (int j = 0; j < D; ++j) y[j] = yh[j];
                seg = sh;
                cnt.rejections += (uint32_t)kk + (okh ? 0u : 1u);
                if (okh) att = next + kk;
                else { att = WOI_ATTEMPT_CAP; cnt.caps++; }
                pend = false;
            } else {
                cnt.rejections += (uint32_t)kk;
                next += per;
            }
        }
        pm = __ballot(pend);
    }
    return att;
}

// Whether the wave may sample cooperatively: a shared schedule (the same interface in every
// lane) and all 64 lanes active.
__device__ __forceinline__ bool wave_full(bool shared_sched) {
    return shared_sched && __builtin_amdgcn_read_exec() == ~0ull;
}

// ---- line / ray intersections
// Quadric (sphere, ellipsoid): returns q in {0, 1} and t.
template <typename R, int D>
__device__ __forceinline__ int quadric_hit(const DevRegion& g, const R* __restrict__ pay, const R y[D], const R d[D],
                                           bool ray, R& t) {
    const R* q = pay + Pay<R>::g(g);
    R yc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) yc[i] = y[i] - q[i];
    R a, b, cc;
    if (g.kind == WOI_SHAPE_SPHERE) {
        a = 1; b = 0; cc = -q[D] * q[D];
#pragma unroll
        for (int i = 0; i < D; ++i) { b += yc[i] * d[i]; cc += yc[i] * yc[i]; }
    } else {
        a = 0; b = 0; cc = -1;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            R s1 = 0, s2 = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) { s1 += q[D + i * D + j] * d[j]; s2 += q[D + i * D + j] * yc[j]; }
            a += d[i] * s1; b += d[i] * s2; cc += yc[i] * s2;
        }
    }
    if (!ray) {   // y on the quadric: other root of t (a t + 2 b) = 0
        t = RO<R>::div(R(-2) * b, a);
        return t != R(0) ? 1 : 0;
    }
    const R disc = b * b - a * cc;
    if (disc < R(0)) return 0;
    t = RO<R>::div(-b + RO<R>::sq(disc), a);
    return t > R(0) ? 1 : 0;
}

// Polyline: hits of the line / ray y + t d in segment order.  The signed distance of
// vertex j from the line is h_j = d x (v_j - y); segment j is hit iff h_j = 0 != h_{j+1}
// or the signs differ (the half-open segment [v_j, v_{j+1})), the line excludes the segment
// of y, and the crossing parameter passes the line / ray test.  One flat loop per lane
// walks the vertex index with an adaptive aligned stride 2^l: a block whose chord bound
// keeps all its vertices strictly on one side of the line is skipped, otherwise it is
// halved; at stride 1 the sign test picks out candidate segments.  Every iteration costs the
// same (one vertex, one bound), so lanes of a wave stay in step.  The walk only queues the
// candidates; their crossing parameters are tested after it, so that the wave does not run
// the test in every iteration in which some lane reaches a candidate.

// Up to eight segment indices of 16 bits, slot k in half (k & 1) of word k >> 1.  push()
// moves every slot up by one (slot 7 drops out) and writes slot 0; pop() takes slot 0 and
// moves every slot down.
struct Queue16 {
    uint32_t w0, w1, w2, w3;
    __device__ __forceinline__ void push(uint32_t j) {
        w3 = __builtin_amdgcn_alignbit(w3, w2, 16);
        w2 = __builtin_amdgcn_alignbit(w2, w1, 16);
        w1 = __builtin_amdgcn_alignbit(w1, w0, 16);
        w0 = (w0 << 16) | j;
    }
    __device__ __forceinline__ uint32_t pop() {
        const uint32_t j = w0 & 0xFFFFu;
        w0 = __builtin_amdgcn_alignbit(w1, w0, 16);
        w1 = __builtin_amdgcn_alignbit(w2, w1, 16);
        w2 = __builtin_amdgcn_alignbit(w3, w2, 16);
        w3 >>= 16;
        return j;
    }
    __device__ __forceinline__ uint32_t at(int k) const {   // select on the bits of k (registers only)
        const uint32_t lo = (k & 2) ? w1 : w0, hi = (k & 2) ? w3 : w2;
        return (((k & 4) ? hi : lo) >> ((k & 1) << 4)) & 0xFFFFu;
    }
};
constexpr int POLY_QUEUE = 8;

constexpr bool COUNT_POLY = true;   // dead code unless the counting kernel reads the counters

// FP32 walks: crossing parameters below this magnitude are decided in FP64 (polylines, meshes).
constexpr float POLY_T_BAND = 1e-4f;
// A line from y never counts a crossing this close to y (it is y itself, up to the FP32 state's
// own rounding); the FP64 walk's threshold is RO<double>::line_eps.
constexpr double LINE_EPS_F32_STATE = 1e-6;

// FP64 decision of polyline segment j for an FP32 walker at y, direction d (both taken exactly
// to FP64): the FP64 path's sign test on the FP64 vertices, then the crossing parameter.
__device__ __forceinline__ bool poly_hit_fp64(const DevProblem* dp, const DevRegion& g, const float y[2], const float d[2],
                                           int j, bool ray) {
    const double* a = Pay<double>::base(dp) + g.g64 + 2 * j;
    const double y0 = y[0], y1 = y[1], d0 = d[0], d1 = d[1];
    const double ha = d0 * (a[1] - y1) - d1 * (a[0] - y0), hb = d0 * (a[3] - y1) - d1 * (a[2] - y0);
    const bool cross = (hb != 0.0) & ((ha == 0.0) | ((ha > 0.0) != (hb > 0.0)));
    const double ex = a[2] - a[0], ey = a[3] - a[1], den = d0 * ey - d1 * ex;
    const double t = ((a[0] - y0) * ey - (a[1] - y1) * ex) / den;
    return cross & (den != 0.0) & (ray ? (t > 0.0) : (fabs(t) > LINE_EPS_F32_STATE));
}

// The walk: calls cand(j) for every candidate segment j in increasing order, and stops
// early when cand returns true.
// Search modes: PS_RAY when every lane of the wave searches along a ray, else PS_ANY (the plain
// walk; each lane's line or ray applies in the exact test of the candidates).  The ray mode also skips blocks behind the ray's origin: every
// vertex v of a block has d.(v - y) <= max(g_j, g_e) + bound (the bound holds in every
// direction), and a crossing point z with t = d.(z - y) <= 0 is no ray hit.  For a segment the
// bound is the FP32 rounding band, which covers the error of the FP32 g values, so a segment
// skipped this way has t < 0 in exact arithmetic too (the exact test would reject it).  Mixed
// waves gain nothing from it (a wave waits for its slowest lane), so PS_ANY keeps the plain walk.
enum : int { PS_ANY = 0, PS_RAY = 1 };

template <typename R, bool LDS, int MODE, class Cand>
__device__ __forceinline__ void poly_walk(const DevProblem* dp, const DevRegion& g, const R* __restrict__ pay,
                                          const R y[2], const R d[2], Counts& cnt, Cand cand) {
    constexpr bool RAY = MODE == PS_RAY;    // the walk keeps the ray parameters
    constexpr bool F32 = std::is_same<R, float>::value;
    const int n = g.nv, n2 = g.n2, top = g.top;
    // block tests run in FP32 on the staged (or global) FP32 copy; bounds absorb the rounding
    const float yf0 = (float)y[0], yf1 = (float)y[1], df0 = (float)d[0], df1 = (float)d[1];
    // h(v) = d x (v - y) = d0 v1 - d1 v0 - (d0 y1 - d1 y0): two FMAs per vertex
    const float hc = df0 * yf1 - df1 * yf0;
    // g(v) = d . (v - y), the ray parameter of v's projection (rays only)
    const float gc = df0 * yf0 + df1 * yf1;
    auto bound = [&](int idx) -> float {
        if constexpr (LDS) return __half2float(reinterpret_cast<const __half*>(woi_smem + g.lds_b)[idx]);
        else return Pay<float>::base(dp)[g.bnd + idx];
    };
    // The walk position is kept as jn = n2 + j: block (j, lvl) then sits at heap index
    // jn >> lvl, segments included (their bound is 0), and ctz(jn) is the highest level a
    // block starting at j may take.  The walk starts with the block [0, 2^top] and after
    // each skipped block takes the largest aligned block that follows.
    const int jend = n2 + n;
    // h of vertex jn - n2; the LDS byte offset of vertex 0 less 8 n2, in wrapping 32-bit
    // arithmetic, makes the address one shift-add of jn
    const uint32_t vbase = (uint32_t)g.lds_v - 8u * (uint32_t)n2;
    const float2* __restrict__ vg = reinterpret_cast<const float2*>(Pay<float>::base(dp) + g.g32);
    auto hn = [&](int jn) -> float {
        float2 p;
        if constexpr (LDS) p = *reinterpret_cast<const float2*>(woi_smem + (vbase + 8u * (uint32_t)jn));
        else p = vg[jn - n2];
        return fmaf(df0, p.y, fmaf(-df1, p.x, -hc));
    };
    auto gn = [&](int jn) -> float {
        float2 p;
        if constexpr (LDS) p = *reinterpret_cast<const float2*>(woi_smem + (vbase + 8u * (uint32_t)jn));
        else p = vg[jn - n2];
        return fmaf(df0, p.x, fmaf(df1, p.y, -gc));
    };
    const R* __restrict__ v = poly_xy<R, LDS>(g, pay);       // exact values (FP64)
    int jn = n2, lvl = top;
    float hj = hn(jn), gj = RAY ? gn(jn) : 0.0f;
    while (jn < jend) {
        const int je = jn + (1 << lvl);   // <= 2 n2: the FP32 vertices are padded to n2 + 1
        const float he = hn(je), ge = RAY ? gn(je) : 0.0f;
        const bool seg = lvl == 0;
        const float b = bound(jn >> lvl);
        // Every vertex of the block strictly on one side of the line: the end value nearer
        // zero, med3(h_j, h_e, 0) (zero when the signs differ), exceeds the bound in magnitude.
        // For a segment the bound is the FP32 rounding band: FP32 walks queue every segment
        // that is not clearly on one side (a sign change, or an end value within the band) and
        // decide it exactly after the walk (in FP64 when inside the band).
        bool skip = fabsf(__builtin_amdgcn_fmed3f(hj, he, 0.0f)) > b;
        if constexpr (RAY) skip |= (gj < -b) & (ge < -b);   // (fmaxf would add a NaN canonicalisation)
        bool cross;
        if constexpr (F32) {
            cross = !skip;
        } else {                                              // FP64 exact values at stride 1 only:
            // a zero start value belongs to this segment, a zero end value to the next
            R ha = R(0), hb = R(0);
            if (seg) {
                const R* a = v + 2 * (jn - n2);
                ha = d[0] * (a[1] - y[1]) - d[1] * (a[0] - y[0]);
                hb = d[0] * (a[3] - y[1]) - d[1] * (a[2] - y[0]);
            }
            cross = (hb != R(0)) & ((ha == R(0)) | ((ha > R(0)) != (hb > R(0))));
        }
        if (seg & cross) {
            if (cand(jn - n2)) return;
        }
        if (COUNT_POLY) { cnt.nodes += seg ? 0 : 1; cnt.segs += seg ? 1 : 0; }
        const bool adv = seg | skip;
        const int lz = (int)__builtin_ctz((unsigned)je);
        jn = adv ? je : jn;
        hj = adv ? he : hj;
        if constexpr (RAY) gj = adv ? ge : gj;
        lvl = adv ? lz : lvl - 1;
    }
}

// Number of hits q and, when q > 0, the segment jp of hit `pick` = min(floor(up q), q - 1)
// (uniform among the hits).  With more than POLY_QUEUE candidates (or segment indices past
// 16 bits) the hits are counted by a second walk and found by a third.
template <typename R, bool LDS, int MODE>
__device__ __forceinline__ int poly_pick_t(const DevProblem* dp, const DevRegion& g, const R* __restrict__ pay,
                                           const R y[2], const R d[2], bool ray_lane, int yseg, R up, int& pick,
                                           int& jp, Counts& cnt) {
    const bool ray = MODE == PS_RAY || ray_lane;
    const R* __restrict__ v = poly_xy<R, LDS>(g, pay);
    // Exact test of candidate segment j: its ends on opposite sides of the line (a zero start
    // value belongs to this segment, a zero end value to the next), and the crossing parameter
    // passes the line / ray test.  FP32 walks decide in FP32 only when every quantity is clear
    // of its rounding band, else from the FP64 vertices (counted as an FP64 recheck).
    auto hit = [&](int j) -> bool {
        if (!ray & (j == yseg)) return false;   // a line excludes the segment of y (the walk queues it)
        const R* a = v + 2 * j;
        const R ex = a[2] - a[0], ey = a[3] - a[1];
        const R den = d[0] * ey - d[1] * ex;
        const R t = RO<R>::div((a[0] - y[0]) * ey - (a[1] - y[1]) * ex, den);
        if constexpr (std::is_same<R, float>::value) {
            // signed distances of the ends from the line: h_a = d x (a - y), h_b = h_a + d x e; with
            // both clear of the band their signs are trusted (the walk's own values, computed
            // differently, may sit on the other side of the band edge)
            const float ha = d[0] * (a[1] - y[1]) - d[1] * (a[0] - y[0]), hb = ha + den;
            const bool amb = (fminf(fabsf(ha), fabsf(hb)) <= g.hband_f) | (fabsf(t) < POLY_T_BAND);
            if (!amb) return (ha * hb < 0.0f) & (!ray | (t > 0.0f));
            cnt.fb++;
            return poly_hit_fp64(dp, g, y, d, j, ray);
        } else {
            return (den != R(0)) & (ray ? (t > R(0)) : (fabs(t) > RO<R>::line_eps));
        }
    };
    Queue16 cq{0u, 0u, 0u, 0u};
    int c = 0;
    poly_walk<R, LDS, MODE>(dp, g, pay, y, d, cnt, [&](int j) -> bool {
        cq.push((uint32_t)j);
        ++c;
        return false;
    });
    int q = 0;
    if (c <= POLY_QUEUE && g.nv <= 0xFFFF) {
        // newest candidate first, so the hit queue ends with the first hit in slot 0
        Queue16 hq{0u, 0u, 0u, 0u};
        for (int k = 0; k < c; ++k) {
            const uint32_t j = cq.pop();
            if (hit((int)j)) { hq.push(j); ++q; }
        }
        if (q > 0) {
            pick = min((int)(up * (R)q), q - 1);
            jp = (int)hq.at(pick);
        }
        return q;
    }
    poly_walk<R, LDS, MODE>(dp, g, pay, y, d, cnt, [&](int j) -> bool { q += hit(j) ? 1 : 0; return false; });
    if (q > 0) {
        pick = min((int)(up * (R)q), q - 1);
        int k = 0;
        poly_walk<R, LDS, MODE>(dp, g, pay, y, d, cnt, [&](int j) -> bool {
            if (!hit(j)) return false;
            jp = j;
            return k++ == pick;
        });
    }
    return q;
}

template <typename R, bool LDS>
__device__ __forceinline__ int poly_pick(const DevProblem* dp, const DevRegion& g, const R* __restrict__ pay,
                                         const R y[2], const R d[2], bool ray, int yseg, R up, int& pick, int& jp,
                                         Counts& cnt) {
    // wave-uniform choice of the search mode (every wave is uniform when the schedule is shared)
    if (__ballot(ray) == __builtin_amdgcn_read_exec())
        return poly_pick_t<R, LDS, PS_RAY>(dp, g, pay, y, d, true, yseg, up, pick, jp, cnt);
    return poly_pick_t<R, LDS, PS_ANY>(dp, g, pay, y, d, ray, yseg, up, pick, jp, cnt);
}

// Triangle mesh: hits of the line / ray y + t d in triangle order (Moller-Trumbore with the
// closed barycentric bounds; a line skips the triangle of y and |t| <= eps, a ray keeps t > 0).
// Returns q and, when q > 0, the parameter t and triangle of hit `pick` = min(floor(up q), q - 1).
// Moller-Trumbore in precision Q for one triangle (a, e1 = b - a, e2 = c - a): barycentric u, v,
// parameter t and the determinant.
template <typename Q, typename P>
__device__ __forceinline__ void moller_trumbore(const Q* a, const P* y, const P* d, Q& u, Q& v, Q& t, Q& det) {
    const Q *e1 = a + 3, *e2 = a + 6;
    const Q yq[3] = {(Q)y[0], (Q)y[1], (Q)y[2]}, dq[3] = {(Q)d[0], (Q)d[1], (Q)d[2]};
    const Q sv[3] = {yq[0] - a[0], yq[1] - a[1], yq[2] - a[2]};
    const Q pv[3] = {dq[1] * e2[2] - dq[2] * e2[1], dq[2] * e2[0] - dq[0] * e2[2], dq[0] * e2[1] - dq[1] * e2[0]};
    det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
    u = RO<Q>::div(sv[0] * pv[0] + sv[1] * pv[1] + sv[2] * pv[2], det);
    const Q qv[3] = {sv[1] * e1[2] - sv[2] * e1[1], sv[2] * e1[0] - sv[0] * e1[2], sv[0] * e1[1] - sv[1] * e1[0]};
    v = RO<Q>::div(dq[0] * qv[0] + dq[1] * qv[1] + dq[2] * qv[2], det);
    t = RO<Q>::div(e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2], det);
}

// FP32 walks: a triangle test whose barycentric coordinates lie within this band of an edge,
// or whose parameter lies within POLY_T_BAND of 0, is decided in FP64.
constexpr float MESH_UV_BAND = 2e-6f;

template <typename R>
struct MeshHit {
    const R* __restrict__ T;   // per triangle (a, b - a, c - a)
    const double* __restrict__ T64;   // the same in FP64 (the FP64 recheck of FP32 walks)
    const R *y, *d;
    bool ray;
    int yseg;
    Counts* cnt;
    __device__ __forceinline__ bool operator()(int j, R& t) const {
        if (!ray & (j == yseg)) return false;
        R u, v, det;
        moller_trumbore<R, R>(T + 9 * j, y, d, u, v, t, det);
        if constexpr (std::is_same<R, float>::value) {
            const float w = 1.0f - u - v;
            const bool amb = (fminf(fminf(fabsf(u), fabsf(v)), fminf(fabsf(w), fminf(fabsf(1.0f - u), fabsf(1.0f - v)))) <
                              MESH_UV_BAND) | (fabsf(t) < POLY_T_BAND) | (det == 0.0f);
            if (amb) {
                cnt->fb++;
                double u6, v6, t6, det6;
                moller_trumbore<double, float>(T64 + 9 * j, y, d, u6, v6, t6, det6);
                t = (float)t6;
                return (det6 != 0.0) & (u6 >= 0.0) & (u6 <= 1.0) & (v6 >= 0.0) & (u6 + v6 <= 1.0) &
                       (ray ? (t6 > 0.0) : (fabs(t6) > LINE_EPS_F32_STATE));
            }
        }
        return (det != R(0)) & (u >= R(0)) & (u <= R(1)) & (v >= R(0)) & (u + v <= R(1)) &
               (ray ? (t > R(0)) : (fabs(t) > RO<R>::line_eps));
    }
};

// Every triangle in order (wave-uniform: all lanes test the same triangle).  The first scan
// counts the hits and keeps the first two; a second scan finds a later pick.
template <typename R>
__device__ __forceinline__ int mesh_scan(const MeshHit<R>& hit, int n, R up, int& pick, R& tp, int& jp, Counts& cnt) {
    int q = 0, j0 = 0, j1 = 0;
    R t0 = 0, t1 = 0;
    for (int j = 0; j < n; ++j) {
        R t;
        const bool h = hit(j, t);
        t0 = (h & (q == 0)) ? t : t0; j0 = (h & (q == 0)) ? j : j0;
        t1 = (h & (q == 1)) ? t : t1; j1 = (h & (q == 1)) ? j : j1;
        q += h ? 1 : 0;
        if (COUNT_POLY) cnt.segs++;
    }
    if (q > 0) {
        pick = min((int)(up * (R)q), q - 1);
        tp = pick == 0 ? t0 : t1;
        jp = pick == 0 ? j0 : j1;
        if (pick >= 2) {
            int k = 0;
            for (int j = 0; j < n; ++j) {
                R t;
                if (hit(j, t)) {
                    if (k == pick) { tp = t; jp = j; break; }
                    ++k;
                }
            }
        }
    }
    return q;
}

// Through the mesh's BVH: a stackless walk over the depth-first node list (enter a node whose
// widened box meets the line -- an FP32 slab test -- else jump to the node after its subtree),
// exact tests of the triangles of the leaves reached, hits queued by triangle index.  The hit
// of rank `pick` among the queued indices is the pick-th in triangle order.  More than
// POLY_QUEUE hits (or indices past 16 bits) fall back to the scan.
template <typename R>
__device__ __forceinline__ int mesh_pick(const DevProblem* dp, const DevRegion& g, const R* __restrict__ pay,
                                         const R y[3], const R d[3], bool ray, int yseg, R up, int& pick, R& tp,
                                         int& jp, Counts& cnt) {
    const MeshHit<R> hit{pay + Pay<R>::g(g), Pay<double>::base(dp) + g.g64, y, d, ray, yseg, &cnt};
    const int n = g.nv;
    const float* __restrict__ nodes = Pay<float>::base(dp) + g.bvh;
    const int* __restrict__ list = int_payload(dp) + g.bvhidx;
    const float yf[3] = {(float)y[0], (float)y[1], (float)y[2]};
    const float inv[3] = {1.0f / (float)d[0], 1.0f / (float)d[1], 1.0f / (float)d[2]};
    const float tlo = ray ? 0.0f : -INFINITY;
    Queue16 hq{0u, 0u, 0u, 0u};
    int q = 0;
    for (int i = 0; i < g.nbvh;) {
        const float* nd = nodes + 8 * i;
        float t0 = tlo, t1 = INFINITY;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float a = (nd[k] - yf[k]) * inv[k], b = (nd[3 + k] - yf[k]) * inv[k];
            t0 = fmaxf(t0, fminf(a, b));
            t1 = fminf(t1, fmaxf(a, b));
        }
        const bool in = t0 <= t1;
        const float lf = nd[7];
        if (in & (lf >= 0.0f)) {
            const int code = (int)lf, first = code >> 3, count = code & 7;
            for (int c = 0; c < count; ++c) {
                const int j = list[first + c];
                R t;
                if (hit(j, t)) {
                    if (q < POLY_QUEUE) hq.push((uint32_t)j);
                    ++q;
                }
                if (COUNT_POLY) cnt.segs++;
            }
        }
        if (COUNT_POLY) cnt.nodes++;
        i = (in & (lf < 0.0f)) ? i + 1 : (int)nd[6];
    }
    if (q == 0) return 0;
    if (q > POLY_QUEUE || n > 0xFFFF) return mesh_scan<R>(hit, n, up, pick, tp, jp, cnt);
    pick = min((int)(up * (R)q), q - 1);
    int jb = 0;
    for (int a = 0; a < q; ++a) {
        const int ja = (int)hq.at(a);
        int rank = 0;
        for (int b = 0; b < q; ++b) rank += (int)hq.at(b) < ja ? 1 : 0;
        jb = rank == pick ? ja : jb;
    }
    R t = 0;
    hit(jb, t);
    tp = t;
    jp = jb;
    return q;
}

// ----------------------------------------------------------------------------- FP64 sign recheck
// The sign factor of Eq. naive_woi_T in FP64 for an FP32 walker that moved from y to yn on
// interface g (segment or triangle seg), used when the FP32 dot product lies inside its rounding
// band (|dn| <= DevProblem::sign_band_f).  Polylines and meshes: (a - y) . n with a a vertex of
// the segment / triangle and n its FP64 normal (yn - a is parallel to the segment / triangle).
// A uniform point on a quadric: (yn - y) . n(yn) in FP64.  (A line or ray on a quadric never
// gets here: its sign is + exactly, see transition.)
template <int D, bool LDS>
__device__ __forceinline__ float sign_fp64(const DevProblem* dp, const DevRegion& g, const float y[D], const float yn[D],
                                        int seg) {
    const double* p64 = Pay<double>::base(dp);
    double s = 0;
    if (g.kind == WOI_SHAPE_POLYLINE2D) {
        if constexpr (D == 2) {
            const double *a = p64 + g.g64 + 2 * seg, *n = p64 + g.nrm64 + 2 * seg;
            s = (a[0] - (double)y[0]) * n[0] + (a[1] - (double)y[1]) * n[1];
        }
    } else if (D == 3 && LDS && g.kind == WOI_SHAPE_MESH3D) {
        const double *a = p64 + g.g64 + 9 * seg, *n = p64 + g.nrm64 + 3 * seg;
#pragma unroll
        for (int k = 0; k < D && k < 3; ++k) s += (a[k] - (double)y[k]) * n[k];
    } else {
        double yn6[D], n6[D];
#pragma unroll
        for (int j = 0; j < D; ++j) yn6[j] = yn[j];
        normal_at<double, D, LDS>(g, p64, yn6, seg, n6);
#pragma unroll
        for (int j = 0; j < D; ++j) s += (yn6[j] - (double)y[j]) * n6[j];
    }
    return s < 0.0 ? -1.0f : 1.0f;
}

// ----------------------------------------------------------------------------- accumulation
template <typename R, int D>
__device__ __forceinline__ void add_term(const DevProblem* dp, const R xh[D], const R xl[D], const R y[D], R c,
                                         R& F, R G[D], Counts& cnt) {
    R d[D], r2 = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) { d[i] = (xh[i] - y[i]) + xl[i]; r2 += d[i] * d[i]; }
    if (r2 == R(0)) { cnt.zero++; return; }
    R phi, irm;   // Phi(x, y), |x - y|^{-m}
    if constexpr (D == 2) {
        if constexpr (std::is_same<R, float>::value)
            phi = __log2f(r2) * -0.0551589000381629f;   // -ln 2 / (4 pi): -ln(r2) / (4 pi) from the hardware log2
        else
            phi = -RO<R>::lg(r2) * R(0.0795774715459476678844418816863);   // 1/(4 pi)
        irm = RO<R>::rcp(r2);
    } else {
        const R ir = RO<R>::rsq(r2);
        R ir2 = ir * ir, p = R(1);
#pragma unroll
        for (int i = 0; i < (D - 2) / 2; ++i) p *= ir2;
        if constexpr (D % 2) p *= ir;   // p = r^{2-m}
        phi = Pay<R>::pc(dp) * p;
        irm = p * ir2;
    }
    F += c * phi;
    R gs;
    if constexpr (std::is_same<R, float>::value) gs = -c * irm * dp->inv_unit_area_f;
    else gs = RO<R>::div(-c * irm, Pay<R>::ua(dp));
#pragma unroll
    for (int i = 0; i < D; ++i) G[i] += gs * d[i];
}

__device__ __forceinline__ uint32_t trace_word(int h, int cs, int q, int pick, int neg, int att) {
    q = min(q, 255); pick = min(pick, 255); att = min(att, 127);
    return (uint32_t)h | ((uint32_t)cs << 6) | ((uint32_t)q << 8) | ((uint32_t)pick << 16) |
           ((uint32_t)(neg ? 1 : 0) << 24) | ((uint32_t)att << 25);
}

// One transition from y (on the previous interface; segment or triangle seg) onto interface
// g (the three cases of Eq. naive_woi_p): uniform on dOmega_g with Q *= |K*(y_i, y_{i-1})|
// |dOmega_g| ("other"), or the isotropic line (same interface, Q *= 1/2) or ray (descendant to
// ancestor) with a uniform pick among its q hits.  Returns T's factor
// q sign((y_i - y_{i-1}) . n(y_i)) (Eq. naive_woi_T), or 0 when no line or ray hit turned up
// within WOI_ATTEMPT_CAP draws (the walk stops there).  Draws come from st at `step`.
// coop: the wave shares the interface (shared schedule) -- rejection sampling on an ellipsoid is
// then done cooperatively (same points and counts).
template <typename R, int D, bool LDS>
__device__ __forceinline__ R transition(const DevProblem* __restrict__ dp, const R* __restrict__ pay,
                                        const DevRegion* g, int rel, const Stream& st, uint32_t step,
                                        const R y[D], int seg, R yn[D], int& segn, R& Q, int& qn, int& pick,
                                        int& att, Counts& cnt, const uint32_t* pre = nullptr, bool coop = false) {
    R nn[D];
    segn = 0; qn = 1; pick = 0;
    if (rel == REL_OTHER) {
        cnt.other++;
        if (D == 3 && g->kind == WOI_SHAPE_ELLIPSOID && wave_full(coop)) {
            auto try_at = [&](uint32_t c0, uint32_t c1, int a, R yy[D], int& sg) -> bool {
                const Stream s2{st.k0, st.k1, c0, c1, st.c2};
                return surf_attempt<R, D, LDS>(dp, *g, pay, s2, step, a, yy, sg);
            };
            att = coop_first_accept<R, D>(try_at, st.c0, st.c1, yn, segn, cnt);
        } else {
            for (att = 0; att < WOI_ATTEMPT_CAP; ++att) {
                if (surf_attempt<R, D, LDS>(dp, *g, pay, st, step, att, yn, segn, pre)) break;
                cnt.rejections++;
            }
            if (att == WOI_ATTEMPT_CAP) cnt.caps++;
        }
        normal_at<R, D, LDS>(*g, pay, yn, segn, nn);
        R dn = 0, r2 = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) { const R e = yn[j] - y[j]; dn += e * nn[j]; r2 += e * e; }
        R rm = R(1);
#pragma unroll
        for (int j = 0; j < D / 2; ++j) rm *= r2;
        if constexpr (D % 2) rm *= RO<R>::sq(r2);
        Q *= fabs(RO<R>::div(dn, Pay<R>::ua(dp) * rm)) * Pay<R>::area(*g);
    } else {
        const bool ray = rel == REL_DESC;
        constexpr int NW = dir_words(D) + 1, NB = (NW + 3) / 4;
        bool found = false;
        for (att = 0; att < WOI_ATTEMPT_CAP; ++att) {
            Words<NW> W; W.take(st, step, (uint32_t)(att * NB), pre);
            R d[D];
            unit_dir<R, D>(W, d);
            const R up = RO<R>::u(W.w[NW - 1]);
            if (g->kind == WOI_SHAPE_POLYLINE2D) {
                if constexpr (D == 2) {
                    int j = 0;
                    qn = poly_pick<R, LDS>(dp, *g, pay, y, d, ray, seg, up, pick, j, cnt);
                    if (qn == 0) { cnt.redraws++; continue; }
                    const R* v = poly_xy<R, LDS>(*g, pay) + 2 * j;
                    const R ex = v[2] - v[0], ey = v[3] - v[1];
                    const R den = d[0] * ey - d[1] * ex;
                    const R s = RO<R>::div((v[0] - y[0]) * d[1] - (v[1] - y[1]) * d[0], den);
                    yn[0] = v[0] + s * ex; yn[1] = v[1] + s * ey; segn = j;
                }
            } else if (D == 3 && LDS && g->kind == WOI_SHAPE_MESH3D) {
                if constexpr (D == 3) {
                    R t = 0;
                    int j = 0;
                    qn = mesh_pick<R>(dp, *g, pay, y, d, ray, seg, up, pick, t, j, cnt);
                    if (qn == 0) { cnt.redraws++; continue; }
#pragma unroll
                    for (int k = 0; k < D; ++k) yn[k] = y[k] + t * d[k];
                    segn = j;
                }
            } else {
                R t;
                qn = quadric_hit<R, D>(*g, pay, y, d, ray, t);
                if (qn == 0) { cnt.redraws++; continue; }
                pick = 0;
#pragma unroll
                for (int j = 0; j < D; ++j) yn[j] = y[j] + t * d[j];
            }
            found = true;
            break;
        }
        if (!found) { cnt.caps++; return R(0); }
        if (!ray) Q *= R(0.5);
        // A line or ray on a quadric (convex): the sign is + exactly -- the far end of a chord
        // through y has (yn - y) . A (yn - c) = t (b + t a), which is 2 b^2 / a for the line's
        // other root t = -2 b / a and t sqrt(b^2 - a cc) > 0 for a ray from inside.  FP32 walks
        // take it without the dot product (which they could only confirm or, inside its rounding
        // band, recheck to +); FP64 walks form it as the oracle does.
        if constexpr (std::is_same<R, float>::value)
            if (g->kind == WOI_SHAPE_SPHERE || g->kind == WOI_SHAPE_ELLIPSOID) return (R)qn;
        normal_at<R, D, LDS>(*g, pay, yn, segn, nn);
    }
    R dn = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) dn += (yn[j] - y[j]) * nn[j];
    if constexpr (std::is_same<R, float>::value) {
        if (fabsf(dn) <= dp->sign_band_f) {   // inside the FP32 rounding band: the sign from FP64
            cnt.fb++;
            dn = sign_fp64<D, LDS>(dp, *g, y, yn, segn);
        }
    }
    return dn < R(0) ? -(R)qn : (R)qn;
}

// ----------------------------------------------------------------------------- one sample
// Where a walker's terms c_i (y_i) go: accumulated at the lane's point, or stored as a
// trajectory for evaluation at a batch of points (shared trajectories, Sec. 4.6).
template <typename R, int D>
struct AccumSink {
    const DevProblem* dp;
    R xh[D], xl[D];
    R F, G[D];
    __device__ __forceinline__ void begin() {
        F = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) G[i] = 0;
    }
    __device__ __forceinline__ void add(int, R c, const R y[D], Counts& cnt) { add_term<R, D>(dp, xh, xl, y, c, F, G, cnt); }
    __device__ __forceinline__ void finish(int) {}
};

// Trajectory planes: component q (0 = c, 1.. = y) of step i of walker k of local sample s of
// group g sits at plane[q][((s K + k)(M + 1) + i) NG + g], g fastest (coalesced stores).
template <typename R, int D>
struct StoreSink {
    R* base;           // &plane[0][((s K + k)(M + 1)) NG + g]
    size_t plane;      // elements per plane
    int ng, M;
    bool on;           // lanes past the last group walk (keeping the wave uniform) but store nothing
    __device__ __forceinline__ void begin() {}
    __device__ __forceinline__ void add(int i, R c, const R y[D], Counts&) {
        if (!on) return;
        R* p = base + (size_t)i * ng;
        p[0] = c;
#pragma unroll
        for (int q = 0; q < D; ++q) p[(q + 1) * plane] = y[q];
    }
    __device__ __forceinline__ void finish(int i_next) {   // steps never reached contribute 0
        if (!on) return;
        for (int i = i_next; i <= M; ++i) {
            R* p = base + (size_t)i * ng;
            p[0] = R(0);
#pragma unroll
            for (int q = 0; q < D; ++q) p[(q + 1) * plane] = R(0);
        }
    }
};

// First point of a VR walker, drawn before its walk (see vr_starts).
template <typename R, int D>
struct Start {
    R y[D];
    int seg, att;
};

// floor(u(w) N) for u(w) = (w + 1/2) 2^-32: the FP64 product is exact (w + 1/2 has 33
// significant bits, N at most 32), so it equals ((2w + 1) N) >> 33 in integers.
__device__ __forceinline__ int region0(uint32_t w, int N) {
    return (int)((((uint64_t)w << 1 | 1u) * (uint64_t)N) >> 33);
}

// Region H_0 of sample w (Theorem 2: uniform over the regions); wave-uniform with the shared
// schedule.  The walker draws it from the same counter.  SH: the shared schedule is known at
// compile time (kp.shared_sched is then not read), so the compiler sees the schedule's region
// indices as uniform.
template <bool SH = false>
__device__ __forceinline__ int first_region(const DevProblem* __restrict__ dp, const KParams& kp, uint32_t w,
                                            uint32_t group) {
    const bool shared = SH || kp.shared_sched;
    const uint32_t inst = (kp.instance & 0xFFFFFFu) << 8;
    const uint4 sb = shared ? philox(make_uint4(w, 0xFFFFFFFFu, inst, 0u), kp.k0, kp.k1)
                            : philox(make_uint4(w, group, inst, 0u), kp.k0, kp.k1);
    const int t = region0(sb.x, dp->N);
    int h = t < dp->N ? t : dp->N - 1;
    if (shared) h = __builtin_amdgcn_readfirstlane(h);
    return h;
}

// First points of both walkers of a VR sample (Alg. 3: walker 0 on {beta >= 0}, walker 1 on
// {beta < 0} of dOmega_{H_0}) drawn by one rejection loop: each lane draws for whichever of
// its walkers still lacks a point, so a wave waits for its slowest lane once rather than once
// per walker.  Walker k keeps its own stream and attempt count, so the points, attempt counts
// and cap rule (after WOI_ATTEMPT_CAP attempts the last proposal is kept) are exactly those
// of drawing the walkers one after the other.  A walker whose half is empty draws nothing.
template <typename R, int D, bool LDS, bool SH = false>
__device__ __forceinline__ void vr_starts(const DevProblem* __restrict__ dp, const R* __restrict__ pay,
                                          const KParams& kp, uint32_t w, uint32_t group, int h, Start<R, D> s[2],
                                          Counts& cnt) {
    const DevRegion& g = dp->reg[h];
    const uint32_t inst = (kp.instance & 0xFFFFFFu) << 8;
    const Stream st0{kp.k0, kp.k1, w, group, inst | 1u};
    const Stream st1{kp.k0, kp.k1, w, group, inst | (1u << 4) | 1u};
    bool need0 = Pay<R>::meas(g, 0) != R(0), need1 = Pay<R>::meas(g, 1) != R(0);
    s[0].att = s[1].att = 0;
    s[0].seg = s[1].seg = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) { s[0].y[i] = R(0); s[1].y[i] = R(0); }
    if (D == 3 && wave_full(SH || kp.shared_sched)) {   // the same interface in every lane: cooperative
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (!(k ? need1 : need0)) continue;     // wave-uniform (the measures are the interface's)
            const Stream& sk = k ? st1 : st0;
            auto try_at = [&](uint32_t c0, uint32_t c1, int a, R yy[D], int& sg) -> bool {
                const Stream s2{sk.k0, sk.k1, c0, c1, sk.c2};
                return vr_attempt<R, D, LDS>(dp, g, pay, k, s2, a, yy, sg);
            };
            s[k].att = coop_first_accept<R, D>(try_at, sk.c0, sk.c1, s[k].y, s[k].seg, cnt);
        }
        return;
    }
    while (need0 || need1) {
        const int k = need0 ? 0 : 1;
        const int att = k ? s[1].att : s[0].att;
        R y[D];
        int seg = 0;
        const bool ok = vr_attempt<R, D, LDS>(dp, g, pay, k, k ? st1 : st0, att, y, seg);
        if (!ok) cnt.rejections++;
        const bool done = ok || att + 1 == WOI_ATTEMPT_CAP;
        if (!ok && done) cnt.caps++;
        Start<R, D>& t = k ? s[1] : s[0];
#pragma unroll
        for (int i = 0; i < D; ++i) t.y[i] = y[i];
        t.seg = seg;
        t.att = ok ? att : att + 1;
        if (k) need1 = !done;
        else need0 = !done;
    }
}

// Walker k of sample `w`: emits c_i and y_i, i = 0..M, to the sink (the accumulating sink
// forms sum_i c_i Phi(x, y_i) and sum_i c_i grad_x Phi; the caller multiplies by N).
// pre: the walker's first point drawn beforehand (VR, see vr_starts), or null.  SH: see
// first_region.
template <typename R, int D, bool VR, bool LDS, class Sink, bool SH = false>
__device__ __forceinline__ void walker(const DevProblem* __restrict__ dp, const R* __restrict__ pay,
                                       const KParams& kp, uint32_t w, uint32_t group, int k, Sink& sink,
                                       uint32_t* __restrict__ tr, Counts& cnt, const Start<R, D>* pre = nullptr) {
    const int N = dp->N, M = kp.M;
    const bool shared = SH || kp.shared_sched;
    const uint32_t inst = (kp.instance & 0xFFFFFFu) << 8;
    // Schedule words: counter (w, group or all-ones, instance, draw).  With the shared schedule
    // every input is wave-uniform and the block runs on the scalar unit.
    auto sched_block = [&](uint32_t draw) -> uint4 {
        if (shared) return philox(make_uint4(w, 0xFFFFFFFFu, inst, draw), kp.k0, kp.k1);
        return philox(make_uint4(w, group, inst, draw), kp.k0, kp.k1);
    };
    const Stream st{kp.k0, kp.k1, w, group, inst | ((uint32_t)k << 4) | 1u};
    sink.begin();

    // schedule H_0 (Theorem 2): uniform over regions
    uint4 sb = sched_block(0);
    int h;
    {
        int t = region0(sb.x, N);
        h = t < N ? t : N - 1;
        if (shared) h = __builtin_amdgcn_readfirstlane(h);
    }
    const DevRegion* g = &dp->reg[h];
    const R meas = VR ? Pay<R>::meas(*g, k) : Pay<R>::area(*g);
    if (meas == R(0)) {   // empty VR half: the walker contributes nothing
        if (tr) for (int i = 0; i <= M; ++i) tr[i] = i ? 0u : trace_word(h, 0, 0, 0, 0, 0);
        sink.finish(0);
        return;
    }
    R y[D];
    int seg = 0, att;
    if (pre) {
#pragma unroll
        for (int i = 0; i < D; ++i) y[i] = pre->y[i];
        seg = pre->seg;
        att = pre->att;
    } else {
        if (!VR && D == 3 && g->kind == WOI_SHAPE_ELLIPSOID && wave_full(shared)) {
            auto try_at = [&](uint32_t c0, uint32_t c1, int a, R yy[D], int& sg) -> bool {
                const Stream s2{st.k0, st.k1, c0, c1, st.c2};
                return surf_attempt<R, D, LDS>(dp, *g, pay, s2, 0, a, yy, sg);
            };
            att = coop_first_accept<R, D>(try_at, st.c0, st.c1, y, seg, cnt);
        } else {
            for (att = 0; att < WOI_ATTEMPT_CAP; ++att) {
                bool ok;
                if constexpr (VR) ok = vr_attempt<R, D, LDS>(dp, *g, pay, k, st, att, y, seg);
                else ok = surf_attempt<R, D, LDS>(dp, *g, pay, st, 0, att, y, seg);
                if (ok) break;
                cnt.rejections++;
            }
            if (att == WOI_ATTEMPT_CAP) cnt.caps++;
        }
    }
    R Q = Pay<R>::s(*g) * data_b<R, D, LDS>(dp, *g, pay, y, seg) * meas, T = 1;
    sink.add(0, (M == 0 ? R(0.5) : R(1)) * Q * T, y, cnt);
    cnt.steps++;
    if (tr) tr[0] = trace_word(h, 0, 1, 0, 0, att);
    int done = 1;
    R S = 1, pw = 1;
    const R l1 = Pay<R>::l1(dp);
    uint4 pb = make_uint4(0u, 0u, 0u, 0u);
    for (int i = 1; i <= M; ++i) {
        if ((i & 3) == 0) sb = sched_block((uint32_t)(i >> 2));
        const uint32_t wv = (i & 3) == 0 ? sb.x : (i & 3) == 1 ? sb.y : (i & 3) == 2 ? sb.z : sb.w;
        // inverse CDF: the first region with u(wv) < cdf, searched from the guide entry of u(wv)
        // (floor(64 u(wv)) = wv >> 26; the CDF test in integers, see DevProblem::sthr)
        int hn = dp->sguide[wv >> 26];
        while (hn < N - 1 && !((uint64_t)wv < dp->sthr[hn])) ++hn;
        if (shared) hn = __builtin_amdgcn_readfirstlane(hn);
        const int rel = dp->rel[h][hn];
        h = hn;
        g = &dp->reg[h];
        S *= Pay<R>::sgn(*g);
        pw *= l1;
        R yn[D];
        int segn = 0, qn = 1, pick = 0;
        // 2D: the first attempts of steps 2k+1 and 2k+2 share one block (two words each)
        uint32_t pre[2] = {0u, 0u};
        if constexpr (D == 2) {
            if (i & 1) pb = st.block(0x8000u | (uint32_t)((i - 1) >> 1), 0u);
            pre[0] = (i & 1) ? pb.x : pb.z;
            pre[1] = (i & 1) ? pb.y : pb.w;
        }
        const R tf = transition<R, D, LDS>(dp, pay, g, rel, st, (uint32_t)i, y, seg, yn, segn, Q, qn, pick, att,
                                                cnt, D == 2 ? pre : nullptr, shared);
        if (tf == R(0)) {   // no hit after the attempt cap: the walker stops here
            if (tr) for (int j = i; j <= M; ++j) tr[j] = trace_word(h, rel, 0, 0, 0, att);
            break;
        }
        T *= tf;
#pragma unroll
        for (int j = 0; j < D; ++j) y[j] = yn[j];
        seg = segn;
        sink.add(i, (i == M ? R(0.5) : R(1)) * pw * S * Q * T, y, cnt);
        cnt.steps++;
        done = i + 1;
        if (tr) tr[i] = trace_word(h, rel, qn, pick, tf < R(0), att);
    }
    sink.finish(done);
}

// ----------------------------------------------------------------------------- kernels
template <typename R, int D>
__device__ __forceinline__ void load_point(const double* __restrict__ pts, int64_t p, R xh[D], R xl[D]) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const double v = pts[p * D + i];
        xh[i] = (R)v;
        xl[i] = (R)(v - (double)xh[i]);
    }
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Stage every polyline's FP32 vertices and FP16 block bounds into LDS (LDS variant), and its
// FP32 arclength CDF and guide table where the problem's layout gives them room.
__device__ __forceinline__ void stage_polylines(const DevProblem* __restrict__ dp) {
    const float* __restrict__ f32 = Pay<float>::base(dp);
    for (int i = 0; i < dp->N; ++i) {
        const DevRegion& g = dp->reg[i];
        if (g.lds_v < 0) continue;
        float2* dv = reinterpret_cast<float2*>(woi_smem + g.lds_v);
        const float2* sv = reinterpret_cast<const float2*>(f32 + g.g32);
        for (int t = threadIdx.x; t <= g.n2; t += blockDim.x) dv[t] = sv[t];   // padded copy
        __half* db = reinterpret_cast<__half*>(woi_smem + g.lds_b);
        for (int t = threadIdx.x; t < g.n2 + g.nv; t += blockDim.x) db[t] = __float2half_ru(f32[g.bnd + t]);
        if (g.lds_c < 0) continue;
        float2* dc = reinterpret_cast<float2*>(woi_smem + g.lds_c);
        const float2* sc = reinterpret_cast<const float2*>(f32 + g.cum32);
        for (int t = threadIdx.x; t <= g.nv; t += blockDim.x) dc[t] = sc[t];
        int* dg = reinterpret_cast<int*>(woi_smem + g.lds_g);
        const int* sg = int_payload(dp) + g.guide;
        for (int t = threadIdx.x; t < g.nv; t += blockDim.x) dg[t] = sg[t];
    }
    __syncthreads();
}

// Running (n, mean, M2) of per-sample values, merged chunk by chunk from the chunk's sample
// count and FP64 sums of values and squares (Chan, Golub & LeVeque's pairwise update).
struct Moments {
    double n, mu, m2;
    __device__ __forceinline__ void merge(double nc, double s1, double s2) {
        const double mc = s1 / nc, m2c = s2 - s1 * mc, nt = n + nc, dl = mc - mu;
        mu += dl * nc / nt;
        m2 += m2c + dl * dl * n * nc / nt;
        n = nt;
    }
    // merge another running triple (the same update with the other side's mean and M2)
    __device__ __forceinline__ void combine(const Moments& b) {
        const double nt = n + b.n;
        if (nt == 0) return;
        const double dl = b.mu - mu;
        mu += dl * b.n / nt;
        m2 += b.m2 + dl * dl * n * b.n / nt;
        n = nt;
    }
    // standard error of the mean
    __device__ __forceinline__ double se() const { return n > 1 ? sqrt(fmax(m2, 0.0) / (n - 1) / n) : 0.0; }
};

__device__ __forceinline__ Moments shfl_xor_moments(const Moments& a, int o) {
    return Moments{__shfl_xor(a.n, o, 64), __shfl_xor(a.mu, o, 64), __shfl_xor(a.m2, o, 64)};
}

// Merge one partial record (sum F, sum F^2, sum G[D], sum G^2[D]) of nc samples.
__device__ __forceinline__ void merge_partial(Moments& f, Moments* g, int D, double nc, const double* __restrict__ o) {
    f.merge(nc, o[0], o[1]);
    for (int i = 0; i < D; ++i) g[i].merge(nc, o[2 + i], o[2 + D + i]);
}

__device__ __forceinline__ void store_moments(const Moments& f, const Moments* g, int D, int64_t p, double* mean,
                                              double* se, double* grad, double* grad_se) {
    mean[p] = f.mu;
    se[p] = f.se();
    for (int i = 0; i < D; ++i) {
        if (grad) grad[p * D + i] = g[i].mu;
        if (grad_se) grad_se[p * D + i] = g[i].se();
    }
}

}  // namespace woi
