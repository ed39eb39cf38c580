// woi_training.hip -- training data of the neural-network surrogate (Sec. 5, Eq. MLP_loss):
// interior grid points inside dOmega and boundary points with normals and flux targets, made on
// the device; the WoI estimates at the interior points come from woi_estimate.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "woi_device.h"
#include "woi_launch.h"
#include "woi_walk.h"

namespace woi {

// x strictly inside interface g (sphere, ellipsoid: the quadric form; polyline: crossing number
// of the ray x + t e_1, t > 0)
template <int D>
__device__ bool train_inside(const DevRegion& g, const double* pay, const double x[D]) {
    const double* q = pay + g.g64;
    if (g.kind == WOI_SHAPE_SPHERE) {
        double r2 = 0;
        for (int i = 0; i < D; ++i) r2 += (x[i] - q[i]) * (x[i] - q[i]);
        return r2 < q[D] * q[D];
    }
    if (g.kind == WOI_SHAPE_ELLIPSOID) {
        double s = 0;
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) s += (x[i] - q[i]) * q[D + i * D + j] * (x[j] - q[j]);
        return s < 1.0;
    }
    bool in = false;
    if constexpr (D == 2) {
        for (int j = 0; j < g.nv; ++j) {
            const double *a = q + 2 * j, *b = q + 2 * j + 2;
            if ((a[1] > x[1]) != (b[1] > x[1])) {
                const double xi = a[0] + (x[1] - a[1]) / (b[1] - a[1]) * (b[0] - a[0]);
                if (x[0] < xi) in = !in;
            }
        }
    }
    return in;
}

// distance of x from interface g (ellipsoid: the first-order level-set distance |q - 1| / |grad q|)
template <int D>
__device__ double train_distance(const DevRegion& g, const double* pay, const double x[D]) {
    const double* q = pay + g.g64;
    if (g.kind == WOI_SHAPE_SPHERE) {
        double r2 = 0;
        for (int i = 0; i < D; ++i) r2 += (x[i] - q[i]) * (x[i] - q[i]);
        return fabs(sqrt(r2) - q[D]);
    }
    if (g.kind == WOI_SHAPE_ELLIPSOID) {
        double s = 0, gn = 0;
        for (int i = 0; i < D; ++i) {
            double t = 0;
            for (int j = 0; j < D; ++j) t += q[D + i * D + j] * (x[j] - q[j]);
            s += (x[i] - q[i]) * t;
            gn += t * t;
        }
        return fabs(s - 1.0) / (2.0 * sqrt(gn));
    }
    double best = INFINITY;
    if constexpr (D == 2) {
        for (int j = 0; j < g.nv; ++j) {
            const double *a = q + 2 * j, *b = q + 2 * j + 2;
            const double ex = b[0] - a[0], ey = b[1] - a[1], l2 = ex * ex + ey * ey;
            double s = ((x[0] - a[0]) * ex + (x[1] - a[1]) * ey) / l2;
            s = s < 0 ? 0 : (s > 1 ? 1 : s);
            const double dx = x[0] - (a[0] + s * ex), dy = x[1] - (a[1] + s * ey), dd = sqrt(dx * dx + dy * dy);
            best = dd < best ? dd : best;
        }
    }
    return best;
}

// Interior nodes, in grid order: one workgroup walks the grid 1024 nodes at a time and places the
// nodes it keeps by a workgroup prefix count, so the output order does not depend on scheduling.
template <int D>
__global__ __launch_bounds__(1024) void train_grid_kernel(TrainParams tp) {
    __shared__ uint32_t wsum[16];
    __shared__ unsigned long long base;
    const DevProblem* dp = tp.dp;
    const double* pay = Pay<double>::base(dp);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (uint64_t c0 = 0; c0 < tp.nodes; c0 += blockDim.x) {
        const uint64_t k = c0 + threadIdx.x;
        double x[D];
        bool keep = false;
        if (k < tp.nodes) {
            uint64_t r = k;
            for (int d = D - 1; d >= 0; --d) {
                x[d] = tp.lo[d] + ((double)(r % (uint64_t)tp.n) + 0.5) * tp.step[d];
                r /= (uint64_t)tp.n;
            }
            keep = train_inside<D>(dp->reg[0], pay, x);
            if (keep && tp.margin > 0)
                for (int i = 0; i < dp->N && keep; ++i) keep = train_distance<D>(dp->reg[i], pay, x) > tp.margin;
        }
        const uint64_t ball = __ballot(keep);
        if (lane == 0) wsum[wv] = (uint32_t)__popcll(ball);
        __syncthreads();
        uint64_t pos = base + (uint64_t)__popcll(ball & ((1ull << lane) - 1ull));
        for (int w = 0; w < wv; ++w) pos += wsum[w];
        if (keep && pos < (uint64_t)tp.cap)
            for (int d = 0; d < D; ++d) tp.out[pos * D + d] = x[d];
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += wsum[w];
            base += t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *tp.count = (int64_t)base;
}

// Boundary node k: 2D angle 2 pi k / n (circle about its centre, polyline: the farthest crossing of
// the ray from its vertex mean); 3D polar angle pi (i + 1/2) / n, azimuth pi j / n, j < 2 n, through
// the sphere or ellipsoid parametrisation.  Outward normal and b_1 / sigma_1.
template <int D>
__global__ __launch_bounds__(256) void train_boundary_kernel(TrainParams tp) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= tp.n_bc) return;
    const DevProblem* dp = tp.dp;
    const double* pay = Pay<double>::base(dp);
    const DevRegion& g = dp->reg[0];
    const double* q = pay + g.g64;
    double y[D], n[D];
    int seg = 0;
    for (int a = 0; a < D; ++a) y[a] = 0;
    if constexpr (D == 2) {
        const double th = 2 * 3.14159265358979323846 * (double)k / tp.bc_n, d0 = cos(th), d1 = sin(th);
        if (g.kind == WOI_SHAPE_SPHERE) {
            y[0] = q[0] + q[2] * d0;
            y[1] = q[1] + q[2] * d1;
        } else {
            double z0 = 0, z1 = 0, tbest = -1;
            for (int j = 0; j < g.nv; ++j) { z0 += q[2 * j] / g.nv; z1 += q[2 * j + 1] / g.nv; }
            for (int j = 0; j < g.nv; ++j) {
                const double *a = q + 2 * j, *b = q + 2 * j + 2;
                const double ex = b[0] - a[0], ey = b[1] - a[1], den = d0 * ey - d1 * ex;
                if (den == 0) continue;
                const double t = ((a[0] - z0) * ey - (a[1] - z1) * ex) / den;
                const double sp = ((a[0] - z0) * d1 - (a[1] - z1) * d0) / den;
                if (sp < 0 || sp >= 1 || !(t > 0) || t <= tbest) continue;
                tbest = t;
                seg = j;
                y[0] = a[0] + sp * ex;
                y[1] = a[1] + sp * ey;
            }
        }
    } else if constexpr (D == 3) {
        const int64_t i = k / (2 * tp.bc_n), j = k % (2 * tp.bc_n);
        const double pi = 3.14159265358979323846;
        const double th = pi * ((double)i + 0.5) / tp.bc_n, ph = pi * (double)j / tp.bc_n;
        const double u[3] = {sin(th) * cos(ph), sin(th) * sin(ph), cos(th)};
        if (g.kind == WOI_SHAPE_SPHERE) {
            for (int a = 0; a < 3; ++a) y[a] = q[a] + q[3] * u[a];
        } else {   // L = A^{-1/2} after the centre and A
            for (int a = 0; a < 3; ++a) {
                double t = 0;
                for (int b = 0; b < 3; ++b) t += q[3 + 9 + a * 3 + b] * u[b];
                y[a] = q[a] + t;
            }
        }
    }
    normal_at<double, D, false>(g, pay, y, seg, n);
    for (int a = 0; a < D; ++a) {
        tp.bc_points[k * D + a] = y[a];
        tp.bc_normals[k * D + a] = n[a];
    }
    tp.bc_flux[k] = data_b<double, D, false>(dp, g, pay, y, seg) * (0.5 * g.s);   // s = 2 / sigma_1
}

hipError_t launch_training(const TrainParams& tp, int dim, hipStream_t s) {
    if (dim == 2) {
        hipLaunchKernelGGL(train_grid_kernel<2>, dim3(1), dim3(1024), 0, s, tp);
        if (tp.n_bc > 0)
            hipLaunchKernelGGL(train_boundary_kernel<2>, dim3((unsigned)((tp.n_bc + 255) / 256)), dim3(256), 0, s, tp);
    } else if (dim == 3) {
        hipLaunchKernelGGL(train_grid_kernel<3>, dim3(1), dim3(1024), 0, s, tp);
        if (tp.n_bc > 0)
            hipLaunchKernelGGL(train_boundary_kernel<3>, dim3((unsigned)((tp.n_bc + 255) / 256)), dim3(256), 0, s, tp);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace woi
