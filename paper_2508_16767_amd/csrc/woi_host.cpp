// woi_host.cpp -- problem compiler and C ABI of the Walk-on-Interfaces library.
//
// Problem compile (once per problem, host FP64):
//   alpha_i, beta scalings                      Eq. unit_coeff_charge_density_sys
//   schedule CDF over |alpha| / ||alpha||_1     Theorem 2, Eq. scheduled_interface_pdf
//   relation of consecutive interfaces          Eq. naive_woi_p (same / descendant / other)
//   surface measures |dOmega_i|                 Eqs. naive_woi_p0, naive_woi_p
//   halves {beta >= 0}, {beta < 0}              Sec. 4.4 (variance reduction)
//   compatibility  int b_i dA = 0               Sec. 1 (after Eq. interface_problem)
// then one device upload.  Estimation launches the walk kernel over (point tile, sample
// chunk) and a deterministic reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <functional>
#include <atomic>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "woi.h"
#include "woi_device.h"
#include "woi_internal.h"
#include "woi_launch.h"

using woi::DevProblem;
using woi::DevRegion;

namespace {

thread_local std::string g_err;

woi_status fail(woi_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------- small linear algebra
// Symmetric eigen-decomposition by cyclic Jacobi rotations: A = V diag(ev) V^T.
void sym_eig(int m, const double* A, double* ev, double* V) {
    double a[WOI_MAX_DIM * WOI_MAX_DIM];
    std::memcpy(a, A, sizeof(double) * m * m);
    for (int i = 0; i < m * m; ++i) V[i] = 0.0;
    for (int i = 0; i < m; ++i) V[i * m + i] = 1.0;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j)
                if (i != j) off += a[i * m + j] * a[i * m + j];
        if (off < 1e-280) break;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = a[p * m + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double tau = (a[q * m + q] - a[p * m + p]) / (2.0 * apq);
                const double t = std::copysign(1.0, tau) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < m; ++k) {
                    const double x = a[k * m + p], y = a[k * m + q];
                    a[k * m + p] = c * x - s * y;
                    a[k * m + q] = s * x + c * y;
                }
                for (int k = 0; k < m; ++k) {
                    const double x = a[p * m + k], y = a[q * m + k];
                    a[p * m + k] = c * x - s * y;
                    a[q * m + k] = s * x + c * y;
                }
                for (int k = 0; k < m; ++k) {
                    const double x = V[k * m + p], y = V[k * m + q];
                    V[k * m + p] = c * x - s * y;
                    V[k * m + q] = s * x + c * y;
                }
            }
    }
    for (int i = 0; i < m; ++i) ev[i] = a[i * m + i];
}

// Gauss-Legendre rule on [-1, 1] (Golub-Welsch free: Newton iteration on P_n).
void gl_rule(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 60; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// ---------------------------------------------------------------------------- host geometry
struct HostRegion {
    int kind = 0, dkind = 0, nt = 0;
    double c[WOI_MAX_DIM] = {0}, R = 0;
    double A[WOI_MAX_DIM * WOI_MAX_DIM] = {0}, L[WOI_MAX_DIM * WOI_MAX_DIM] = {0};
    double lam_max = 0, detL = 1;
    std::vector<double> v;      // polyline vertices, closed (nv + 1)
    std::vector<double> len, cum;
    double total = 0, area = 0;
    std::vector<double> coef;   // data payload: coefficients then centre / source
    std::vector<uint8_t> exps;
    double alpha = 0, s = 0, flux = 0, absflux = 0;
    double meas[2] = {0, 0};
    std::vector<double> brk;
    int class0 = 0;
    std::vector<double> mv;     // mesh vertices (3 each)
    std::vector<int> tri;       // mesh triangles (3 vertex indices each); cum holds cumulative areas
    std::vector<double> tn;     // mesh unit outward normals (3 per triangle)
    int nv() const { return (int)len.size(); }
    int ntri() const { return (int)tri.size() / 3; }
};

struct Host {
    int m = 0, N = 0;
    int parent[WOI_MAX_REGIONS] = {0};
    double sigma[WOI_MAX_REGIONS] = {0};
    HostRegion r[WOI_MAX_REGIONS];
    double alpha_l1 = 0;
};

void outward_normal(const Host& H, const HostRegion& g, const double* y, int seg, double* n) {
    const int m = H.m;
    if (g.kind == WOI_SHAPE_SPHERE) {
        for (int i = 0; i < m; ++i) n[i] = (y[i] - g.c[i]) / g.R;
    } else if (g.kind == WOI_SHAPE_ELLIPSOID) {
        double nn = 0;
        for (int i = 0; i < m; ++i) {
            double t = 0;
            for (int j = 0; j < m; ++j) t += g.A[i * m + j] * (y[j] - g.c[j]);
            n[i] = t;
            nn += t * t;
        }
        nn = std::sqrt(nn);
        for (int i = 0; i < m; ++i) n[i] /= nn;
    } else if (g.kind == WOI_SHAPE_MESH3D) {
        for (int i = 0; i < 3; ++i) n[i] = g.tn[3 * seg + i];
    } else {
        const double ex = g.v[2 * seg + 2] - g.v[2 * seg], ey = g.v[2 * seg + 3] - g.v[2 * seg + 1];
        const double l = std::sqrt(ex * ex + ey * ey);
        n[0] = ey / l;
        n[1] = -ex / l;
    }
}

// Ray y + t d (t > 0) against triangle (a, b, c): true on a hit (barycentric test).
bool ray_hits_triangle(const double* y, const double* d, const double* a, const double* b, const double* c) {
    double e1[3], e2[3], w[3];
    for (int k = 0; k < 3; ++k) { e1[k] = b[k] - a[k]; e2[k] = c[k] - a[k]; w[k] = y[k] - a[k]; }
    const double p[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    const double det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
    if (det == 0) return false;
    const double u = (w[0] * p[0] + w[1] * p[1] + w[2] * p[2]) / det;
    if (u < 0 || u > 1) return false;
    const double q[3] = {w[1] * e1[2] - w[2] * e1[1], w[2] * e1[0] - w[0] * e1[2], w[0] * e1[1] - w[1] * e1[0]};
    const double v = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) / det;
    if (v < 0 || u + v > 1) return false;
    return (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) / det > 0;
}

// b_i(y): data payload layout matches the device (coefficients, then centre / source)
double b_value(const Host& H, const HostRegion& g, const double* y, int seg) {
    const int m = H.m;
    switch (g.dkind) {
        case WOI_DATA_ZERO: return 0.0;
        case WOI_DATA_FIELD_FLUX: {
            double n[WOI_MAX_DIM], b = 0;
            outward_normal(H, g, y, seg, n);
            for (int i = 0; i < m; ++i) b += g.coef[i] * n[i];
            return b;
        }
        case WOI_DATA_SOURCE_FLUX: {
            double n[WOI_MAX_DIM], dn = 0, r2 = 0;
            outward_normal(H, g, y, seg, n);
            for (int i = 0; i < m; ++i) {
                const double e = y[i] - g.coef[1 + i];
                dn += e * n[i];
                r2 += e * e;
            }
            return g.coef[0] * dn / std::pow(r2, 0.5 * m);
        }
        default: break;
    }
    const int nc = g.dkind == WOI_DATA_FOURIER2D ? 2 * g.nt + 1 : g.nt;
    const double* c = g.coef.data() + nc;
    double e[WOI_MAX_DIM], r2 = 0;
    for (int i = 0; i < m; ++i) {
        e[i] = y[i] - c[i];
        r2 += e[i] * e[i];
    }
    const double ir = 1.0 / std::sqrt(r2);
    for (int i = 0; i < m; ++i) e[i] *= ir;
    if (g.dkind == WOI_DATA_FOURIER2D) {
        const double th = std::atan2(e[1], e[0]);
        double b = g.coef[0];
        for (int k = 1; k <= g.nt; ++k) b += g.coef[2 * k - 1] * std::cos(k * th) + g.coef[2 * k] * std::sin(k * th);
        return b;
    }
    double b = 0;
    for (int t = 0; t < g.nt; ++t) {
        double term = g.coef[t];
        for (int i = 0; i < m; ++i)
            for (int p = 0; p < g.exps[t * m + i]; ++p) term *= e[i];
        b += term;
    }
    return b;
}

// point of a sphere / ellipsoid from a unit vector u, and the surface Jacobian
void quadric_point(const Host& H, const HostRegion& g, const double* u, double* y, double* J) {
    const int m = H.m;
    if (g.kind == WOI_SHAPE_SPHERE) {
        for (int i = 0; i < m; ++i) y[i] = g.c[i] + g.R * u[i];
        *J = std::pow(g.R, m - 1);
        return;
    }
    double uAu = 0;
    for (int i = 0; i < m; ++i) {
        double t = 0, l = 0;
        for (int j = 0; j < m; ++j) {
            t += g.A[i * m + j] * u[j];
            l += g.L[i * m + j] * u[j];
        }
        uAu += u[i] * t;
        y[i] = g.c[i] + l;
    }
    *J = g.detL * std::sqrt(uAu);
}

// Integral over S^{m-1} in hyperspherical angles: Gauss-Legendre in each polar angle
// (nodes np per angle), periodic trapezoid (2 np nodes) in the azimuth.
template <class F>
double sphere_quad(int m, int np, F&& f) {
    if (m == 2) {
        const int n = 8 * np;
        double s = 0;
        for (int j = 0; j < n; ++j) {
            const double ph = 2 * kPi * (j + 0.5) / n;
            const double u[2] = {std::cos(ph), std::sin(ph)};
            s += f(u);
        }
        return s * 2 * kPi / n;
    }
    std::vector<double> gx, gw;
    gl_rule(np, gx, gw);
    const int npol = m - 2, naz = 2 * np;
    std::vector<int> idx(npol, 0);
    double total = 0;
    while (true) {
        double u[WOI_MAX_DIM], w = 1, sprod = 1;
        for (int a = 0; a < npol; ++a) {
            const double th = 0.5 * kPi * (gx[idx[a]] + 1.0);
            u[a] = sprod * std::cos(th);
            w *= 0.5 * kPi * gw[idx[a]] * std::pow(std::sin(th), m - 2 - a);
            sprod *= std::sin(th);
        }
        for (int j = 0; j < naz; ++j) {
            const double ph = 2 * kPi * (j + 0.5) / naz;
            u[m - 2] = sprod * std::cos(ph);
            u[m - 1] = sprod * std::sin(ph);
            total += w * (2 * kPi / naz) * f(u);
        }
        int a = 0;
        while (a < npol && ++idx[a] == np) idx[a++] = 0;
        if (a == npol) break;
    }
    return total;
}

int quad_order(int m) { return m == 2 ? 256 : m == 3 ? 96 : m == 4 ? 48 : m == 5 ? 32 : m == 6 ? 24 : 16; }

bool point_inside(const Host& H, const HostRegion& g, const double* y) {
    const int m = H.m;
    if (g.kind == WOI_SHAPE_SPHERE) {
        double r2 = 0;
        for (int i = 0; i < m; ++i) r2 += (y[i] - g.c[i]) * (y[i] - g.c[i]);
        return r2 < g.R * g.R;
    }
    if (g.kind == WOI_SHAPE_ELLIPSOID) {
        double q = 0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) q += (y[i] - g.c[i]) * g.A[i * m + j] * (y[j] - g.c[j]);
        return q < 1.0;
    }
    if (g.kind == WOI_SHAPE_MESH3D) {   // parity of the crossings of a ray in a fixed skew direction
        static const double d[3] = {0.5376448, 0.6427876, 0.5457595};
        bool in = false;
        for (int j = 0; j < g.ntri(); ++j) {
            const int* t = &g.tri[3 * j];
            if (ray_hits_triangle(y, d, &g.mv[3 * t[0]], &g.mv[3 * t[1]], &g.mv[3 * t[2]])) in = !in;
        }
        return in;
    }
    bool in = false;   // crossing number
    for (int j = 0; j < g.nv(); ++j) {
        const double* a = &g.v[2 * j];
        const double* b = &g.v[2 * j + 2];
        if ((a[1] > y[1]) != (b[1] > y[1])) {
            const double xi = a[0] + (y[1] - a[1]) / (b[1] - a[1]) * (b[0] - a[0]);
            if (y[0] < xi) in = !in;
        }
    }
    return in;
}

// deterministic sample points on an interface for validation
void probe_points(const Host& H, const HostRegion& g, std::vector<double>& pts) {
    const int m = H.m;
    pts.clear();
    if (g.kind == WOI_SHAPE_MESH3D) {   // vertices and triangle centroids
        pts = g.mv;
        for (int j = 0; j < g.ntri(); ++j)
            for (int k = 0; k < 3; ++k)
                pts.push_back((g.mv[3 * g.tri[3 * j] + k] + g.mv[3 * g.tri[3 * j + 1] + k] + g.mv[3 * g.tri[3 * j + 2] + k]) / 3.0);
        return;
    }
    if (g.kind == WOI_SHAPE_POLYLINE2D) {
        for (int j = 0; j < g.nv(); ++j)
            for (int s = 0; s < 2; ++s) {
                const double f = 0.5 * s;
                pts.push_back(g.v[2 * j] + f * (g.v[2 * j + 2] - g.v[2 * j]));
                pts.push_back(g.v[2 * j + 1] + f * (g.v[2 * j + 3] - g.v[2 * j + 1]));
            }
        return;
    }
    // Fibonacci-like lattice on S^{m-1} via low-discrepancy Gaussian directions
    const int n = m == 2 ? 720 : 4000;
    uint64_t st = 0x9E3779B97F4A7C15ull;
    for (int k = 0; k < n; ++k) {
        double u[WOI_MAX_DIM], nn = 0;
        for (int i = 0; i < m; ++i) {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            const double a = ((st >> 11) + 0.5) * 0x1p-53;
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            const double b = ((st >> 11) + 0.5) * 0x1p-53;
            u[i] = std::sqrt(-2 * std::log(a)) * std::cos(2 * kPi * b);
            nn += u[i] * u[i];
        }
        nn = std::sqrt(nn);
        for (int i = 0; i < m; ++i) u[i] /= nn;
        if (m == 2) {
            u[0] = std::cos(2 * kPi * (k + 0.5) / n);
            u[1] = std::sin(2 * kPi * (k + 0.5) / n);
        }
        double y[WOI_MAX_DIM], J;
        quadric_point(H, g, u, y, &J);
        for (int i = 0; i < m; ++i) pts.push_back(y[i]);
    }
}

// ---------------------------------------------------------------------------- VR halves
double curve_beta(const Host& H, const HostRegion& g, double s) {
    double y[2];
    int seg = 0;
    if (g.kind == WOI_SHAPE_POLYLINE2D) {
        const int n = g.nv();
        int j = (int)(std::upper_bound(g.cum.begin(), g.cum.begin() + n, s) - g.cum.begin()) - 1;
        j = std::max(0, std::min(j, n - 1));
        const double f = (s - g.cum[j]) / g.len[j];
        y[0] = g.v[2 * j] + f * (g.v[2 * j + 2] - g.v[2 * j]);
        y[1] = g.v[2 * j + 1] + f * (g.v[2 * j + 3] - g.v[2 * j + 1]);
        seg = j;
    } else {
        y[0] = g.c[0] + g.R * std::cos(s / g.R);
        y[1] = g.c[1] + g.R * std::sin(s / g.R);
    }
    return g.s * b_value(H, g, y, seg);
}

void vr_halves_2d(const Host& H, HostRegion& g) {
    const int n = g.kind == WOI_SHAPE_POLYLINE2D ? 16 * g.nv() : 16384;
    g.brk.clear();
    auto cls = [&](double s) { return curve_beta(H, g, s) >= 0.0 ? 0 : 1; };
    int c_prev = cls(0.0);
    g.class0 = c_prev;
    double s_prev = 0.0;
    for (int j = 1; j <= n; ++j) {
        const double s = g.total * j / n;
        const int c = j == n ? g.class0 : cls(s);
        if (c != c_prev) {
            double lo = s_prev, hi = s;
            const int clo = c_prev;
            for (int it = 0; it < 80; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                if (cls(mid) == clo) lo = mid; else hi = mid;
            }
            g.brk.push_back(0.5 * (lo + hi));
        }
        s_prev = s;
        c_prev = c;
    }
    g.meas[0] = g.meas[1] = 0.0;
    double start = 0.0;
    int c = g.class0;
    for (size_t p = 0; p <= g.brk.size(); ++p) {
        const double end = p < g.brk.size() ? g.brk[p] : g.total;
        g.meas[c] += end - start;
        start = end;
        c ^= 1;
    }
}

// 3D halves: for each polar angle th, exact breakpoints of sign(beta) along the azimuth,
// Gauss-Legendre (5 nodes) for the surface Jacobian on every piece; adaptive
// Gauss-Kronrod (7/15) over th.
double ring_measure(const Host& H, const HostRegion& g, double th, int want) {
    const int n = 192;
    static const double x5[5] = {-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831, 0.9061798459386640};
    static const double w5[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889, 0.4786286704993665, 0.2369268850561891};
    const double st = std::sin(th), ct = std::cos(th);
    auto eval = [&](double ph, double* J) {
        const double u[3] = {st * std::cos(ph), st * std::sin(ph), ct};
        double y[3];
        quadric_point(H, g, u, y, J);
        return g.s * b_value(H, g, y, 0) >= 0.0 ? 0 : 1;
    };
    auto piece = [&](double a, double b) {
        double s = 0, J;
        for (int k = 0; k < 5; ++k) {
            eval(0.5 * (a + b) + 0.5 * (b - a) * x5[k], &J);
            s += 0.5 * (b - a) * w5[k] * J;
        }
        return s;
    };
    double total = 0, J;
    int ca = eval(0.0, &J);
    for (int j = 0; j < n; ++j) {
        const double a = 2 * kPi * j / n, b = 2 * kPi * (j + 1) / n;
        const int cb = eval(b, &J);
        if (ca == cb) {
            if (ca == want) total += piece(a, b);
        } else {
            double lo = a, hi = b;
            for (int it = 0; it < 80; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                if (eval(mid, &J) == ca) lo = mid; else hi = mid;
            }
            const double r = 0.5 * (lo + hi);
            total += ca == want ? piece(a, r) : piece(r, b);
        }
        ca = cb;
    }
    return total * st;
}

double gk15(const Host& H, const HostRegion& g, int want, double a, double b, double* err) {
    static const double xk[8] = {0.991455371120812639, 0.949107912342758525, 0.864864423359769073, 0.741531185599394440,
                                 0.586087235467691130, 0.405845151377397167, 0.207784955007898468, 0.0};
    static const double wk[8] = {0.022935322010529225, 0.063092092629978553, 0.104790010322250184, 0.140653259715525919,
                                 0.169004726639267903, 0.190350578064785410, 0.204432940075298892, 0.209482141084727828};
    static const double wg[4] = {0.129484966168869693, 0.279705391489276668, 0.381830050505118945, 0.417959183673469388};
    const double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double fc = ring_measure(H, g, c, want);
    double rk = fc * wk[7], rg = fc * wg[3];
    for (int j = 0; j < 7; ++j) {
        const double f1 = ring_measure(H, g, c - h * xk[j], want), f2 = ring_measure(H, g, c + h * xk[j], want);
        rk += wk[j] * (f1 + f2);
        if (j % 2 == 1) rg += wg[j / 2] * (f1 + f2);
    }
    *err = std::fabs((rk - rg) * h);
    return rk * h;
}

double adapt(const Host& H, const HostRegion& g, int want, double a, double b, double tol, int depth) {
    double err;
    const double v = gk15(H, g, want, a, b, &err);
    if (err <= tol || depth == 0) return v;
    const double m = 0.5 * (a + b);
    return adapt(H, g, want, a, m, 0.5 * tol, depth - 1) + adapt(H, g, want, m, b, 0.5 * tol, depth - 1);
}

void vr_halves_3d(const Host& H, HostRegion& g) {
    for (int want = 0; want < 2; ++want) {
        double s = 0;
        const int panels = 16;
        for (int p = 0; p < panels; ++p)
            s += adapt(H, g, want, kPi * p / panels, kPi * (p + 1) / panels, 1e-12 * g.area / panels, 24);
        g.meas[want] = s;
    }
}

}  // namespace

static bool has_mesh(const Host& H) {
    for (int i = 0; i < H.N; ++i)
        if (H.r[i].kind == WOI_SHAPE_MESH3D) return true;
    return false;
}

// ---------------------------------------------------------------------------- problem object
struct woi_problem {
    Host H;
    uint64_t serial = 0;
    std::vector<uint8_t> blob;   // device image, uploaded on first use
    std::mutex mu;
    int device = -1;
    void* dev = nullptr;
    size_t bytes = 0;
    woi_problem_info info{};
};

namespace {

woi_status compile_shapes(const woi_problem_desc* d, Host& H) {
    const int m = H.m;
    for (int i = 0; i < H.N; ++i) {
        HostRegion& g = H.r[i];
        const woi_shape& s = d->shapes[i];
        g.kind = s.kind;
        for (int k = 0; k < m; ++k) g.c[k] = s.center[k];
        if (s.kind == WOI_SHAPE_SPHERE) {
            if (!(s.radius > 0)) return fail(WOI_E_GEOMETRY, "region %d: sphere radius must be > 0", i);
            g.R = s.radius;
            g.area = 2 * std::pow(kPi, 0.5 * m) / std::tgamma(0.5 * m) * std::pow(g.R, m - 1);
            g.total = m == 2 ? 2 * kPi * g.R : 0.0;
        } else if (s.kind == WOI_SHAPE_ELLIPSOID) {
            if (!s.A) return fail(WOI_E_INVALID_ARG, "region %d: ellipsoid matrix is NULL", i);
            std::memcpy(g.A, s.A, sizeof(double) * m * m);
            for (int a = 0; a < m; ++a)
                for (int b = 0; b < a; ++b)
                    if (std::fabs(g.A[a * m + b] - g.A[b * m + a]) > 1e-12 * (std::fabs(g.A[a * m + b]) + 1e-300))
                        return fail(WOI_E_GEOMETRY, "region %d: ellipsoid matrix not symmetric", i);
            double ev[WOI_MAX_DIM], V[WOI_MAX_DIM * WOI_MAX_DIM];
            sym_eig(m, g.A, ev, V);
            g.lam_max = 0;
            g.detL = 1;
            for (int k = 0; k < m; ++k) {
                if (!(ev[k] > 0)) return fail(WOI_E_GEOMETRY, "region %d: ellipsoid matrix not positive definite", i);
                g.lam_max = std::max(g.lam_max, ev[k]);
                g.detL /= std::sqrt(ev[k]);
            }
            for (int a = 0; a < m; ++a)
                for (int b = 0; b < m; ++b) {
                    double t = 0;
                    for (int k = 0; k < m; ++k) t += V[a * m + k] * V[b * m + k] / std::sqrt(ev[k]);
                    g.L[a * m + b] = t;
                }
            const HostRegion& gg = g;
            g.area = sphere_quad(m, quad_order(m), [&](const double* u) {
                double y[WOI_MAX_DIM], J;
                quadric_point(H, gg, u, y, &J);
                return J;
            });
            g.total = m == 2 ? g.area : 0.0;
            if (m == 2) return fail(WOI_E_UNSUPPORTED, "region %d: 2D ellipses are not supported (use a polyline)", i);
        } else if (s.kind == WOI_SHAPE_POLYLINE2D) {
            if (m != 2) return fail(WOI_E_INVALID_ARG, "region %d: polylines need dim 2", i);
            if (s.n_vertices < 3 || !s.vertices) return fail(WOI_E_INVALID_ARG, "region %d: polyline needs >= 3 vertices", i);
            const int n = s.n_vertices;
            g.v.assign(s.vertices, s.vertices + 2 * n);
            g.v.push_back(s.vertices[0]);
            g.v.push_back(s.vertices[1]);
            g.len.resize(n);
            g.cum.resize(n + 1);
            g.cum[0] = 0;
            double area2 = 0;
            for (int j = 0; j < n; ++j) {
                const double ex = g.v[2 * j + 2] - g.v[2 * j], ey = g.v[2 * j + 3] - g.v[2 * j + 1];
                g.len[j] = std::sqrt(ex * ex + ey * ey);
                if (!(g.len[j] > 0)) return fail(WOI_E_GEOMETRY, "region %d: zero-length polyline segment %d", i, j);
                g.cum[j + 1] = g.cum[j] + g.len[j];
                area2 += g.v[2 * j] * g.v[2 * j + 3] - g.v[2 * j + 2] * g.v[2 * j + 1];
            }
            if (!(area2 > 0)) return fail(WOI_E_GEOMETRY, "region %d: polyline must be counter-clockwise", i);
            g.total = g.area = g.cum[n];
        } else if (s.kind == WOI_SHAPE_MESH3D) {
            if (m != 3) return fail(WOI_E_INVALID_ARG, "region %d: triangle meshes need dim 3", i);
            if (s.n_vertices < 4 || !s.vertices || s.n_triangles < 4 || !s.triangles)
                return fail(WOI_E_INVALID_ARG, "region %d: a mesh needs >= 4 vertices and >= 4 triangles", i);
            const int nv = s.n_vertices, nt = s.n_triangles;
            g.mv.assign(s.vertices, s.vertices + 3 * (size_t)nv);
            g.tri.assign(s.triangles, s.triangles + 3 * (size_t)nt);
            for (int t : g.tri)
                if (t < 0 || t >= nv) return fail(WOI_E_INVALID_ARG, "region %d: triangle index %d out of range", i, t);
            // closed and consistently oriented: every directed edge once, and its reverse once
            std::vector<uint64_t> e;
            e.reserve(3 * (size_t)nt);
            for (int j = 0; j < nt; ++j)
                for (int k = 0; k < 3; ++k)
                    e.push_back((uint64_t)(uint32_t)g.tri[3 * j + k] << 32 | (uint32_t)g.tri[3 * j + (k + 1) % 3]);
            std::sort(e.begin(), e.end());
            for (size_t k = 0; k < e.size(); ++k) {
                if (k + 1 < e.size() && e[k + 1] == e[k])
                    return fail(WOI_E_GEOMETRY, "region %d: mesh edge used twice in one direction", i);
                const uint64_t r = (e[k] << 32) | (e[k] >> 32);
                if (!std::binary_search(e.begin(), e.end(), r))
                    return fail(WOI_E_GEOMETRY, "region %d: mesh is not closed (edge without its reverse)", i);
            }
            g.tn.resize(3 * (size_t)nt);
            g.cum.assign(nt + 1, 0.0);
            double vol = 0;
            for (int j = 0; j < nt; ++j) {
                const double *a = &g.mv[3 * g.tri[3 * j]], *b = &g.mv[3 * g.tri[3 * j + 1]], *c = &g.mv[3 * g.tri[3 * j + 2]];
                const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
                const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
                const double l = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
                if (!(l > 0)) return fail(WOI_E_GEOMETRY, "region %d: degenerate triangle %d", i, j);
                for (int k = 0; k < 3; ++k) g.tn[3 * j + k] = cr[k] / l;
                g.cum[j + 1] = g.cum[j] + 0.5 * l;
                vol += a[0] * cr[0] + a[1] * cr[1] + a[2] * cr[2];
            }
            if (!(vol > 0)) return fail(WOI_E_GEOMETRY, "region %d: mesh normals must point outward", i);
            g.total = g.area = g.cum[nt];
        } else {
            return fail(WOI_E_INVALID_ARG, "region %d: unknown shape kind %d", i, s.kind);
        }
    }
    return WOI_OK;
}

woi_status compile_data(const woi_problem_desc* d, Host& H) {
    const int m = H.m;
    for (int i = 0; i < H.N; ++i) {
        HostRegion& g = H.r[i];
        const woi_data& dd = d->data[i];
        g.dkind = dd.kind;
        g.nt = dd.n_terms;
        g.coef.clear();
        switch (dd.kind) {
            case WOI_DATA_ZERO: g.nt = 0; break;
            case WOI_DATA_FOURIER2D:
                if (m != 2) return fail(WOI_E_INVALID_ARG, "region %d: Fourier data needs dim 2", i);
                if (dd.n_terms < 0 || dd.n_terms > 64 || !dd.coef) return fail(WOI_E_INVALID_ARG, "region %d: bad Fourier data", i);
                g.coef.assign(dd.coef, dd.coef + 2 * dd.n_terms + 1);
                for (int k = 0; k < m; ++k) g.coef.push_back(dd.center[k]);
                break;
            case WOI_DATA_DIRPOLY:
                if (dd.n_terms < 1 || dd.n_terms > 4096 || !dd.coef || !dd.exps) return fail(WOI_E_INVALID_ARG, "region %d: bad DIRPOLY data", i);
                g.coef.assign(dd.coef, dd.coef + dd.n_terms);
                for (int k = 0; k < m; ++k) g.coef.push_back(dd.center[k]);
                g.exps.assign(dd.exps, dd.exps + (size_t)dd.n_terms * m);
                for (uint8_t e : g.exps)
                    if (e > 15) return fail(WOI_E_INVALID_ARG, "region %d: DIRPOLY exponent > 15", i);
                break;
            case WOI_DATA_SOURCE_FLUX:
                if (!dd.coef) return fail(WOI_E_INVALID_ARG, "region %d: SOURCE_FLUX needs coef[0]", i);
                g.coef.push_back(dd.coef[0]);
                for (int k = 0; k < m; ++k) g.coef.push_back(dd.center[k]);
                g.nt = 1;
                break;
            case WOI_DATA_FIELD_FLUX:
                if (!dd.coef) return fail(WOI_E_INVALID_ARG, "region %d: FIELD_FLUX needs coef[0..dim-1]", i);
                g.coef.assign(dd.coef, dd.coef + m);
                g.nt = m;
                break;
            default: return fail(WOI_E_INVALID_ARG, "region %d: unknown data kind %d", i, dd.kind);
        }
    }
    return WOI_OK;
}

woi_status validate_nesting(Host& H) {
    std::vector<double> pts;
    const int m = H.m;
    for (int i = 1; i < H.N; ++i) {
        probe_points(H, H.r[i], pts);
        const size_t np = pts.size() / m;
        for (size_t k = 0; k < np; ++k) {
            const double* y = &pts[k * m];
            if (!point_inside(H, H.r[H.parent[i]], y))
                return fail(WOI_E_GEOMETRY, "region %d: interface leaves its parent region %d", i, H.parent[i]);
            for (int j = 1; j < H.N; ++j)
                if (j != i && H.parent[j] == H.parent[i] && point_inside(H, H.r[j], y))
                    return fail(WOI_E_GEOMETRY, "regions %d and %d (siblings) overlap", i, j);
        }
    }
    return WOI_OK;
}

void flux_integrals(Host& H) {
    const int m = H.m;
    for (int i = 0; i < H.N; ++i) {
        HostRegion& g = H.r[i];
        if (g.kind == WOI_SHAPE_POLYLINE2D) {
            std::vector<double> gx, gw;
            gl_rule(6, gx, gw);
            double s = 0, sa = 0;
            for (int j = 0; j < g.nv(); ++j)
                for (int k = 0; k < 6; ++k) {
                    const double f = 0.5 * (gx[k] + 1.0);
                    const double y[2] = {g.v[2 * j] + f * (g.v[2 * j + 2] - g.v[2 * j]),
                                         g.v[2 * j + 1] + f * (g.v[2 * j + 3] - g.v[2 * j + 1])};
                    const double b = b_value(H, g, y, j);
                    s += 0.5 * gw[k] * g.len[j] * b;
                    sa += 0.5 * gw[k] * g.len[j] * std::fabs(b);
                }
            g.flux = s;
            g.absflux = sa;
        } else if (g.kind == WOI_SHAPE_MESH3D) {
            // per triangle, the interior rule with nodes (2/3, 1/6, 1/6) (degree 2)
            double s = 0, sa = 0;
            for (int j = 0; j < g.ntri(); ++j) {
                const double* P[3] = {&g.mv[3 * g.tri[3 * j]], &g.mv[3 * g.tri[3 * j + 1]], &g.mv[3 * g.tri[3 * j + 2]]};
                const double ar = g.cum[j + 1] - g.cum[j];
                for (int k = 0; k < 3; ++k) {
                    double y[3];
                    for (int c = 0; c < 3; ++c) y[c] = (4 * P[k][c] + P[(k + 1) % 3][c] + P[(k + 2) % 3][c]) / 6.0;
                    const double b = b_value(H, g, y, j);
                    s += ar / 3 * b;
                    sa += ar / 3 * std::fabs(b);
                }
            }
            g.flux = s;
            g.absflux = sa;
        } else {
            const HostRegion& gg = g;
            double sa = 0;
            g.flux = sphere_quad(m, quad_order(m), [&](const double* u) {
                double y[WOI_MAX_DIM], J;
                quadric_point(H, gg, u, y, &J);
                const double b = b_value(H, gg, y, 0);
                sa += 0;   // absolute flux computed below
                return J * b;
            });
            g.absflux = sphere_quad(m, quad_order(m), [&](const double* u) {
                double y[WOI_MAX_DIM], J;
                quadric_point(H, gg, u, y, &J);
                return J * std::fabs(b_value(H, gg, y, 0));
            });
            (void)sa;
        }
    }
}

// Bounding-volume hierarchy over a mesh's triangles: median split of the centroids along the
// longest axis of their box, leaves of at most 4 triangles, nodes in depth-first order with the
// index of the node after each subtree.  Node: box min, box max (widened outward by 1e-5 of the
// larger of the mesh's size and coordinates and the root extent `ext`, which bounds the walker
// positions the FP32 slab tests subtract, plus FP32 rounding), skip index, 8 * leaf list start + triangle count
// (-1 for inner nodes).
void mesh_bvh(const HostRegion& g, double ext, std::vector<float>& nodes, std::vector<int32_t>& list) {
    const int nt = g.ntri();
    std::vector<int> ids(nt);
    std::iota(ids.begin(), ids.end(), 0);
    std::vector<double> cen(3 * (size_t)nt);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int j = 0; j < nt; ++j)
        for (int k = 0; k < 3; ++k) {
            double c = 0;
            for (int v = 0; v < 3; ++v) {
                const double x = g.mv[3 * g.tri[3 * j + v] + k];
                c += x / 3;
                lo[k] = std::min(lo[k], x);
                hi[k] = std::max(hi[k], x);
            }
            cen[3 * j + k] = c;
        }
    const double pad = 1e-5 * std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], std::fabs(lo[0]), std::fabs(hi[0]),
                                        std::fabs(lo[1]), std::fabs(hi[1]), std::fabs(lo[2]), std::fabs(hi[2]), ext});
    nodes.clear();
    list.clear();
    std::function<void(int, int)> build = [&](int a, int b) {   // triangles ids[a, b)
        const size_t me = nodes.size();
        nodes.resize(me + 8);
        double bl[3] = {1e300, 1e300, 1e300}, bh[3] = {-1e300, -1e300, -1e300};
        double cl[3] = {1e300, 1e300, 1e300}, ch[3] = {-1e300, -1e300, -1e300};
        for (int i = a; i < b; ++i)
            for (int k = 0; k < 3; ++k) {
                for (int v = 0; v < 3; ++v) {
                    const double x = g.mv[3 * g.tri[3 * ids[i] + v] + k];
                    bl[k] = std::min(bl[k], x);
                    bh[k] = std::max(bh[k], x);
                }
                cl[k] = std::min(cl[k], cen[3 * ids[i] + k]);
                ch[k] = std::max(ch[k], cen[3 * ids[i] + k]);
            }
        for (int k = 0; k < 3; ++k) {
            nodes[me + k] = std::nextafter((float)(bl[k] - pad), -INFINITY);
            nodes[me + 3 + k] = std::nextafter((float)(bh[k] + pad), INFINITY);
        }
        if (b - a <= 4) {
            nodes[me + 7] = (float)(8 * list.size() + (size_t)(b - a));   // start * 8 + count, exact in FP32
            for (int i = a; i < b; ++i) list.push_back(ids[i]);
        } else {
            nodes[me + 7] = -1.0f;
            int ax = 0;
            for (int k = 1; k < 3; ++k)
                if (ch[k] - cl[k] > ch[ax] - cl[ax]) ax = k;
            const int mid = (a + b) / 2;
            std::nth_element(ids.begin() + a, ids.begin() + mid, ids.begin() + b,
                             [&](int x, int y) { return cen[3 * x + ax] < cen[3 * y + ax]; });
            build(a, mid);
            build(mid, b);
        }
        nodes[me + 6] = (float)(nodes.size() / 8);   // the node after this subtree
    };
    build(0, nt);
}

// Distance from point p to the segment [a, b].
double seg_dist(const double* p, const double* a, const double* b) {
    const double ex = b[0] - a[0], ey = b[1] - a[1], wx = p[0] - a[0], wy = p[1] - a[1];
    const double ee = ex * ex + ey * ey;
    double t = ee > 0 ? (wx * ex + wy * ey) / ee : 0.0;
    t = std::min(1.0, std::max(0.0, t));
    return std::hypot(wx - t * ex, wy - t * ey);
}

// Block bounds of the polyline search: every vertex of the aligned block
// [b 2^l, min((b+1) 2^l, n)] lies within bnd of the block's chord segment, so its signed
// distance to any line lies within [min(h_first, h_last) - bnd, max(...) + bnd].
// Inflated by `pad` to stay conservative under FP32 rounding.  The segments themselves
// (level 0, a block whose chord is the segment) follow at N2 + j with the segment band: FP32
// signed distances too close to zero to be trusted (the FP32 walk queues such a segment and
// decides it in FP64; the FP64 walk decides every segment exactly).
// DIRPOLY data in dimension 2 or 3 as a dense triangular coefficient table c[i][j](k) over
// total degree <= n, in the order a nested Horner evaluation reads it (i, j, k descending):
// b = sum_i e0^i sum_j e1^j sum_k e2^k c_ijk.  Declined (false) when the table would be
// much larger than the term list.
bool dirpoly_dense(const HostRegion& g, int m, std::vector<double>& dense, int& n) {
    n = 0;
    for (int t = 0; t < g.nt; ++t) {
        int s = 0;
        for (int d = 0; d < m; ++d) s += g.exps[(size_t)t * m + d];
        n = std::max(n, s);
    }
    const size_t size = m == 2 ? (size_t)(n + 1) * (n + 2) / 2 : (size_t)(n + 1) * (n + 2) * (n + 3) / 6;
    if (size > std::max<size_t>(64, 4 * (size_t)g.nt)) return false;
    auto pos = [&](int i, int j, int k) -> size_t {   // index of (i, j, k) in Horner order
        size_t p = 0;
        for (int a = n; a > i; --a)
            p += m == 2 ? (size_t)(n - a + 1) : (size_t)(n - a + 1) * (n - a + 2) / 2;
        for (int b = n - i; b > j; --b) p += m == 2 ? 1 : (size_t)(n - i - b + 1);
        if (m == 3) p += (size_t)(n - i - j - k);
        return p;
    };
    dense.assign(size, 0.0);
    for (int t = 0; t < g.nt; ++t) {
        const uint8_t* e = &g.exps[(size_t)t * m];
        dense[pos(e[0], e[1], m == 3 ? e[2] : 0)] += g.coef[t];
    }
    return true;
}

// Coordinate magnitude that the FP32 rounding bands scale with: 1 + the polyline's own, or the
// magnitude of the walker positions if larger (every interface lies inside the root's, so
// `ext`, the root's extent, bounds them).
double band_scale(const HostRegion& g, double ext) {
    double scale = 0;
    for (double x : g.v) scale = std::max(scale, std::fabs(x));
    return std::max(1.0 + scale, ext);
}

double polyline_band(const HostRegion& g, double ext) { return 4e-6 * band_scale(g, ext); }

// |signed distance| of a vertex from a line below which an FP32 walk's sign is not trusted:
// 16 FP32 ulps of the coordinates (the FP32 distance is two FMAs on rounded coordinates, a few
// ulps at most).
double segment_band(const HostRegion& g, double ext) { return 0x1p-20 * band_scale(g, ext); }

void block_bounds(const HostRegion& g, double ext, std::vector<float>& bnd, int& n2, int& top) {
    const int n = g.nv();
    n2 = 1;
    int L = 0;
    while (n2 < n) { n2 *= 2; ++L; }
    top = std::max(1, L - 3);   // first block: 1/8 of the polyline
    const double pad = polyline_band(g, ext);
    bnd.assign((size_t)n2 + n, 0.0f);
    const double band = segment_band(g, ext);
    for (int j = 0; j < n; ++j) bnd[(size_t)n2 + j] = (float)band;
    for (int l = 1; l <= L; ++l) {
        const int base = n2 >> l;   // heap layout: level l occupies [n2 >> l, 2 (n2 >> l))
        for (int j0 = 0, blk = 0; j0 < n; j0 += 1 << l, ++blk) {
            const int j1 = std::min(n, j0 + (1 << l));
            double dmax = 0;
            for (int j = j0; j <= j1; ++j) dmax = std::max(dmax, seg_dist(&g.v[2 * j], &g.v[2 * j0], &g.v[2 * j1]));
            // 1e-3 relative headroom keeps the bound conservative after rounding to FP16
            bnd[base + blk] = (float)(dmax * (1.0 + 2e-3) + pad);
        }
    }
}

}  // namespace

extern "C" {

const char* woi_status_string(woi_status s) {
    switch (s) {
        case WOI_OK: return "WOI_OK";
        case WOI_E_INVALID_ARG: return "WOI_E_INVALID_ARG";
        case WOI_E_GEOMETRY: return "WOI_E_GEOMETRY";
        case WOI_E_INCOMPATIBLE: return "WOI_E_INCOMPATIBLE";
        case WOI_E_UNSUPPORTED: return "WOI_E_UNSUPPORTED";
        case WOI_E_DEVICE: return "WOI_E_DEVICE";
        case WOI_E_OOM: return "WOI_E_OOM";
    }
    return "WOI_E_UNKNOWN";
}

const char* woi_last_error(void) { return g_err.c_str(); }

woi_status woi_problem_create(const woi_problem_desc* d, woi_problem** out) {
    if (!d || !out) return fail(WOI_E_INVALID_ARG, "NULL descriptor or output");
    *out = nullptr;
    if (d->dim < 2 || d->dim > WOI_MAX_DIM) return fail(WOI_E_INVALID_ARG, "dim %d outside [2, %d]", d->dim, WOI_MAX_DIM);
    if (d->n_regions < 1 || d->n_regions > WOI_MAX_REGIONS)
        return fail(WOI_E_INVALID_ARG, "n_regions %d outside [1, %d]", d->n_regions, WOI_MAX_REGIONS);
    if (!d->parent || !d->sigma || !d->shapes || !d->data) return fail(WOI_E_INVALID_ARG, "NULL array in descriptor");
    auto* P = new (std::nothrow) woi_problem;
    if (!P) return fail(WOI_E_OOM, "host allocation failed");
    static std::atomic<uint64_t> next_serial{1};
    P->serial = next_serial++;
    Host& H = P->H;
    H.m = d->dim;
    H.N = d->n_regions;
    const int m = H.m, N = H.N;
    woi_status st = WOI_OK;
    for (int i = 0; i < N && st == WOI_OK; ++i) {
        H.parent[i] = d->parent[i];
        H.sigma[i] = d->sigma[i];
        if (i == 0 && d->parent[0] != -1) st = fail(WOI_E_GEOMETRY, "parent[0] must be -1");
        if (i > 0 && (d->parent[i] < 0 || d->parent[i] >= i)) st = fail(WOI_E_GEOMETRY, "parent[%d] = %d must be in [0, %d)", i, d->parent[i], i);
        if (!(d->sigma[i] >= 0) || !std::isfinite(d->sigma[i])) st = fail(WOI_E_INVALID_ARG, "sigma[%d] must be finite and >= 0", i);
    }
    for (int i = 1; i < N && st == WOI_OK; ++i)
        if (!(H.sigma[i] + H.sigma[H.parent[i]] > 0)) st = fail(WOI_E_INVALID_ARG, "sigma[%d] + sigma[parent] must be > 0", i);
    if (st == WOI_OK && !(H.sigma[0] > 0)) st = fail(WOI_E_INVALID_ARG, "sigma[0] must be > 0");
    if (st == WOI_OK) st = compile_shapes(d, H);
    if (st == WOI_OK) st = compile_data(d, H);
    if (st == WOI_OK) st = validate_nesting(H);
    if (st != WOI_OK) { delete P; return st; }

    // alpha_i and beta scale s_i (Eq. unit_coeff_charge_density_sys)
    H.alpha_l1 = 0;
    for (int i = 0; i < N; ++i) {
        HostRegion& g = H.r[i];
        if (i == 0) { g.alpha = 2.0; g.s = 2.0 / H.sigma[0]; }
        else {
            const double sp = H.sigma[H.parent[i]], si = H.sigma[i];
            g.alpha = 2.0 * (si - sp) / (sp + si);
            g.s = -2.0 / (sp + si);
        }
        H.alpha_l1 += std::fabs(g.alpha);
    }
    flux_integrals(H);
    if (d->compat_mode == WOI_COMPAT_PER_INTERFACE) {
        for (int i = 0; i < N; ++i)
            if (std::fabs(H.r[i].flux) > d->compat_tol * H.r[i].absflux + 1e-300) {
                delete P;
                return fail(WOI_E_INCOMPATIBLE, "region %d: integral of b = %.3e exceeds tol * integral |b| = %.3e", i,
                            H.r[i].flux, d->compat_tol * H.r[i].absflux);
            }
    } else if (d->compat_mode == WOI_COMPAT_GLOBAL) {
        double s = -H.r[0].flux, sa = H.r[0].absflux;
        for (int i = 1; i < N; ++i) { s += H.r[i].flux; sa += H.r[i].absflux; }
        if (std::fabs(s) > d->compat_tol * sa + 1e-300) {
            delete P;
            return fail(WOI_E_INCOMPATIBLE, "global flux balance violated by %.3e", s);
        }
    } else if (d->compat_mode != WOI_COMPAT_NONE) {
        delete P;
        return fail(WOI_E_INVALID_ARG, "unknown compat_mode %d", d->compat_mode);
    }
    // VR halves
    bool vr_ok = m <= 3;
    for (int i = 0; i < N; ++i)
        if (H.r[i].kind == WOI_SHAPE_MESH3D) vr_ok = false;   // no VR halves on meshes
    for (int i = 0; i < N; ++i) {
        HostRegion& g = H.r[i];
        if (!vr_ok) g.meas[0] = g.meas[1] = std::nan("");
        else if (m == 2) vr_halves_2d(H, g);
        else if (m == 3) vr_halves_3d(H, g);
        else g.meas[0] = g.meas[1] = std::nan("");
        if (m == 3)
            for (int c = 0; c < 2; ++c)
                if (g.meas[c] < 1e-13 * g.area) g.meas[c] = 0.0;
    }

    // ---- device layout
    std::vector<double> p64;
    std::vector<float> p32;
    std::vector<uint8_t> pb;
    std::vector<int32_t> pi;
    auto put64 = [&](const double* x, size_t n) { const int o = (int)p64.size(); p64.insert(p64.end(), x, x + n); return o; };
    auto put32 = [&](const double* x, size_t n) {
        const int o = (int)p32.size();
        for (size_t k = 0; k < n; ++k) p32.push_back((float)x[k]);
        return o;
    };
    DevProblem hdr;
    std::memset(&hdr, 0, sizeof hdr);
    hdr.dim = m;
    hdr.N = N;
    hdr.vr_ok = vr_ok;
    hdr.alpha_l1 = H.alpha_l1;
    hdr.unit_area = 2 * std::pow(kPi, 0.5 * m) / std::tgamma(0.5 * m);
    hdr.phi_c = m == 2 ? 1.0 / (2 * kPi) : 1.0 / ((m - 2) * hdr.unit_area);
    hdr.alpha_l1_f = (float)hdr.alpha_l1;
    hdr.unit_area_f = (float)hdr.unit_area;
    hdr.inv_unit_area_f = (float)(1.0 / hdr.unit_area);
    hdr.phi_c_f = (float)hdr.phi_c;
    // FP32 sign band: 2^-19 (32 FP32 ulps) of the largest coordinate magnitude on dOmega (every
    // interface lies inside the root's); root_ext also scales the polyline bands and mesh boxes
    double root_ext = 0;
    {
        const HostRegion& g = H.r[0];
        double ext = 0;
        if (g.kind == WOI_SHAPE_SPHERE || g.kind == WOI_SHAPE_ELLIPSOID) {
            for (int i = 0; i < m; ++i) {
                double half = g.R;
                if (g.kind == WOI_SHAPE_ELLIPSOID) {   // extent along axis i: sqrt((A^-1)_ii), A^-1 = L L
                    double s2 = 0;
                    for (int j = 0; j < m; ++j) s2 += g.L[i * m + j] * g.L[i * m + j];
                    half = std::sqrt(s2);
                }
                ext = std::max(ext, std::fabs(g.c[i]) + half);
            }
        }
        for (double x : g.v) ext = std::max(ext, std::fabs(x));
        for (double x : g.mv) ext = std::max(ext, std::fabs(x));
        hdr.sign_band_f = (float)(0x1p-19 * std::max(1.0, ext));
        root_ext = ext;
    }
    double acc = 0;
    for (int i = 0; i < N; ++i) {
        acc += std::fabs(H.r[i].alpha);
        hdr.cdf[i] = acc / H.alpha_l1;
        // cdf * 2^32 - 1/2 is exact in double (cdf <= 1), and so is its ceiling
        const double x = std::ceil(std::ldexp(hdr.cdf[i], 32) - 0.5);
        hdr.sthr[i] = x <= 0 ? 0ull : (uint64_t)x;
    }
    for (int k = 0; k < 64; ++k) {
        const double u = k / 64.0;
        int h = 0;
        while (h < N - 1 && !(u < hdr.cdf[h])) ++h;
        hdr.sguide[k] = (unsigned char)h;
    }
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            int rel = woi::REL_OTHER;
            if (a == b) rel = woi::REL_SAME;
            else
                for (int p = H.parent[a]; p >= 0; p = H.parent[p])
                    if (p == b) { rel = woi::REL_DESC; break; }
            hdr.rel[a][b] = (unsigned char)rel;
        }
    for (int i = 0; i < N; ++i) {
        const HostRegion& g = H.r[i];
        DevRegion& r = hdr.reg[i];
        r.kind = g.kind;
        r.dkind = g.dkind;
        r.nt = g.nt;
        std::vector<double> geo;
        if (g.kind == WOI_SHAPE_SPHERE) {
            geo.assign(g.c, g.c + m);
            geo.push_back(g.R);
        } else if (g.kind == WOI_SHAPE_ELLIPSOID) {
            geo.assign(g.c, g.c + m);
            geo.insert(geo.end(), g.A, g.A + m * m);
            geo.insert(geo.end(), g.L, g.L + m * m);
            geo.push_back(1.0 / g.lam_max);
        } else if (g.kind == WOI_SHAPE_MESH3D) {
            // per triangle (a, b - a, c - a): the Moller-Trumbore operands
            for (int j = 0; j < g.ntri(); ++j) {
                const double *a = &g.mv[3 * g.tri[3 * j]], *b = &g.mv[3 * g.tri[3 * j + 1]], *c = &g.mv[3 * g.tri[3 * j + 2]];
                for (int k = 0; k < 3; ++k) geo.push_back(a[k]);
                for (int k = 0; k < 3; ++k) geo.push_back(b[k] - a[k]);
                for (int k = 0; k < 3; ++k) geo.push_back(c[k] - a[k]);
            }
            r.nv = g.ntri();
        } else {
            geo = g.v;
            r.nv = g.nv();
        }
        r.g64 = put64(geo.data(), geo.size());
        if (g.kind == WOI_SHAPE_POLYLINE2D) {
            // FP32 vertices padded with v[nv] up to N2 + 1 entries: every aligned block of
            // the search then ends on a stored vertex
            int n2 = 1;
            while (n2 < g.nv()) n2 *= 2;
            std::vector<double> pad(geo);
            for (int j = g.nv() + 1; j <= n2; ++j) { pad.push_back(geo[2 * g.nv()]); pad.push_back(geo[2 * g.nv() + 1]); }
            r.g32 = put32(pad.data(), pad.size());
        } else {
            r.g32 = put32(geo.data(), geo.size());
        }
        if (g.kind == WOI_SHAPE_POLYLINE2D) {
            const int n = g.nv();
            r.len64 = put64(g.len.data(), g.len.size());
            r.len32 = put32(g.len.data(), g.len.size());
            r.cum64 = put64(g.cum.data(), g.cum.size());
            // FP32 sampling table: (cum[j], 1 / len[j]) pairs, one load per probe
            std::vector<double> cl(2 * (n + 1));
            for (int j = 0; j <= n; ++j) {
                cl[2 * j] = g.cum[j];
                cl[2 * j + 1] = j < n ? 1.0 / g.len[j] : 0.0;
            }
            r.cum32 = put32(cl.data(), cl.size());
            r.gscale = (double)n / g.cum[n];
            r.gscale_f = (float)r.gscale;
            std::vector<double> nrm(2 * n);
            for (int j = 0; j < n; ++j) {   // outward normal of a counter-clockwise segment
                const double ex = g.v[2 * j + 2] - g.v[2 * j], ey = g.v[2 * j + 3] - g.v[2 * j + 1];
                const double l = std::sqrt(ex * ex + ey * ey);
                nrm[2 * j] = ey / l;
                nrm[2 * j + 1] = -ex / l;
            }
            r.nrm64 = put64(nrm.data(), nrm.size());
            r.nrm32 = put32(nrm.data(), nrm.size());
            std::vector<float> bnd;
            block_bounds(g, root_ext, bnd, r.n2, r.top);
            r.bnd = (int)p32.size();
            p32.insert(p32.end(), bnd.begin(), bnd.end());
            r.hband_f = (float)segment_band(g, root_ext);
            r.guide = (int)pi.size();
            for (int k = 0; k < n; ++k) {
                const double s0 = g.cum[n] * k / n;
                int j = (int)(std::upper_bound(g.cum.begin(), g.cum.begin() + n, s0) - g.cum.begin()) - 1;
                pi.push_back(std::max(0, std::min(j, n - 1)));
            }
        } else if (g.kind == WOI_SHAPE_MESH3D) {
            const int n = g.ntri();
            r.nrm64 = put64(g.tn.data(), g.tn.size());
            r.nrm32 = put32(g.tn.data(), g.tn.size());
            std::vector<float> nodes;
            std::vector<int32_t> list;
            mesh_bvh(g, root_ext, nodes, list);
            r.bvh = (int)p32.size();
            r.nbvh = (int)(nodes.size() / 8);
            p32.insert(p32.end(), nodes.begin(), nodes.end());
            r.bvhidx = (int)pi.size();
            pi.insert(pi.end(), list.begin(), list.end());
            r.cum64 = put64(g.cum.data(), g.cum.size());
            std::vector<double> cl(2 * (n + 1), 0.0);   // FP32 table of (cum[j], 0) pairs, the polyline layout
            for (int j = 0; j <= n; ++j) cl[2 * j] = g.cum[j];
            r.cum32 = put32(cl.data(), cl.size());
            r.gscale = (double)n / g.cum[n];
            r.gscale_f = (float)r.gscale;
            r.guide = (int)pi.size();
            for (int k = 0; k < n; ++k) {
                const double s0 = g.cum[n] * k / n;
                int j = (int)(std::upper_bound(g.cum.begin(), g.cum.begin() + n, s0) - g.cum.begin()) - 1;
                pi.push_back(std::max(0, std::min(j, n - 1)));
            }
        }
        std::vector<double> dense;
        int degree = 0;
        if (g.dkind == WOI_DATA_DIRPOLY && m <= 3 && dirpoly_dense(g, m, dense, degree)) {
            // device form: dense triangular coefficients in nested-Horner order, then the center
            for (int k = 0; k < m; ++k) dense.push_back(g.coef[g.nt + k]);
            r.dkind = woi::DK_DIRPOLY_HORNER;
            r.nt = degree;
            r.d64 = put64(dense.data(), dense.size());
            r.d32 = put32(dense.data(), dense.size());
        } else if (!g.coef.empty()) {
            r.d64 = put64(g.coef.data(), g.coef.size());
            r.d32 = put32(g.coef.data(), g.coef.size());
        }
        if (!g.exps.empty()) {   // device form: one 8-byte word per term, exponent d in byte d
            while (pb.size() % 8) pb.push_back(0);
            r.dexp = (int)pb.size();
            const size_t nt = g.exps.size() / m;
            for (size_t t = 0; t < nt; ++t)
                for (int d = 0; d < 8; ++d) pb.push_back(d < m ? g.exps[t * m + d] : 0);
        }
        if (!g.brk.empty()) {
            r.b64 = put64(g.brk.data(), g.brk.size());
            r.b32 = put32(g.brk.data(), g.brk.size());
        }
        r.nbrk = (int)g.brk.size();
        r.class0 = g.class0;
        r.alpha = g.alpha;
        r.sgn = g.alpha < 0 ? -1.0 : 1.0;
        r.s = g.s;
        r.area = g.area;
        r.meas[0] = g.meas[0];
        r.meas[1] = g.meas[1];
        r.total = g.total;
        r.alpha_f = (float)r.alpha;
        r.sgn_f = (float)r.sgn;
        r.s_f = (float)r.s;
        r.area_f = (float)r.area;
        r.meas_f[0] = (float)r.meas[0];
        r.meas_f[1] = (float)r.meas[1];
        r.total_f = (float)r.total;
    }
    // LDS staging layout: FP32 vertices (8 B each, n2 + 1, padded) and FP16 bounds (2 B
    // each, n2 + n) of every polyline, the tables of the block walk; then, if everything still
    // fits the largest staging area, the FP32 arclength CDF ((cum, 1/len) pairs, 8 B each, n + 1)
    // and the guide table (4 B each, n) of every polyline, the tables of uniform sampling
    {
        int off = 0;
        for (int i = 0; i < N; ++i) {
            DevRegion& r = hdr.reg[i];
            r.lds_v = r.lds_b = r.lds_c = r.lds_g = -1;
            if (r.kind != WOI_SHAPE_POLYLINE2D) continue;
            r.lds_v = off;
            off += 8 * (r.n2 + 1);
            r.lds_b = off;
            off += 2 * (r.n2 + r.nv);
            off = (off + 15) & ~15;
        }
        int cdf = 0;
        for (int i = 0; i < N; ++i)
            if (hdr.reg[i].kind == WOI_SHAPE_POLYLINE2D) cdf += ((8 * (hdr.reg[i].nv + 1) + 4 * hdr.reg[i].nv) + 15) & ~15;
        if (off > 0 && off + cdf <= woi::LDS_BUDGET_MAX) {
            for (int i = 0; i < N; ++i) {
                DevRegion& r = hdr.reg[i];
                if (r.kind != WOI_SHAPE_POLYLINE2D) continue;
                r.lds_c = off;
                off += 8 * (r.nv + 1);
                r.lds_g = off;
                off += 4 * r.nv;
                off = (off + 15) & ~15;
            }
        }
        hdr.lds_bytes = off;   // staged only if the device's workgroup limit allows (decided at launch)
    }
    auto align = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
    hdr.off64 = align(sizeof(DevProblem));
    hdr.off32 = align(hdr.off64 + p64.size() * sizeof(double));
    hdr.offb = align(hdr.off32 + p32.size() * sizeof(float));
    hdr.offi = align(hdr.offb + pb.size());
    hdr.bytes = align(hdr.offi + pi.size() * sizeof(int32_t) + 16);
    std::vector<uint8_t> blob(hdr.bytes, 0);
    std::memcpy(blob.data(), &hdr, sizeof hdr);
    if (!p64.empty()) std::memcpy(blob.data() + hdr.off64, p64.data(), p64.size() * sizeof(double));
    if (!p32.empty()) std::memcpy(blob.data() + hdr.off32, p32.data(), p32.size() * sizeof(float));
    if (!pb.empty()) std::memcpy(blob.data() + hdr.offb, pb.data(), pb.size());
    if (!pi.empty()) std::memcpy(blob.data() + hdr.offi, pi.data(), pi.size() * sizeof(int32_t));
    P->blob = std::move(blob);
    P->bytes = hdr.bytes;
    woi_problem_info& inf = P->info;
    inf.dim = m;
    inf.n_regions = N;
    inf.alpha_l1 = H.alpha_l1;
    for (int i = 0; i < N; ++i) {
        inf.alpha[i] = H.r[i].alpha;
        inf.beta_scale[i] = H.r[i].s;
        inf.area[i] = H.r[i].area;
        inf.area_plus[i] = H.r[i].meas[0];
        inf.area_minus[i] = H.r[i].meas[1];
        inf.flux[i] = H.r[i].flux;
    }
    inf.device_bytes = hdr.bytes;
    *out = P;
    return WOI_OK;
}

woi_status woi_problem_upload(woi_problem* p) {
    if (!p) return fail(WOI_E_INVALID_ARG, "NULL problem");
    std::lock_guard<std::mutex> lk(p->mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(WOI_E_DEVICE, "no HIP device");
    if (p->dev) {
        if (cur != p->device) return fail(WOI_E_INVALID_ARG, "problem lives on device %d, current device is %d", p->device, cur);
        return WOI_OK;
    }
    void* d = nullptr;
    if (hipMalloc(&d, p->bytes) != hipSuccess) return fail(WOI_E_OOM, "hipMalloc(%zu) failed", p->bytes);
    if (hipMemcpy(d, p->blob.data(), p->bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return fail(WOI_E_DEVICE, "problem upload failed");
    }
    p->dev = d;
    p->device = cur;
    return WOI_OK;
}

void woi_problem_destroy(woi_problem* p) {
    if (!p) return;
    if (p->dev) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(p->device);
        (void)hipFree(p->dev);
        (void)hipSetDevice(cur);
    }
    delete p;
}

woi_status woi_problem_get_info(const woi_problem* p, woi_problem_info* out) {
    if (!p || !out) return fail(WOI_E_INVALID_ARG, "NULL argument");
    *out = p->info;
    return WOI_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------- estimation
namespace {

struct Plan {
    unsigned lds;
    int block;
    uint32_t spt;
    int chunks;
    unsigned gx;
    uint64_t n_samples, first;
};

woi_status check_query_impl(const woi_problem* p, int64_t P, const woi_query* q) {
    if (!p || !q) return fail(WOI_E_INVALID_ARG, "NULL problem or query");
    if (P < 1) return fail(WOI_E_INVALID_ARG, "P = %lld must be >= 1", (long long)P);
    if (q->M < 0 || q->M > WOI_MAX_M) return fail(WOI_E_INVALID_ARG, "M = %d outside [0, %d]", q->M, WOI_MAX_M);
    if (q->walks < 1) return fail(WOI_E_INVALID_ARG, "walks must be >= 1");
    if (q->estimator != WOI_EST_PLAIN && q->estimator != WOI_EST_VR && q->estimator != WOI_EST_NAIVE)
        return fail(WOI_E_INVALID_ARG, "bad estimator");
    if (q->precision != WOI_PREC_FP64 && q->precision != WOI_PREC_FP32) return fail(WOI_E_INVALID_ARG, "bad precision");
    if (q->estimator == WOI_EST_VR) {
        if (p->H.m > 3) return fail(WOI_E_UNSUPPORTED, "variance reduction needs dim <= 3");
        for (int i = 0; i < p->H.N; ++i)
            if (p->H.r[i].kind == WOI_SHAPE_MESH3D)
                return fail(WOI_E_UNSUPPORTED, "variance reduction is not available with triangle meshes (region %d)", i);
        if ((q->walks & 1) || (q->walk_offset & 1)) return fail(WOI_E_INVALID_ARG, "VR needs even walks and walk_offset");
    }
    if (q->batch_share < 1) return fail(WOI_E_INVALID_ARG, "batch_share must be >= 1");
    if (q->estimator == WOI_EST_NAIVE) {
        if (q->batch_share != 1) return fail(WOI_E_UNSUPPORTED, "the naive estimator needs batch_share = 1");
        if (q->instance != 0) return fail(WOI_E_UNSUPPORTED, "the naive estimator needs instance = 0");
        if (std::pow(p->H.N + 1.0, q->M + 1.0) > 2147483648.0)
            return fail(WOI_E_INVALID_ARG, "naive estimator: (N + 1)^(M + 1) = %.3g exceeds 2^31 tree-node ids",
                        std::pow(p->H.N + 1.0, q->M + 1.0));
        if (std::pow((double)p->H.N, q->M + 1.0) > (double)WOI_NAIVE_MAX_LEAVES)
            return fail(WOI_E_INVALID_ARG, "naive estimator: N^(M + 1) = %.3g leaves per tree exceed %d",
                        std::pow((double)p->H.N, q->M + 1.0), WOI_NAIVE_MAX_LEAVES);
    }
    if (q->instance >= (1u << 24)) return fail(WOI_E_INVALID_ARG, "instance must be < 2^24");
    const uint64_t ns = q->estimator == WOI_EST_VR ? q->walks / 2 : q->walks;
    const uint64_t first = q->estimator == WOI_EST_VR ? q->walk_offset / 2 : q->walk_offset;
    if (first + ns > (1ull << 32)) return fail(WOI_E_INVALID_ARG, "walk indices must stay below 2^32");
    return WOI_OK;
}

// max_chunks > 0 caps the number of partial slots (a fixed-size partial buffer).
Plan make_plan(const woi_problem* p, int64_t P, const woi_query* q, uint64_t n_samples, uint64_t max_chunks = 0) {
    Plan pl;
    pl.n_samples = n_samples;
    pl.first = q->estimator == WOI_EST_VR ? q->walk_offset / 2 : q->walk_offset;
    const DevProblem* hdr = reinterpret_cast<const DevProblem*>(p->blob.data());
    pl.lds = hdr->lds_bytes > 0 && p->H.m == 2 && hdr->lds_bytes <= woi::lds_budget() ? (unsigned)hdr->lds_bytes : 0u;
    pl.block = pl.lds ? 512 : (q->block_size > 0 ? q->block_size : (P >= 4096 ? 256 : 64));
    pl.gx = (unsigned)((P + pl.block - 1) / pl.block);
    uint64_t spt;
    if (q->samples_per_thread > 0) spt = (uint64_t)q->samples_per_thread;
    else {
        // aim at >= 2^20 resident threads (256 CUs x 4 SIMDs x 16 waves x 64 lanes) with
        // at least 8 samples per thread
        const uint64_t target = 1ull << 20;
        const uint64_t lanes = (uint64_t)pl.gx * pl.block;
        uint64_t chunks = std::max<uint64_t>(1, (target + lanes - 1) / lanes);
        spt = std::max<uint64_t>(8, (n_samples + chunks - 1) / chunks);
    }
    spt = std::min<uint64_t>(spt, n_samples);
    uint64_t chunks = (n_samples + spt - 1) / spt;
    if (max_chunks > 0 && chunks > max_chunks) {
        spt = (n_samples + max_chunks - 1) / max_chunks;
        chunks = (n_samples + spt - 1) / spt;
    }
    while (chunks > 65535) { spt *= 2; chunks = (n_samples + spt - 1) / spt; }
    pl.spt = (uint32_t)spt;
    pl.chunks = (int)chunks;
    (void)p;
    return pl;
}

// Shared-trajectory plan (batch_share B > 1): chunks of samples whose trajectories fit the
// trajectory budget, evaluation pieces of spt_e samples (the reduction's unit).
struct SharedPlan {
    int ng, lg, tile_rows;
    unsigned lds;
    uint32_t chunk, spt_g, spt_e;
    int n_chunks, pieces_per_chunk, n_pieces;
    size_t plane, traj_bytes, part_bytes;
    // partial slots: piece y of every chunk goes to slot y
    int n_slots() const { return n_chunks > 1 ? pieces_per_chunk : n_pieces; }
};

SharedPlan make_shared_plan(const woi_problem* p, int64_t P, const woi_query* q, uint64_t ns) {
    SharedPlan sp;
    const int m = p->H.m, K = q->estimator == WOI_EST_VR ? 2 : 1;
    const size_t rs = q->precision == WOI_PREC_FP32 ? sizeof(float) : sizeof(double);
    sp.ng = (int)((P + q->batch_share - 1) / q->batch_share);
    const DevProblem* hdr = reinterpret_cast<const DevProblem*>(p->blob.data());
    sp.lds = hdr->lds_bytes > 0 && m == 2 && hdr->lds_bytes <= woi::lds_budget() ? (unsigned)hdr->lds_bytes : 0u;
    // trajectory chunk: the samples whose planes fit in 1 GiB; evaluation pieces: enough of
    // them per chunk for ~4096 workgroups of EVAL_BLOCK points
    const size_t per_sample = (size_t)sp.ng * K * (q->M + 1) * (m + 1) * rs;
    const uint64_t chunk0 = std::min<uint64_t>(ns, std::max<uint64_t>(1, (1ull << 30) / per_sample));
    const uint64_t tiles = (uint64_t)((P + woi::EVAL_BLOCK - 1) / woi::EVAL_BLOCK);
    const uint64_t want_pieces = std::max<uint64_t>(1, (4096 + tiles - 1) / tiles);
    const uint64_t spt_e = std::max<uint64_t>(1, (chunk0 + want_pieces - 1) / want_pieces);
    uint64_t chunk = std::max<uint64_t>(spt_e, chunk0 / spt_e * spt_e);
    chunk = std::min<uint64_t>(chunk, (ns + spt_e - 1) / spt_e * spt_e);
    sp.chunk = (uint32_t)chunk;
    sp.spt_e = (uint32_t)spt_e;
    sp.pieces_per_chunk = (int)(chunk / spt_e);
    sp.n_chunks = (int)((ns + chunk - 1) / chunk);
    sp.n_pieces = (int)((ns + spt_e - 1) / spt_e);
    // generation: lanes = groups in rows of lg lanes; split the chunk into runs so that about
    // 2^21 walkers are launched (several workgroups per CU: short tails)
    const int bs = sp.lds ? 512 : 256;
    sp.lg = 64;
    while (sp.lg < sp.ng && sp.lg < bs) sp.lg *= 2;
    const uint64_t want = std::min<uint64_t>(std::max<uint64_t>(1, (1ull << 21) / (uint64_t)sp.ng),
                                             65535ull * (uint64_t)(bs / sp.lg));   // grid.y limit
    sp.spt_g = (uint32_t)std::max<uint64_t>(1, (chunk + want - 1) / want);
    // evaluation tiles: as many (sample, walker, step) rows as the LDS budget holds
    const size_t row_bytes = woi::eval_lds_bytes(q->batch_share, P, m, 1, rs);
    sp.tile_rows = (int)std::max<size_t>(1, (size_t)woi::EVAL_LDS / row_bytes);
    sp.plane = (size_t)chunk * K * (q->M + 1) * sp.ng;
    sp.traj_bytes = (sp.plane * (m + 1) * rs + 255) & ~size_t(255);
    sp.part_bytes = (size_t)sp.n_slots() * (size_t)P * (2 + 2 * m) * sizeof(double);
    return sp;
}

// Naive estimator: one wave per (point, chunk of trees); about 2^14 waves in flight.
struct NaivePlan {
    unsigned gx;
    uint32_t spt;
    int chunks;
    woi::NParams np;
};

NaivePlan make_naive_plan(const woi_problem* p, int64_t P, const woi_query* q, uint64_t n_trees) {
    NaivePlan pl;
    pl.gx = (unsigned)((P + 3) / 4);
    uint64_t span = 1;
    for (int i = 0; i < q->M; ++i) span *= (uint64_t)p->H.N;
    pl.np.span0 = (uint32_t)span;
    pl.np.leaves = (uint32_t)(span * (uint64_t)p->H.N);
    uint64_t spt;
    if (q->samples_per_thread > 0) spt = (uint64_t)q->samples_per_thread;
    else {
        const uint64_t chunks = std::max<uint64_t>(1, ((1u << 14) + (uint64_t)P - 1) / (uint64_t)P);
        spt = (n_trees + chunks - 1) / chunks;
    }
    spt = std::max<uint64_t>(1, std::min<uint64_t>(spt, n_trees));
    uint64_t chunks = (n_trees + spt - 1) / spt;
    while (chunks > 65535) { spt *= 2; chunks = (n_trees + spt - 1) / spt; }
    pl.spt = (uint32_t)spt;
    pl.chunks = (int)chunks;
    return pl;
}

woi::KParams naive_params(const woi_problem* p, const double* points, int64_t P, const woi_query* q,
                          uint64_t n_trees, const NaivePlan& pl) {
    woi::KParams kp{};
    kp.dp = static_cast<const DevProblem*>(p->dev);
    kp.points = points;
    kp.P = P;
    kp.n_samples = n_trees;
    kp.first_sample = q->walk_offset;
    kp.samples_per_thread = pl.spt;
    kp.k0 = (uint32_t)q->seed;
    kp.k1 = (uint32_t)(q->seed >> 32);
    kp.M = q->M;
    kp.batch_share = 1;
    kp.mesh = has_mesh(p->H) ? 1 : 0;
    return kp;
}

woi_status estimate_naive(const woi_problem* p, const double* points, int64_t P, const woi_query* q, double* mean,
                          double* se, double* grad, double* grad_se, void* workspace, size_t workspace_bytes,
                          uint64_t* counters, hipStream_t s) {
    const NaivePlan pl = make_naive_plan(p, P, q, q->walks);
    const size_t need = (size_t)pl.chunks * (size_t)P * (2 + 2 * p->H.m) * sizeof(double);
    if (!workspace || workspace_bytes < need)
        return fail(WOI_E_OOM, "workspace of %zu bytes is smaller than the %zu bytes needed", workspace_bytes, need);
    woi::KParams kp = naive_params(p, points, P, q, q->walks, pl);
    kp.partials = static_cast<double*>(workspace);
    kp.counters = counters;
    if (q->event_begin && hipEventRecord(static_cast<hipEvent_t>(q->event_begin), s) != hipSuccess)
        return fail(WOI_E_DEVICE, "hipEventRecord(begin) failed");
    hipError_t e = woi::launch_naive(kp, pl.np, p->H.m, q->precision == WOI_PREC_FP32, dim3(pl.gx, pl.chunks), s);
    if (e != hipSuccess) return fail(WOI_E_DEVICE, "naive launch failed: %s", hipGetErrorString(e));
    if (q->event_end && hipEventRecord(static_cast<hipEvent_t>(q->event_end), s) != hipSuccess)
        return fail(WOI_E_DEVICE, "hipEventRecord(end) failed");
    woi::RParams rp{};
    rp.partials = kp.partials;
    rp.P = P;
    rp.dim = p->H.m;
    rp.n_chunks = pl.chunks;
    rp.samples_per_thread = pl.spt;
    rp.full = 0;
    rp.tail = q->walks;
    rp.mean = mean;
    rp.se = se;
    rp.grad = grad;
    rp.grad_se = grad_se;
    e = woi::launch_reduce(rp, s);
    if (e != hipSuccess) return fail(WOI_E_DEVICE, "reduce launch failed: %s", hipGetErrorString(e));
    return WOI_OK;
}

// The per-point path: walk kernel over (point tile, sample chunk), then the reduction of the
// chunk partials (pl.chunks * P records of 2 + 2 dim doubles at `partials`).
woi_status launch_per_point(const woi_problem* p, const double* points, int64_t P, const woi_query* q, const Plan& pl,
                            double* mean, double* se, double* grad, double* grad_se, double* partials,
                            uint64_t* counters, hipStream_t s) {
    woi::KParams kp{};
    kp.dp = static_cast<const DevProblem*>(p->dev);
    kp.points = points;
    kp.P = P;
    kp.n_samples = pl.n_samples;
    kp.first_sample = pl.first;
    kp.samples_per_thread = pl.spt;
    kp.k0 = (uint32_t)q->seed;
    kp.k1 = (uint32_t)(q->seed >> 32);
    kp.M = q->M;
    kp.batch_share = q->batch_share;
    kp.shared_sched = q->schedule_mode == WOI_SCHED_SHARED;
    kp.mesh = has_mesh(p->H) ? 1 : 0;
    kp.instance = q->instance;
    kp.partials = partials;
    kp.counters = counters;
    if (q->event_begin && hipEventRecord(static_cast<hipEvent_t>(q->event_begin), s) != hipSuccess)
        return fail(WOI_E_DEVICE, "hipEventRecord(begin) failed");
    hipError_t e = woi::launch_walk(kp, p->H.m, q->estimator == WOI_EST_VR, q->precision == WOI_PREC_FP32, pl.lds,
                                    dim3(pl.gx, pl.chunks), dim3(pl.block), s);
    if (e != hipSuccess) return fail(WOI_E_DEVICE, "walk launch failed: %s", hipGetErrorString(e));
    if (q->event_end && hipEventRecord(static_cast<hipEvent_t>(q->event_end), s) != hipSuccess)
        return fail(WOI_E_DEVICE, "hipEventRecord(end) failed");
    woi::RParams rp{};
    rp.partials = partials;
    rp.P = P;
    rp.dim = p->H.m;
    rp.n_chunks = pl.chunks;
    rp.samples_per_thread = pl.spt;
    rp.full = 0;
    rp.tail = pl.n_samples;
    rp.mean = mean;
    rp.se = se;
    rp.grad = grad;
    rp.grad_se = grad_se;
    e = woi::launch_reduce(rp, s);
    if (e != hipSuccess) return fail(WOI_E_DEVICE, "reduce launch failed: %s", hipGetErrorString(e));
    return WOI_OK;
}

// Shared trajectories: per chunk, generate the trajectories of every point group, then
// evaluate them at the group's points; finally the deterministic per-point reduction.
woi_status estimate_shared(const woi_problem* p, const double* points, int64_t P, const woi_query* q, uint64_t ns,
                           double* mean, double* se, double* grad, double* grad_se, void* workspace,
                           size_t workspace_bytes, uint64_t* counters, hipStream_t s,
                           const uint64_t* seed_tab = nullptr) {
    const SharedPlan sp = make_shared_plan(p, P, q, ns);
    if (!workspace || workspace_bytes < sp.traj_bytes + sp.part_bytes)
        return fail(WOI_E_OOM, "workspace of %zu bytes is smaller than the %zu bytes needed", workspace_bytes,
                    sp.traj_bytes + sp.part_bytes);
    const unsigned lds = sp.lds;
    const bool vr = q->estimator == WOI_EST_VR, f32 = q->precision == WOI_PREC_FP32;
    woi::KParams kp{};
    kp.dp = static_cast<const DevProblem*>(p->dev);
    kp.points = points;
    kp.P = P;
    kp.n_samples = ns;
    kp.first_sample = q->estimator == WOI_EST_VR ? q->walk_offset / 2 : q->walk_offset;
    kp.k0 = (uint32_t)q->seed;
    kp.k1 = (uint32_t)(q->seed >> 32);
    kp.M = q->M;
    kp.batch_share = q->batch_share;
    kp.shared_sched = q->schedule_mode == WOI_SCHED_SHARED;
    kp.mesh = has_mesh(p->H) ? 1 : 0;
    kp.instance = q->instance;
    kp.partials = reinterpret_cast<double*>(static_cast<char*>(workspace) + sp.traj_bytes);
    kp.counters = counters;
    kp.seed_tab = seed_tab;
    woi::TParams tp{};
    tp.traj = workspace;
    tp.plane = sp.plane;
    tp.ng = sp.ng;
    tp.spt = sp.spt_g;
    tp.lg = sp.lg;
    tp.spt_e = sp.spt_e;
    tp.tile_rows = sp.tile_rows;
    if (q->event_begin && hipEventRecord(static_cast<hipEvent_t>(q->event_begin), s) != hipSuccess)
        return fail(WOI_E_DEVICE, "hipEventRecord(begin) failed");
    for (int c = 0; c < sp.n_chunks; ++c) {
        tp.chunk_first = (uint64_t)c * sp.chunk;
        tp.ns = (uint32_t)std::min<uint64_t>(sp.chunk, ns - tp.chunk_first);
        tp.accumulate = c > 0;
        hipError_t e = woi::launch_traj(kp, tp, p->H.m, vr, f32, lds, s);
        if (e != hipSuccess) return fail(WOI_E_DEVICE, "trajectory launch failed: %s", hipGetErrorString(e));
        e = woi::launch_eval(kp, tp, p->H.m, vr, f32, s);
        if (e != hipSuccess) return fail(WOI_E_DEVICE, "evaluation launch failed: %s", hipGetErrorString(e));
    }
    if (q->event_end && hipEventRecord(static_cast<hipEvent_t>(q->event_end), s) != hipSuccess)
        return fail(WOI_E_DEVICE, "hipEventRecord(end) failed");
    woi::RParams rp{};
    rp.partials = kp.partials;
    rp.P = P;
    rp.dim = p->H.m;
    rp.n_chunks = sp.n_slots();
    rp.samples_per_thread = sp.spt_e;
    rp.full = (uint64_t)(sp.n_chunks - 1) * sp.spt_e;
    rp.tail = ns - (uint64_t)(sp.n_chunks - 1) * sp.chunk;
    rp.mean = mean;
    rp.se = se;
    rp.grad = grad;
    rp.grad_se = grad_se;
    hipError_t e = woi::launch_reduce(rp, s);
    if (e != hipSuccess) return fail(WOI_E_DEVICE, "reduce launch failed: %s", hipGetErrorString(e));
    return WOI_OK;
}

}  // namespace

extern "C" {

woi_status woi_workspace_size(const woi_problem* p, int64_t P, const woi_query* q, size_t* bytes) {
    woi_status st = check_query_impl(p, P, q);
    if (st != WOI_OK) return st;
    if (!bytes) return fail(WOI_E_INVALID_ARG, "NULL bytes");
    const uint64_t ns = q->estimator == WOI_EST_VR ? q->walks / 2 : q->walks;
    if (q->estimator == WOI_EST_NAIVE) {
        const NaivePlan pl = make_naive_plan(p, P, q, ns);
        *bytes = (size_t)pl.chunks * (size_t)P * (2 + 2 * p->H.m) * sizeof(double);
        return WOI_OK;
    }
    if (q->batch_share > 1) {
        const SharedPlan sp = make_shared_plan(p, P, q, ns);
        *bytes = sp.traj_bytes + sp.part_bytes;
        return WOI_OK;
    }
    const Plan pl = make_plan(p, P, q, ns);
    *bytes = (size_t)pl.chunks * (size_t)P * (2 + 2 * p->H.m) * sizeof(double);
    return WOI_OK;
}

woi_status woi_estimate(const woi_problem* p, const double* points, int64_t P, const woi_query* q, double* mean,
                        double* se, double* grad, double* grad_se, void* workspace, size_t workspace_bytes,
                        uint64_t* counters, void* stream) {
    woi_status st = check_query_impl(p, P, q);
    if (st != WOI_OK) return st;
    if (!points || !mean || !se) return fail(WOI_E_INVALID_ARG, "NULL points/mean/se");
    st = woi_problem_upload(const_cast<woi_problem*>(p));
    if (st != WOI_OK) return st;
    const uint64_t ns = q->estimator == WOI_EST_VR ? q->walks / 2 : q->walks;
    if (q->estimator == WOI_EST_NAIVE)
        return estimate_naive(p, points, P, q, mean, se, grad, grad_se, workspace, workspace_bytes, counters,
                              static_cast<hipStream_t>(stream));
    if (q->batch_share > 1)
        return estimate_shared(p, points, P, q, ns, mean, se, grad, grad_se, workspace, workspace_bytes, counters,
                               static_cast<hipStream_t>(stream));
    const Plan pl = make_plan(p, P, q, ns);
    const size_t need = (size_t)pl.chunks * (size_t)P * (2 + 2 * p->H.m) * sizeof(double);
    if (!workspace || workspace_bytes < need)
        return fail(WOI_E_OOM, "workspace of %zu bytes is smaller than the %zu bytes needed", workspace_bytes, need);
    return launch_per_point(p, points, P, q, pl, mean, se, grad, grad_se, static_cast<double*>(workspace), counters,
                            static_cast<hipStream_t>(stream));
}

woi_status woi_stats_read(const uint64_t* counters, void* event_begin, void* event_end, woi_stats* out) {
    if (!out) return fail(WOI_E_INVALID_ARG, "NULL stats");
    uint64_t c[WOI_COUNTERS] = {0};
    if (counters && hipMemcpy(c, counters, sizeof c, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(WOI_E_DEVICE, "hipMemcpy of the counters failed");
    out->walker_steps = c[0];
    out->redraws = c[1];
    out->rejections = c[2];
    out->cap_hits = c[3];
    out->zero_distances = c[4];
    out->search_node_tests = c[5];
    out->segment_tests = c[6];
    out->other_transitions = c[7];
    out->fp64_fallbacks = c[8];
    out->seconds = -1.0;
    if (event_begin && event_end) {
        float ms = 0.0f;
        if (hipEventSynchronize(static_cast<hipEvent_t>(event_end)) != hipSuccess ||
            hipEventElapsedTime(&ms, static_cast<hipEvent_t>(event_begin), static_cast<hipEvent_t>(event_end)) !=
                hipSuccess)
            return fail(WOI_E_DEVICE, "hipEventElapsedTime failed");
        out->seconds = 1e-3 * (double)ms;
    }
    return WOI_OK;
}

woi_status woi_training_points(const woi_problem* p, const woi_training_spec* spec, double* interior, int64_t cap,
                               int64_t* n_interior, double* bc_points, double* bc_normals, double* bc_flux,
                               int64_t* n_bc, void* stream) {
    if (!p || !spec || !n_interior || cap < 0 || (cap > 0 && !interior))
        return fail(WOI_E_INVALID_ARG, "NULL problem, spec or count, or no interior array for cap > 0");
    const Host& H = p->H;
    const int m = H.m;
    if (spec->grid_n < 1 || spec->bc_n < 0 || !(spec->margin >= 0))
        return fail(WOI_E_INVALID_ARG, "grid_n must be >= 1, bc_n >= 0, margin >= 0");
    if (spec->bc_n > 0 && m != 2 && m != 3) return fail(WOI_E_UNSUPPORTED, "boundary samples need dim 2 or 3");
    if (spec->bc_n > 0 && (!bc_points || !bc_normals || !bc_flux)) return fail(WOI_E_INVALID_ARG, "NULL boundary arrays");
    if (has_mesh(H)) return fail(WOI_E_UNSUPPORTED, "training points are not built for triangle meshes");
    if (std::pow((double)spec->grid_n, (double)m) > 1e10) return fail(WOI_E_INVALID_ARG, "grid_n^dim exceeds 1e10 nodes");
    woi_status st = woi_problem_upload(const_cast<woi_problem*>(p));
    if (st != WOI_OK) return st;
    woi::TrainParams tp{};
    tp.dp = static_cast<const DevProblem*>(p->dev);
    tp.n = spec->grid_n;
    const HostRegion& g = H.r[0];
    for (int d = 0; d < m; ++d) {
        double lo = 0, hi = 0;
        if (g.kind == WOI_SHAPE_SPHERE || g.kind == WOI_SHAPE_ELLIPSOID) {
            double half = g.R;
            if (g.kind == WOI_SHAPE_ELLIPSOID) {   // extent along axis d: sqrt((A^-1)_dd), A^-1 = L L
                double s2 = 0;
                for (int j = 0; j < m; ++j) s2 += g.L[d * m + j] * g.L[d * m + j];
                half = std::sqrt(s2);
            }
            lo = g.c[d] - half;
            hi = g.c[d] + half;
        } else {
            lo = hi = g.v[d];
            for (int j = 0; j < g.nv(); ++j) { lo = std::min(lo, g.v[2 * j + d]); hi = std::max(hi, g.v[2 * j + d]); }
        }
        tp.lo[d] = lo;
        tp.step[d] = (hi - lo) / spec->grid_n;
    }
    tp.margin = spec->margin;
    tp.nodes = 1;
    for (int d = 0; d < m; ++d) tp.nodes *= (uint64_t)spec->grid_n;
    tp.out = interior;
    tp.cap = cap;
    tp.bc_n = spec->bc_n;
    tp.n_bc = spec->bc_n == 0 ? 0 : (m == 2 ? spec->bc_n : 2 * (int64_t)spec->bc_n * spec->bc_n);
    tp.bc_points = bc_points;
    tp.bc_normals = bc_normals;
    tp.bc_flux = bc_flux;
    if (n_bc) *n_bc = tp.n_bc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t* dcount = nullptr;
    if (hipMalloc(&dcount, sizeof(int64_t)) != hipSuccess) return fail(WOI_E_OOM, "hipMalloc(8) failed");
    tp.count = dcount;
    hipError_t e = woi::launch_training(tp, m, s);
    if (e == hipSuccess) e = hipMemcpyAsync(n_interior, dcount, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dcount);
    if (e != hipSuccess) return fail(WOI_E_DEVICE, "training points: %s", hipGetErrorString(e));
    return WOI_OK;
}

woi_status woi_trace(const woi_problem* p, const double* points, int64_t P, const woi_query* q, uint64_t n_samples,
                     double* F, double* G, uint32_t* trace, void* stream) {
    woi_query qq = *q;
    qq.walks = q->estimator == WOI_EST_VR ? 2 * n_samples : n_samples;
    woi_status st = check_query_impl(p, P, &qq);
    if (st != WOI_OK) return st;
    if (!points || !F) return fail(WOI_E_INVALID_ARG, "NULL points or F");
    st = woi_problem_upload(const_cast<woi_problem*>(p));
    if (st != WOI_OK) return st;
    if (q->estimator == WOI_EST_NAIVE) {
        if (trace) return fail(WOI_E_INVALID_ARG, "naive trees have no decision words: pass trace = NULL");
        const NaivePlan pl = make_naive_plan(p, P, &qq, n_samples);
        woi::KParams kp = naive_params(p, points, P, &qq, n_samples, pl);
        kp.traceF = F;
        kp.traceG = G;
        hipError_t e = woi::launch_naive(kp, pl.np, p->H.m, q->precision == WOI_PREC_FP32, dim3(pl.gx, pl.chunks),
                                         static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return fail(WOI_E_DEVICE, "naive launch failed: %s", hipGetErrorString(e));
        return WOI_OK;
    }
    const Plan pl = make_plan(p, P, &qq, n_samples);
    woi::KParams kp{};
    kp.dp = static_cast<const DevProblem*>(p->dev);
    kp.points = points;
    kp.P = P;
    kp.n_samples = n_samples;
    kp.first_sample = pl.first;
    kp.samples_per_thread = pl.spt;
    kp.k0 = (uint32_t)q->seed;
    kp.k1 = (uint32_t)(q->seed >> 32);
    kp.M = q->M;
    kp.batch_share = q->batch_share;
    kp.shared_sched = q->schedule_mode == WOI_SCHED_SHARED;
    kp.mesh = has_mesh(p->H) ? 1 : 0;
    kp.instance = q->instance;
    kp.traceF = F;
    kp.traceG = G;
    kp.trace = trace;
    hipError_t e = woi::launch_walk(kp, p->H.m, q->estimator == WOI_EST_VR, q->precision == WOI_PREC_FP32, pl.lds,
                                    dim3(pl.gx, pl.chunks), dim3(pl.block), static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(WOI_E_DEVICE, "walk launch failed: %s", hipGetErrorString(e));
    return WOI_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------- internal helpers
namespace woi {

woi_status set_error(woi_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

woi_status check_query(const woi_problem* p, int64_t P, const woi_query* q) { return check_query_impl(p, P, q); }

size_t shared_workspace_bytes(const woi_problem* p, int64_t P, const woi_query* q) {
    const uint64_t ns = q->estimator == WOI_EST_VR ? q->walks / 2 : q->walks;
    const SharedPlan sp = make_shared_plan(p, P, q, ns);
    return sp.traj_bytes + sp.part_bytes;
}

woi_status enqueue_shared(const woi_problem* p, const double* points, int64_t P, const woi_query* q, double* mean,
                          double* se, double* grad, double* grad_se, void* workspace, size_t workspace_bytes,
                          uint64_t* counters, const uint64_t* seed_tab, void* stream) {
    const uint64_t ns = q->estimator == WOI_EST_VR ? q->walks / 2 : q->walks;
    return estimate_shared(p, points, P, q, ns, mean, se, grad, grad_se, workspace, workspace_bytes, counters,
                           static_cast<hipStream_t>(stream), seed_tab);
}

woi_status estimate_into(const woi_problem* p, const double* points, int64_t P, const woi_query* q, double* mean,
                         double* se, double* grad, double* grad_se, double* partials, size_t partial_bytes,
                         uint64_t* counters, void* stream) {
    woi_status st = check_query_impl(p, P, q);
    if (st != WOI_OK) return st;
    if (!points || !mean || !se) return fail(WOI_E_INVALID_ARG, "NULL points/mean/se");
    if (q->estimator == WOI_EST_NAIVE || q->batch_share != 1)
        return fail(WOI_E_UNSUPPORTED, "the allocation-free path takes the plain and VR estimators with batch_share 1");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(WOI_E_DEVICE, "no HIP device");
    {
        std::lock_guard<std::mutex> lk(const_cast<woi_problem*>(p)->mu);
        if (!p->dev) return fail(WOI_E_INVALID_ARG, "the problem is not on a device: call woi_problem_upload first");
        if (p->device != cur)
            return fail(WOI_E_INVALID_ARG, "problem lives on device %d, current device is %d", p->device, cur);
    }
    const size_t rec = (size_t)P * (2 + 2 * p->H.m) * sizeof(double);   // one chunk of partials
    const uint64_t max_chunks = partial_bytes / rec;
    if (max_chunks < 1)
        return fail(WOI_E_INVALID_ARG, "%lld points need %zu bytes of partial sums, more than the %zu available",
                    (long long)P, rec, partial_bytes);
    const uint64_t ns = q->estimator == WOI_EST_VR ? q->walks / 2 : q->walks;
    const Plan pl = make_plan(p, P, q, ns, max_chunks);
    if ((uint64_t)pl.chunks > max_chunks)
        return fail(WOI_E_INVALID_ARG, "%llu samples need %d partial slots, more than the %llu that fit",
                    (unsigned long long)ns, pl.chunks, (unsigned long long)max_chunks);
    return launch_per_point(p, points, P, q, pl, mean, se, grad, grad_se, partials, counters,
                            static_cast<hipStream_t>(stream));
}
bool problem_has_mesh(const woi_problem* p) { return p && has_mesh(p->H); }

woi_status problem_ref(woi_problem* p, ProblemRef* out) {
    const woi_status st = woi_problem_upload(p);
    if (st != WOI_OK) return st;
    out->dev = static_cast<const DevProblem*>(p->dev);
    out->host = reinterpret_cast<const DevProblem*>(p->blob.data());
    out->dim = p->H.m;
    out->serial = p->serial;
    return WOI_OK;
}

}  // namespace woi
