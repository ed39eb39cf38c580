/*
 * woi_oracle.c -- slow, plain FP64 CPU oracle for Walk-on-Interfaces (WoI).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, the smoke check and the CPU-baseline
 * leg of the benchmark, never by the product path.  Shares no code with the GPU
 * library.  Written for readability: brute-force geometry, one walk at a time,
 * in the order of the paper's algorithms (Ding & Stinchcombe, arXiv 2508.16767).
 *
 * Readings of the paper taken here (the paper is ambiguous or self-contradictory
 * at these points):
 *   - sign product over m = 1..i (Eq. woi_estimator, Theorem 2), not m = 0..i;
 *   - K*_{h_i,h_{i-1}}(y_i, y_{i-1}) uses the normal at y_i (definition of K*_{ij}
 *     in Sec. 3); in the "other" transition the sign is applied once:
 *     Q *= |K*| |dOmega|, T *= sign((y_i - y_{i-1}) . n(y_i));
 *   - line case: q counts intersections other than y_{i-1}; the pick among the q
 *     hits is uniform; hits are ordered by segment index (polylines); a polyline hit
 *     within |t| <= 1e-12 of y_{i-1} (a vertex shared with its segment) is y_{i-1};
 *   - "descendant" means strict descendant in the region tree;
 *   - VR halves: dOmega^+ = {beta >= 0}; an empty half contributes 0; for VR the
 *     walker count W gives W/2 two-walker samples;
 *   - one schedule per sample (S = W in Alg. 1), weights w_i = 1 - delta_{iM}/2;
 *   - q = 0 (rounding at tangency) and rejected proposals redraw from the next
 *     attempt's counters; after OR_MAX_ATTEMPTS the walker stops (counted).
 */
#include "woi_oracle.h"
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_ATTEMPTS 256
/* OR_PLANT selects a deliberately wrong variant, built only by the tests that show
   the pins reject it: 1 sign product from m = 0, 2 sign applied twice in the "other"
   transition, 3 no 1/2 weight on the last term, 4 K* with the normal at y_{i-1},
   5 T without the intersection count q, 6 naive trees weighted by |alpha| instead of alpha,
   7 the ellipsoid surface Jacobian of the VR half-measure quadrature without its square root. */
#ifndef OR_PLANT
#define OR_PLANT 0
#endif
#define OR_PI 3.14159265358979323846

/* ---------------------------------------------------------------- Philox4x32-10 */
/* Salmon et al., SC'11: 10 rounds of the 4x32 Philox S-box with Weyl key schedule. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

static double unif(uint32_t v) { return ((double)v + 0.5) * (1.0 / 4294967296.0); }

/* A word stream for one (walk, stream, instance|walker|purpose, step) counter prefix.
   Paired streams (2D transitions): draw 0 (the first attempt, at most two words) comes from
   the block shared by steps 2k+1 and 2k+2, counter word 3 = (0x8000 | k) << 16, words 0-1
   for step 2k+1 and 2-3 for step 2k+2; later attempts draw from (step, draw) as usual. */
typedef struct {
    uint32_t key[2], c0, c1, c2, step, draw;
    uint32_t buf[4];
    int pos, paired;
} words_t;

static void words_init(words_t *w, uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t step)
{
    w->key[0] = (uint32_t)seed; w->key[1] = (uint32_t)(seed >> 32);
    w->c0 = c0; w->c1 = c1; w->c2 = c2; w->step = step; w->draw = 0; w->pos = 4; w->paired = 0;
}
static void words_seek(words_t *w, uint32_t draw) { w->draw = draw; w->pos = 4; }
static uint32_t words_next(words_t *w)
{
    if (w->pos == 4) {
        const int pair = w->paired && w->draw == 0;
        uint32_t ctr[4] = {w->c0, w->c1, w->c2,
                           pair ? (0x8000u | ((w->step - 1) >> 1)) << 16 : (w->step << 16) | (w->draw & 0xFFFFu)};
        or_philox4x32_10(ctr, w->key, w->buf);
        w->pos = pair ? 2 * (int)((w->step - 1) & 1) : 0;
        w->draw++;
    }
    return w->buf[w->pos++];
}

/* ---------------------------------------------------------------- problem */
typedef struct {
    int kind;
    double c[OR_MAX_DIM], R;
    double A[OR_MAX_DIM * OR_MAX_DIM], L[OR_MAX_DIM * OR_MAX_DIM], lam_max, detL;
    int nv;
    double *v, *len, *cum, total;   /* polyline; mesh: v = vertices (3 each), cum = cumulative triangle areas */
    int ntri, *tri;                 /* mesh triangles (3 vertex indices each) */
    double *tn;                     /* mesh: unit outward normal per triangle */
    double area;
    int dkind, nt;
    double dc[OR_MAX_DIM];
    double *coef;
    unsigned char *exps;
    double alpha, s, flux;
    double meas[2];       /* |dOmega^+|, |dOmega^-| */
    int nbrk, class0;     /* 2D: breakpoints in arclength, class at s = 0 */
    double *brk;
} region_t;

struct or_problem {
    int m, N;
    int parent[OR_MAX_REGIONS];
    double sigma[OR_MAX_REGIONS];
    region_t r[OR_MAX_REGIONS];
    double alpha_l1, cdf[OR_MAX_REGIONS];
    int rel[OR_MAX_REGIONS][OR_MAX_REGIONS]; /* 1 SAME, 2 DESC, 3 OTHER */
    double unit_area;                        /* m alpha(m) = |S^{m-1}| */
    int vr_ok;
};

static double dot(const double *a, const double *b, int m)
{
    double s = 0; for (int i = 0; i < m; ++i) s += a[i] * b[i]; return s;
}

/* Jacobi eigen-decomposition of a symmetric m x m matrix: A = V diag(e) V^T. */
static void jacobi_eig(const double *A, int m, double *e, double *V)
{
    double a[OR_MAX_DIM * OR_MAX_DIM];
    memcpy(a, A, sizeof(double) * m * m);
    for (int i = 0; i < m * m; ++i) V[i] = 0;
    for (int i = 0; i < m; ++i) V[i * m + i] = 1;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0;
        for (int i = 0; i < m; ++i) for (int j = i + 1; j < m; ++j) off += a[i * m + j] * a[i * m + j];
        if (off < 1e-300) break;
        for (int p = 0; p < m; ++p) for (int q = p + 1; q < m; ++q) {
            if (fabs(a[p * m + q]) < 1e-300) continue;
            double th = (a[q * m + q] - a[p * m + p]) / (2 * a[p * m + q]);
            double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1));
            double c = 1 / sqrt(t * t + 1), s = t * c;
            for (int k = 0; k < m; ++k) { /* columns p,q */
                double akp = a[k * m + p], akq = a[k * m + q];
                a[k * m + p] = c * akp - s * akq; a[k * m + q] = s * akp + c * akq;
            }
            for (int k = 0; k < m; ++k) { /* rows p,q */
                double apk = a[p * m + k], aqk = a[q * m + k];
                a[p * m + k] = c * apk - s * aqk; a[q * m + k] = s * apk + c * aqk;
            }
            for (int k = 0; k < m; ++k) {
                double vkp = V[k * m + p], vkq = V[k * m + q];
                V[k * m + p] = c * vkp - s * vkq; V[k * m + q] = s * vkp + c * vkq;
            }
        }
    }
    for (int i = 0; i < m; ++i) e[i] = a[i * m + i];
}

/* Gauss-Legendre nodes/weights on [-1, 1] (Newton on P_n). */
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (n + 0.5)), pp = 0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1, p2 = 0;
            for (int j = 1; j <= n; ++j) { double p3 = p2; p2 = p1; p1 = ((2 * j - 1) * z * p2 - (j - 1) * p3) / j; }
            pp = n * (z * p1 - p2) / (z * z - 1);
            double z1 = z; z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-16) break;
        }
        x[i] = z; w[i] = 2 / ((1 - z * z) * pp * pp);
    }
}

/* ---- point geometry */
static void normal_at(const region_t *g, int m, const double *y, int seg, double *n)
{
    if (g->kind == OR_SPHERE) {
        for (int i = 0; i < m; ++i) n[i] = (y[i] - g->c[i]) / g->R;
    } else if (g->kind == OR_ELLIPSOID) {
        double s = 0;
        for (int i = 0; i < m; ++i) {
            double t = 0; for (int j = 0; j < m; ++j) t += g->A[i * m + j] * (y[j] - g->c[j]);
            n[i] = t; s += t * t;
        }
        s = sqrt(s); for (int i = 0; i < m; ++i) n[i] /= s;
    } else if (g->kind == OR_MESH) {
        for (int i = 0; i < 3; ++i) n[i] = g->tn[3 * seg + i];
    } else {
        const double *a = g->v + 2 * seg, *b = g->v + 2 * ((seg + 1) % g->nv);
        double ex = b[0] - a[0], ey = b[1] - a[1], l = sqrt(ex * ex + ey * ey);
        n[0] = ey / l; n[1] = -ex / l;
    }
}

/* b_i(y): the flux-jump / Neumann datum of the region (Eq. interface_problem). */
static double data_b(const region_t *g, int m, const double *y, int seg)
{
    if (g->dkind == OR_DATA_ZERO) return 0.0;
    if (g->dkind == OR_DATA_FIELD_FLUX) {
        double n[OR_MAX_DIM];
        normal_at(g, m, y, seg, n);
        return dot(g->coef, n, m);
    }
    if (g->dkind == OR_DATA_SOURCE_FLUX) {
        double n[OR_MAX_DIM], d[OR_MAX_DIM], r2 = 0;
        normal_at(g, m, y, seg, n);
        for (int i = 0; i < m; ++i) { d[i] = y[i] - g->dc[i]; r2 += d[i] * d[i]; }
        return g->coef[0] * dot(d, n, m) / pow(r2, 0.5 * m);
    }
    double e[OR_MAX_DIM], r = 0;
    for (int i = 0; i < m; ++i) { e[i] = y[i] - g->dc[i]; r += e[i] * e[i]; }
    r = sqrt(r);
    for (int i = 0; i < m; ++i) e[i] /= r;
    if (g->dkind == OR_DATA_FOURIER2D) {
        double th = atan2(e[1], e[0]), b = g->coef[0];
        for (int k = 1; k <= g->nt; ++k) b += g->coef[2 * k - 1] * cos(k * th) + g->coef[2 * k] * sin(k * th);
        return b;
    }
    double b = 0; /* DIRPOLY */
    for (int t = 0; t < g->nt; ++t) {
        double term = g->coef[t];
        for (int i = 0; i < m; ++i) for (int p = 0; p < g->exps[t * m + i]; ++p) term *= e[i];
        b += term;
    }
    return b;
}

static double beta_at(const or_problem *pr, int h, const double *y, int seg)
{
    return pr->r[h].s * data_b(&pr->r[h], pr->m, y, seg);
}

/* ---- sampling from attempt words */
static int dir_words(int m) { return m == 2 ? 1 : (m == 3 ? 2 : 2 * ((m + 1) / 2)); }

static void unit_dir(int m, words_t *w, double *d)
{
    if (m == 2) {
        double ph = 2 * OR_PI * unif(words_next(w));
        d[0] = cos(ph); d[1] = sin(ph);
    } else if (m == 3) {
        double z = 2 * unif(words_next(w)) - 1, ph = 2 * OR_PI * unif(words_next(w));
        double r = sqrt(fmax(0.0, 1 - z * z));
        d[0] = r * cos(ph); d[1] = r * sin(ph); d[2] = z;
    } else {
        double g[OR_MAX_DIM + 1], s = 0;
        for (int j = 0; j < (m + 1) / 2; ++j) {
            double u1 = unif(words_next(w)), u2 = unif(words_next(w));
            double rr = sqrt(-2 * log(u1));
            g[2 * j] = rr * cos(2 * OR_PI * u2); g[2 * j + 1] = rr * sin(2 * OR_PI * u2);
        }
        for (int i = 0; i < m; ++i) s += g[i] * g[i];
        s = sqrt(s);
        for (int i = 0; i < m; ++i) d[i] = g[i] / s;
    }
}

static void polyline_at(const region_t *g, double s, double *y, int *seg)
{
    int lo = 0, hi = g->nv - 1; /* largest j with cum[j] <= s */
    while (lo < hi) { int mid = (lo + hi + 1) / 2; if (g->cum[mid] <= s) lo = mid; else hi = mid - 1; }
    const double *a = g->v + 2 * lo, *b = g->v + 2 * ((lo + 1) % g->nv);
    double f = (s - g->cum[lo]) / g->len[lo];
    y[0] = a[0] + f * (b[0] - a[0]); y[1] = a[1] + f * (b[1] - a[1]);
    *seg = lo;
}

/* words per attempt of a uniform surface sample */
static int surf_words(const region_t *g, int m)
{
    if (g->kind == OR_POLYLINE) return 1;
    if (g->kind == OR_MESH) return 3;
    return dir_words(m) + (g->kind == OR_ELLIPSOID ? 1 : 0);
}

/* One attempt of a uniform sample on the interface; returns 0 if rejected. */
static int surf_attempt(const region_t *g, int m, words_t *w, double *y, int *seg)
{
    *seg = 0;
    if (g->kind == OR_POLYLINE) { polyline_at(g, unif(words_next(w)) * g->total, y, seg); return 1; }
    if (g->kind == OR_MESH) {
        /* triangle with probability area / total (largest j with cum[j] <= s), then a uniform
           point in it: y = (1 - r) a + r (1 - u) b + r u c with r = sqrt(u1) */
        double s = unif(words_next(w)) * g->total;
        int lo = 0, hi = g->ntri - 1;
        while (lo < hi) { int mid = (lo + hi + 1) / 2; if (g->cum[mid] <= s) lo = mid; else hi = mid - 1; }
        double r = sqrt(unif(words_next(w))), u2 = unif(words_next(w));
        const int *t = g->tri + 3 * lo;
        const double *a = g->v + 3 * t[0], *b = g->v + 3 * t[1], *c = g->v + 3 * t[2];
        for (int i = 0; i < 3; ++i) y[i] = (1 - r) * a[i] + r * (1 - u2) * b[i] + r * u2 * c[i];
        *seg = lo;
        return 1;
    }
    double u[OR_MAX_DIM];
    unit_dir(m, w, u);
    if (g->kind == OR_SPHERE) { for (int i = 0; i < m; ++i) y[i] = g->c[i] + g->R * u[i]; return 1; }
    /* ellipsoid: y = c + A^{-1/2} u, accepted with probability |A^{1/2} u| / sqrt(lam_max) */
    double acc = unif(words_next(w)), uAu = 0;
    for (int i = 0; i < m; ++i) for (int j = 0; j < m; ++j) uAu += u[i] * g->A[i * m + j] * u[j];
    for (int i = 0; i < m; ++i) { double t = 0; for (int j = 0; j < m; ++j) t += g->L[i * m + j] * u[j]; y[i] = g->c[i] + t; }
    return acc < sqrt(uAu / g->lam_max);
}

/* point at arclength s on a 2D closed curve (circle or polyline) */
static void curve_at(const region_t *g, double s, double *y, int *seg)
{
    if (g->kind == OR_POLYLINE) { polyline_at(g, s, y, seg); return; }
    double ph = s / g->R;
    y[0] = g->c[0] + g->R * cos(ph); y[1] = g->c[1] + g->R * sin(ph); *seg = 0;
}

/* uniform sample on the VR half `cls` (0: beta >= 0, 1: beta < 0) */
static int vr_words(const or_problem *pr, const region_t *g)
{
    return pr->m == 2 ? 1 : surf_words(g, pr->m);
}
static int vr_attempt(const or_problem *pr, int h, int cls, words_t *w, double *y, int *seg)
{
    const region_t *g = &pr->r[h];
    if (pr->m == 2) {
        double t = unif(words_next(w)) * g->meas[cls], start = 0, acc = 0;
        int c = g->class0;
        for (int p = 0; p <= g->nbrk; ++p) {
            double end = p < g->nbrk ? g->brk[p] : g->total;
            if (c == cls) {
                double l = end - start;
                if (t < acc + l || p == g->nbrk) { curve_at(g, fmin(start + (t - acc), end), y, seg); return 1; }
                acc += l;
            }
            start = end; c ^= 1;
        }
        curve_at(g, start, y, seg);
        return 1;
    }
    if (!surf_attempt(g, pr->m, w, y, seg)) return 0;
    return (beta_at(pr, h, y, *seg) >= 0) == (cls == 0);
}

/* ---- intersections: hits of the line/ray y + t d with interface g, in segment order.
   Returns the number q of hits; hits first .. first + cap - 1 (in that order) are stored. */
typedef struct { double t; int seg; } hit_t;

static int hits_of(const region_t *g, int m, const double *y, int yseg, const double *d, int ray, hit_t *out,
                   int first, int cap)
{
    if (g->kind == OR_SPHERE || g->kind == OR_ELLIPSOID) {
        double yc[OR_MAX_DIM], Ad[OR_MAX_DIM], Ayc[OR_MAX_DIM];
        for (int i = 0; i < m; ++i) yc[i] = y[i] - g->c[i];
        double a, b, cc;
        if (g->kind == OR_SPHERE) {
            a = 1; b = dot(yc, d, m); cc = dot(yc, yc, m) - g->R * g->R;
        } else {
            for (int i = 0; i < m; ++i) {
                double s1 = 0, s2 = 0;
                for (int j = 0; j < m; ++j) { s1 += g->A[i * m + j] * d[j]; s2 += g->A[i * m + j] * yc[j]; }
                Ad[i] = s1; Ayc[i] = s2;
            }
            a = dot(d, Ad, m); b = dot(d, Ayc, m); cc = dot(yc, Ayc, m) - 1;
        }
        double t;
        if (!ray) { /* y on the quadric: the other root of t (a t + 2 b) = 0 */
            t = -2 * b / a;
            if (t == 0) return 0;
        } else {
            double disc = b * b - a * cc; /* origin strictly inside: cc < 0 */
            if (disc < 0) return 0;
            t = (-b + sqrt(disc)) / a;
            if (!(t > 0)) return 0;
        }
        if (first == 0 && cap > 0) { out[0].t = t; out[0].seg = 0; }
        return 1;
    }
    int q = 0;
    if (g->kind == OR_MESH) {
        /* Moller-Trumbore per triangle, in triangle order; a line skips the triangle of y */
        for (int j = 0; j < g->ntri; ++j) {
            if (!ray && j == yseg) continue;
            const int *tt = g->tri + 3 * j;
            const double *a = g->v + 3 * tt[0], *b = g->v + 3 * tt[1], *c = g->v + 3 * tt[2];
            double e1[3], e2[3], sv[3], pv[3], qv[3];
            for (int i = 0; i < 3; ++i) { e1[i] = b[i] - a[i]; e2[i] = c[i] - a[i]; sv[i] = y[i] - a[i]; }
            pv[0] = d[1] * e2[2] - d[2] * e2[1]; pv[1] = d[2] * e2[0] - d[0] * e2[2]; pv[2] = d[0] * e2[1] - d[1] * e2[0];
            double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
            if (det == 0) continue;
            double u = (sv[0] * pv[0] + sv[1] * pv[1] + sv[2] * pv[2]) / det;
            if (u < 0 || u > 1) continue;
            qv[0] = sv[1] * e1[2] - sv[2] * e1[1]; qv[1] = sv[2] * e1[0] - sv[0] * e1[2]; qv[2] = sv[0] * e1[1] - sv[1] * e1[0];
            double v = (d[0] * qv[0] + d[1] * qv[1] + d[2] * qv[2]) / det;
            if (v < 0 || u + v > 1) continue;
            double t = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) / det;
            if (ray ? !(t > 0) : fabs(t) <= 1e-12) continue;
            if (q >= first && q - first < cap) { out[q - first].t = t; out[q - first].seg = j; }
            q++;
        }
        return q;
    }
    for (int j = 0; j < g->nv; ++j) {
        if (!ray && j == yseg) continue;
        const double *a = g->v + 2 * j, *b = g->v + 2 * ((j + 1) % g->nv);
        double ex = b[0] - a[0], ey = b[1] - a[1];
        double den = d[0] * ey - d[1] * ex;
        if (den == 0) continue;
        double wx = a[0] - y[0], wy = a[1] - y[1];
        double t = (wx * ey - wy * ex) / den;
        double s = (wx * d[1] - wy * d[0]) / den;
        if (s < 0 || s >= 1) continue;
        if (ray ? !(t > 0) : fabs(t) <= 1e-12) continue;   /* |t| <= 1e-12: y_{i-1} itself */
        if (q >= first && q - first < cap) { out[q - first].t = t; out[q - first].seg = j; }
        q++;
    }
    return q;
}

/* ---------------------------------------------------------------- Green's function */
/* Phi(x,y) = -ln|x-y|/(2 pi) (m=2), |x-y|^{2-m}/(m(m-2)alpha(m)) (m>=3);
   grad_x Phi = -(x-y)/(m alpha(m) |x-y|^m)  (Sec. 2). */
static int add_term(const or_problem *pr, const double *x, const double *y, double c, double *F, double *G)
{
    int m = pr->m;
    double d[OR_MAX_DIM], r2 = 0;
    for (int i = 0; i < m; ++i) { d[i] = x[i] - y[i]; r2 += d[i] * d[i]; }
    if (r2 == 0) return 1;
    double r = sqrt(r2), phi;
    if (m == 2) phi = -log(r) / (2 * OR_PI);
    else phi = pow(r, 2 - m) / ((m - 2) * pr->unit_area);
    *F += c * phi;
    double gs = -c / (pr->unit_area * pow(r, m));
    for (int i = 0; i < m; ++i) G[i] += gs * d[i];
    return 0;
}

/* ---------------------------------------------------------------- one sample */
enum { REL_SAME = 1, REL_DESC = 2, REL_OTHER = 3 };

static uint32_t trace_word(int h, int cs, int q, int pick, int neg, int att)
{
    if (q > 255) q = 255;
    if (pick > 255) pick = 255;
    if (att > 127) att = 127;
    return (uint32_t)h | ((uint32_t)cs << 6) | ((uint32_t)q << 8) | ((uint32_t)pick << 16) |
           ((uint32_t)(neg ? 1 : 0) << 24) | ((uint32_t)att << 25);
}

/* One transition y_{i-1} -> y_i onto interface h (the three cases of Eq. naive_woi_p):
   uniform on dOmega_h with Q *= |K*(y_i, y_{i-1})| |dOmega_h| ("other"), or the isotropic
   line (same interface, Q *= 1/2) / ray (descendant -> ancestor) with a uniform pick among
   its q hits.  Returns the factor q sign((y_i - y_{i-1}) . n(y_i)) of T, or 0 when no line
   or ray hit turned up within OR_MAX_ATTEMPTS draws (the walk stops there). */
static double transition(const or_problem *pr, int hprev, int h, words_t *w, const double *y, int seg,
                         double *yn, int *segn, double *nn, double *Q, int *qn_out, int *pick_out, int *att_out,
                         or_counters *cnt)
{
    const int m = pr->m;
    const region_t *g = &pr->r[h];
    const int rel = pr->rel[hprev][h];
    int qn = 1, pick = 0, att;
    *segn = 0;
    if (rel == REL_OTHER) {
        /* y_i uniform on dOmega_{h_i}; Q *= |K*(y_i, y_{i-1})| |dOmega_{h_i}| */
        int nbo = (surf_words(g, m) + 3) / 4;
        for (att = 0; att < OR_MAX_ATTEMPTS; ++att) {
            words_seek(w, (uint32_t)(att * nbo));
            if (surf_attempt(g, m, w, yn, segn)) break;
            cnt->rejections++;
        }
        if (att == OR_MAX_ATTEMPTS) cnt->cap_hits++;
        normal_at(g, m, yn, *segn, nn);
        double dd[OR_MAX_DIM], r2 = 0, nk[OR_MAX_DIM];
        for (int j = 0; j < m; ++j) { dd[j] = yn[j] - y[j]; r2 += dd[j] * dd[j]; }
        if (OR_PLANT == 4) normal_at(&pr->r[hprev], m, y, seg, nk); else memcpy(nk, nn, sizeof nk);
        double kstar = dot(dd, nk, m) / (pr->unit_area * pow(r2, 0.5 * m));
        *Q *= (OR_PLANT == 2 ? kstar : fabs(kstar)) * g->area;
    } else {
        /* isotropic line (same interface) or ray (descendant -> ancestor), uniform pick */
        hit_t hits[512];
        int nbl = (dir_words(m) + 1 + 3) / 4, found = 0;
        for (att = 0; att < OR_MAX_ATTEMPTS; ++att) {
            double d[OR_MAX_DIM];
            words_seek(w, (uint32_t)(att * nbl));
            unit_dir(m, w, d);
            double up = unif(words_next(w));
            qn = hits_of(g, m, y, seg, d, rel == REL_DESC, hits, 0, 512);
            if (qn == 0) { cnt->redraws++; continue; }
            pick = (int)floor(up * qn);
            if (pick >= qn) pick = qn - 1;
            const hit_t *hp = hits + pick;
            if (pick >= 512) {   /* beyond the stored hits: find hit `pick` by a second scan */
                hits_of(g, m, y, seg, d, rel == REL_DESC, hits, pick, 1);
                hp = hits;
            }
            if (g->kind == OR_POLYLINE) {
                int j = hp->seg;
                const double *a = g->v + 2 * j, *b = g->v + 2 * ((j + 1) % g->nv);
                double ex = b[0] - a[0], ey = b[1] - a[1];
                double den = d[0] * ey - d[1] * ex;
                double s = ((a[0] - y[0]) * d[1] - (a[1] - y[1]) * d[0]) / den;
                yn[0] = a[0] + s * ex; yn[1] = a[1] + s * ey; *segn = j;
            } else {   /* quadric (seg 0) or mesh (the triangle hit) */
                for (int j = 0; j < m; ++j) yn[j] = y[j] + hp->t * d[j];
                *segn = hp->seg;
            }
            found = 1;
            break;
        }
        *att_out = att; *qn_out = 0; *pick_out = 0;
        if (!found) { cnt->cap_hits++; return 0.0; }
        if (rel == REL_SAME) *Q *= 0.5;
        normal_at(g, m, yn, *segn, nn);
    }
    double dd[OR_MAX_DIM];
    for (int j = 0; j < m; ++j) dd[j] = yn[j] - y[j];
    double sg = dot(dd, nn, m) < 0 ? -1.0 : 1.0;
    *att_out = att; *qn_out = qn; *pick_out = pick;
    return (OR_PLANT == 5 ? 1 : qn) * sg;
}

static void one_sample(const or_problem *pr, const double *x, const or_query *q, uint64_t wi, uint32_t group,
                       double *Fk, double *Gk, uint32_t *trk, or_counters *cnt)
{
    const int m = pr->m, M = q->M, N = pr->N, K = q->estimator ? 2 : 1;
    const uint32_t w32 = (uint32_t)wi;
    const uint32_t inst = (q->instance & 0xFFFFFFu) << 8;
    int h[OR_MAX_M + 1];
    /* Theorem 2: H_0 ~ U{1..N}, H_i ~ |alpha|/||alpha||_1 (i >= 1). */
    words_t ws;
    words_init(&ws, q->seed, w32, q->schedule_mode ? 0xFFFFFFFFu : group, inst | 0u, 0);
    for (int i = 0; i <= M; ++i) {
        words_seek(&ws, (uint32_t)(i / 4));
        uint32_t v = 0;
        for (int j = 0; j <= i % 4; ++j) v = words_next(&ws);
        double u = unif(v);
        if (i == 0) { int t = (int)floor(u * N); h[0] = t < N ? t : N - 1; }
        else { int n = 0; while (n < N - 1 && !(u < pr->cdf[n])) ++n; h[i] = n; }
    }
    /* coefficient w_i ||alpha||_1^i prod_{m=1}^{i} sign(alpha_{h_m}) (Eq. woi_estimator) */
    double cS[OR_MAX_M + 1], S = 1;
    for (int i = 0; i <= M; ++i) {
        if (i > 0 || OR_PLANT == 1) S *= pr->r[h[i]].alpha < 0 ? -1.0 : 1.0;
        cS[i] = (i == M && OR_PLANT != 3 ? 0.5 : 1.0) * pow(pr->alpha_l1, i) * S;
    }
    for (int k = 0; k < K; ++k) {
        double F = 0, G[OR_MAX_DIM] = {0}, y[OR_MAX_DIM], Q, T = 1;
        int seg = 0, att = 0, ok;
        uint32_t *tr = trk ? trk + (size_t)k * (M + 1) : NULL;
        const uint32_t c2 = inst | ((uint32_t)k << 4) | 1u;
        words_t w;
        /* step 0: y_0 uniform on dOmega_{h0} (VR: on its half), Q = beta(y_0)/p_0 */
        words_init(&w, q->seed, w32, group, c2, 0);
        const region_t *g0 = &pr->r[h[0]];
        double meas = q->estimator ? g0->meas[k] : g0->area;
        if (meas == 0) { /* empty VR half: this walker contributes nothing */
            if (tr) for (int i = 0; i <= M; ++i) tr[i] = i ? 0u : trace_word(h[0], 0, 0, 0, 0, 0);
            Fk[k] = 0; for (int i = 0; i < m; ++i) Gk[k * m + i] = 0;
            continue;
        }
        int nw = q->estimator ? vr_words(pr, g0) : surf_words(g0, m), nb = (nw + 3) / 4;
        for (att = 0; att < OR_MAX_ATTEMPTS; ++att) {
            words_seek(&w, (uint32_t)(att * nb));
            ok = q->estimator ? vr_attempt(pr, h[0], k, &w, y, &seg) : surf_attempt(g0, m, &w, y, &seg);
            if (ok) break;
            cnt->rejections++;
        }
        if (att == OR_MAX_ATTEMPTS) cnt->cap_hits++;
        Q = beta_at(pr, h[0], y, seg) * meas;
        cnt->zero_dist += add_term(pr, x, y, cS[0] * Q * T, &F, G);
        cnt->walk_steps++;
        if (tr) tr[0] = trace_word(h[0], 0, 1, 0, 0, att);
        for (int i = 1; i <= M; ++i) {
            int rel = pr->rel[h[i - 1]][h[i]], qn, pick, segn;
            double yn[OR_MAX_DIM], nn[OR_MAX_DIM];
            words_init(&w, q->seed, w32, group, c2, (uint32_t)i);
            w.paired = m == 2;
            double tf = transition(pr, h[i - 1], h[i], &w, y, seg, yn, &segn, nn, &Q, &qn, &pick, &att, cnt);
            if (tf == 0) { if (tr) for (int j = i; j <= M; ++j) tr[j] = trace_word(h[j], rel, 0, 0, 0, att); break; }
            T *= tf;
            memcpy(y, yn, sizeof(double) * m); seg = segn;
            cnt->zero_dist += add_term(pr, x, y, cS[i] * Q * T, &F, G);
            cnt->walk_steps++;
            if (tr) tr[i] = trace_word(h[i], rel, qn, pick, tf < 0, att);
        }
        Fk[k] = N * F;
        for (int j = 0; j < m; ++j) Gk[k * m + j] = N * G[j];
    }
}

/* ---------------------------------------------------------------- naive WoI */
/* The naive estimator (Sec. 4.2, Eq. naive_woi_estimator): one observation is a Markov tree.
   Its roots are y_(h0), uniform on dOmega_{h0} for every h0 (p_0 of Eq. naive_woi_p0); every
   node (h0, ..., hi), i < M, has a child for every next interface h_{i+1}, drawn from the node
   by the transition of Eq. naive_woi_p (the branch is a Markov chain, reused by all its
   extensions, Sec. 4.2 "Reuse of Markov Chains").  The observation is
     sum over nodes of w_i (prod_{m=1}^{i} alpha_{h_m}) Q T Phi(x, y_(h0..hi)),
   Q and T of Eqs. naive_woi_Q and naive_woi_T, w_i = 1 - delta_{iM}/2.
   Random numbers: node (h0, ..., hi) draws from the counter (tree, point group,
   OR_NAIVE_TAG | id, step i), id = the base-(N+1) number with digits h0+1, ..., hi+1. */
#define OR_NAIVE_TAG 0x80000000u

static void naive_node(const or_problem *pr, const double *x, const or_query *q, uint32_t tree, uint32_t group,
                       int i, int h, uint32_t id, const double *y, int seg, double Q, double T, double A,
                       double *F, double *G, or_counters *cnt)
{
    const int M = q->M, N = pr->N;
    cnt->zero_dist += add_term(pr, x, y, (i == M && OR_PLANT != 3 ? 0.5 : 1.0) * A * Q * T, F, G);
    cnt->walk_steps++;
    if (i == M) return;
    for (int hn = 0; hn < N; ++hn) {
        const uint32_t idn = id * (uint32_t)(N + 1) + (uint32_t)(hn + 1);
        words_t w;
        words_init(&w, q->seed, tree, group, OR_NAIVE_TAG | idn, (uint32_t)(i + 1));
        double yn[OR_MAX_DIM], nn[OR_MAX_DIM], Qn = Q;
        int segn, qn, pick, att;
        double tf = transition(pr, h, hn, &w, y, seg, yn, &segn, nn, &Qn, &qn, &pick, &att, cnt);
        if (tf == 0) continue;   /* no hit within the attempt cap: this subtree contributes nothing */
        const double an = OR_PLANT == 6 ? fabs(pr->r[hn].alpha) : pr->r[hn].alpha;
        naive_node(pr, x, q, tree, group, i + 1, hn, idn, yn, segn, Qn, T * tf, A * an, F, G, cnt);
    }
}

static void naive_tree(const or_problem *pr, const double *x, const or_query *q, uint64_t ti, uint32_t group,
                       double *F, double *G, or_counters *cnt)
{
    const int m = pr->m;
    *F = 0;
    for (int d = 0; d < m; ++d) G[d] = 0;
    for (int h0 = 0; h0 < pr->N; ++h0) {
        const region_t *g0 = &pr->r[h0];
        const uint32_t id = (uint32_t)(h0 + 1);
        words_t w;
        words_init(&w, q->seed, (uint32_t)ti, group, OR_NAIVE_TAG | id, 0);
        double y[OR_MAX_DIM];
        int seg = 0, att, nb = (surf_words(g0, m) + 3) / 4;
        for (att = 0; att < OR_MAX_ATTEMPTS; ++att) {
            words_seek(&w, (uint32_t)(att * nb));
            if (surf_attempt(g0, m, &w, y, &seg)) break;
            cnt->rejections++;
        }
        if (att == OR_MAX_ATTEMPTS) cnt->cap_hits++;
        naive_node(pr, x, q, (uint32_t)ti, group, 0, h0, id, y, seg, beta_at(pr, h0, y, seg) * g0->area, 1.0, 1.0,
                   F, G, cnt);
    }
}

/* ---------------------------------------------------------------- quadrature helpers */
/* integral over S^{m-1} of f(u) by hyperspherical tensor quadrature:
   Gauss-Legendre in the m-2 polar angles, trapezoid in the azimuth. */
typedef double (*sfun_t)(const void *ctx, const double *u);

static double sphere_integral(int m, sfun_t f, const void *ctx, int n)
{
    if (m == 2) {
        int nt = 4 * n; double s = 0;
        for (int j = 0; j < nt; ++j) { double ph = 2 * OR_PI * j / nt, u[2] = {cos(ph), sin(ph)}; s += f(ctx, u); }
        return s * 2 * OR_PI / nt;
    }
    int np = m - 2, na = 2 * n;
    double *gx = malloc(sizeof(double) * n), *gw = malloc(sizeof(double) * n);
    gauss_legendre(n, gx, gw);
    int idx[OR_MAX_DIM] = {0};
    double total = 0;
    for (;;) {
        double u[OR_MAX_DIM], w = 1, sp = 1;
        for (int a = 0; a < np; ++a) {
            double phi = 0.5 * OR_PI * (gx[idx[a]] + 1);
            u[a] = sp * cos(phi);
            w *= 0.5 * OR_PI * gw[idx[a]] * pow(sin(phi), m - 2 - a);
            sp *= sin(phi);
        }
        for (int j = 0; j < na; ++j) {
            double ph = 2 * OR_PI * j / na;
            u[m - 2] = sp * cos(ph); u[m - 1] = sp * sin(ph);
            total += w * (2 * OR_PI / na) * f(ctx, u);
        }
        int a = 0;
        while (a < np && ++idx[a] == n) idx[a++] = 0;
        if (a == np) break;
    }
    free(gx); free(gw);
    return total;
}

typedef struct { const or_problem *pr; int h; int mode; } qctx_t; /* mode 0: area element, 1: b * area element */

static double surf_integrand(const void *vctx, const double *u)
{
    const qctx_t *c = vctx;
    const region_t *g = &c->pr->r[c->h];
    int m = c->pr->m;
    double y[OR_MAX_DIM], J;
    if (g->kind == OR_SPHERE) {
        for (int i = 0; i < m; ++i) y[i] = g->c[i] + g->R * u[i];
        J = pow(g->R, m - 1);
    } else {
        double uAu = 0;
        for (int i = 0; i < m; ++i) for (int j = 0; j < m; ++j) uAu += u[i] * g->A[i * m + j] * u[j];
        for (int i = 0; i < m; ++i) { double t = 0; for (int j = 0; j < m; ++j) t += g->L[i * m + j] * u[j]; y[i] = g->c[i] + t; }
        J = g->detL * sqrt(uAu);
    }
    if (c->mode == 0) return J;
    return J * data_b(g, m, y, 0);
}

static int quad_nodes(int m) { return m == 2 ? 2048 : (m == 3 ? 96 : (m == 4 ? 48 : (m == 5 ? 32 : 24))); }

/* ---- VR halves, m = 2: breakpoints of sign(beta) along arclength */
static double beta_s(const or_problem *pr, int h, double s)
{
    double y[2]; int seg;
    curve_at(&pr->r[h], s, y, &seg);
    return beta_at(pr, h, y, seg);
}

static int vr_prepare_2d(or_problem *pr, int h)
{
    region_t *g = &pr->r[h];
    int ngrid = g->kind == OR_POLYLINE ? 8 * g->nv : 8192;
    double *br = malloc(sizeof(double) * (ngrid + 1));
    if (!br) return OR_ENOMEM;
    int nb = 0;
    double sprev = 0, bprev = beta_s(pr, h, 0);
    g->class0 = bprev >= 0 ? 0 : 1;
    for (int j = 1; j <= ngrid; ++j) {
        double s = g->total * j / ngrid, b = j == ngrid ? beta_s(pr, h, 0) : beta_s(pr, h, s);
        if ((b >= 0) != (bprev >= 0)) {
            double lo = sprev, hi = s; int clo = bprev >= 0;
            for (int it = 0; it < 200 && hi - lo > 1e-16 * g->total; ++it) {
                double mid = 0.5 * (lo + hi);
                if ((beta_s(pr, h, mid) >= 0) == clo) lo = mid; else hi = mid;
            }
            if (j == ngrid && hi >= g->total) { /* crossing right at the wrap point */ }
            br[nb++] = 0.5 * (lo + hi);
        }
        sprev = s; bprev = b;
    }
    g->nbrk = nb; g->brk = br;
    g->meas[0] = g->meas[1] = 0;
    double start = 0; int c = g->class0;
    for (int p = 0; p <= nb; ++p) {
        double end = p < nb ? br[p] : g->total;
        g->meas[c] += end - start;
        start = end; c ^= 1;
    }
    return OR_OK;
}

/* ---- VR halves, m = 3: adaptive Simpson in the polar angle of the ellipsoid/sphere
   parametrisation u(theta, phi), exact phi-breakpoints on each ring. */
typedef struct { const or_problem *pr; int h; } vctx_t;

static void ring_point(const region_t *g, double th, double ph, double *y, double *J)
{
    double u[3] = {sin(th) * cos(ph), sin(th) * sin(ph), cos(th)};
    if (g->kind == OR_SPHERE) {
        for (int i = 0; i < 3; ++i) y[i] = g->c[i] + g->R * u[i];
        *J = g->R * g->R;
    } else {
        double uAu = 0;
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) uAu += u[i] * g->A[i * 3 + j] * u[j];
        for (int i = 0; i < 3; ++i) { double t = 0; for (int j = 0; j < 3; ++j) t += g->L[i * 3 + j] * u[j]; y[i] = g->c[i] + t; }
        /* dA_y = det(A^{-1/2}) |A^{1/2} u| dA_u for y = c + A^{-1/2} u */
        *J = g->detL * (OR_PLANT == 7 ? uAu : sqrt(uAu));
    }
}

static int ring_class(const or_problem *pr, int h, double th, double ph, double *J)
{
    double y[3];
    ring_point(&pr->r[h], th, ph, y, J);
    return beta_at(pr, h, y, 0) >= 0 ? 0 : 1;
}

/* measure of class 0 on the ring at polar angle th: integral of J dphi over {beta >= 0} */
static double ring_piece(const or_problem *pr, int h, double th, double s0, double s1)
{
    static const double gx[3] = {-0.7745966692414834, 0.0, 0.7745966692414834};
    static const double gw[3] = {5.0 / 9, 8.0 / 9, 5.0 / 9};
    double total = 0, J;
    for (int k = 0; k < 3; ++k) {
        ring_class(pr, h, th, 0.5 * (s0 + s1) + 0.5 * (s1 - s0) * gx[k], &J);
        total += 0.5 * (s1 - s0) * gw[k] * J;
    }
    return total;
}

static double ring_measure(const or_problem *pr, int h, double th, int want)
{
    const int n = 256;
    double total = 0, J;
    for (int j = 0; j < n; ++j) {
        double a = 2 * OR_PI * j / n, b = 2 * OR_PI * (j + 1) / n;
        int ca = ring_class(pr, h, th, a, &J), cb = ring_class(pr, h, th, b, &J);
        if (ca == cb) {
            if (ca == want) total += ring_piece(pr, h, th, a, b);
            continue;
        }
        double lo = a, hi = b;
        for (int it = 0; it < 100 && hi - lo > 1e-16; ++it) {
            double mid = 0.5 * (lo + hi);
            if (ring_class(pr, h, th, mid, &J) == ca) lo = mid; else hi = mid;
        }
        double r = 0.5 * (lo + hi);
        if (ca == want) total += ring_piece(pr, h, th, a, r);
        else total += ring_piece(pr, h, th, r, b);
    }
    return total;
}

static double vr_fun(const or_problem *pr, int h, int cls, double th) { return ring_measure(pr, h, th, cls) * sin(th); }

static double simpson_rec(const or_problem *pr, int h, int cls, double a, double b, double fa, double fm, double fb,
                          double whole, double tol, int depth)
{
    double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
    double flm = vr_fun(pr, h, cls, lm), frm = vr_fun(pr, h, cls, rm);
    double left = (m - a) / 6 * (fa + 4 * flm + fm), right = (b - m) / 6 * (fm + 4 * frm + fb);
    if (depth <= 0 || (depth < 40 && fabs(left + right - whole) <= 15 * tol))
        return left + right + (left + right - whole) / 15;
    return simpson_rec(pr, h, cls, a, m, fa, flm, fm, left, tol / 2, depth - 1) +
           simpson_rec(pr, h, cls, m, b, fm, frm, fb, right, tol / 2, depth - 1);
}

static double simpson_uniform_then_adaptive(const or_problem *pr, int h, int cls, double tol)
{
    const int nseg = 64; /* start from a uniform partition so no feature is missed */
    double total = 0;
    for (int j = 0; j < nseg; ++j) {
        double a = OR_PI * j / nseg, b = OR_PI * (j + 1) / nseg, m = 0.5 * (a + b);
        double fa = vr_fun(pr, h, cls, a), fm = vr_fun(pr, h, cls, m), fb = vr_fun(pr, h, cls, b);
        double whole = (b - a) / 6 * (fa + 4 * fm + fb);
        total += simpson_rec(pr, h, cls, a, b, fa, fm, fb, whole, tol / nseg, 30);
    }
    return total;
}

/* ---------------------------------------------------------------- create */
int or_problem_create(const or_problem_in *in, or_problem **out)
{
    if (!in || !out || in->dim < 2 || in->dim > OR_MAX_DIM || in->n_regions < 1 || in->n_regions > OR_MAX_REGIONS)
        return OR_EINVAL;
    or_problem *pr = calloc(1, sizeof(or_problem));
    if (!pr) return OR_ENOMEM;
    int m = pr->m = in->dim, N = pr->N = in->n_regions;
    pr->unit_area = 2 * pow(OR_PI, 0.5 * m) / tgamma(0.5 * m);
    for (int i = 0; i < N; ++i) {
        pr->parent[i] = in->parent[i]; pr->sigma[i] = in->sigma[i];
        if ((i == 0) != (in->parent[i] < 0) || in->parent[i] >= i) { or_problem_destroy(pr); return OR_EGEOM; }
    }
    for (int i = 0; i < N; ++i) {
        region_t *g = &pr->r[i];
        g->kind = in->shape_kind[i];
        for (int d = 0; d < m; ++d) g->c[d] = in->center[i * m + d];
        if (g->kind == OR_SPHERE) {
            g->R = in->radius[i];
            g->area = pr->unit_area * pow(g->R, m - 1);
        } else if (g->kind == OR_ELLIPSOID) {
            double e[OR_MAX_DIM], V[OR_MAX_DIM * OR_MAX_DIM];
            memcpy(g->A, in->A + (size_t)i * m * m, sizeof(double) * m * m);
            jacobi_eig(g->A, m, e, V);
            g->lam_max = 0; g->detL = 1;
            for (int d = 0; d < m; ++d) { if (e[d] <= 0) { or_problem_destroy(pr); return OR_EGEOM; } if (e[d] > g->lam_max) g->lam_max = e[d]; g->detL /= sqrt(e[d]); }
            for (int a = 0; a < m; ++a) for (int b = 0; b < m; ++b) {
                double s = 0; for (int d = 0; d < m; ++d) s += V[a * m + d] * V[b * m + d] / sqrt(e[d]);
                g->L[a * m + b] = s;
            }
        } else if (g->kind == OR_POLYLINE) {
            if (m != 2 || in->n_vertices[i] < 3) { or_problem_destroy(pr); return OR_EINVAL; }
            int nv = g->nv = in->n_vertices[i];
            g->v = malloc(sizeof(double) * 2 * nv); g->len = malloc(sizeof(double) * nv); g->cum = malloc(sizeof(double) * (nv + 1));
            if (!g->v || !g->len || !g->cum) { or_problem_destroy(pr); return OR_ENOMEM; }
            memcpy(g->v, in->vertices + 2 * in->vertex_offset[i], sizeof(double) * 2 * nv);
            g->cum[0] = 0;
            for (int j = 0; j < nv; ++j) {
                const double *a = g->v + 2 * j, *b = g->v + 2 * ((j + 1) % nv);
                double dx = b[0] - a[0], dy = b[1] - a[1];
                g->len[j] = sqrt(dx * dx + dy * dy);
                if (!(g->len[j] > 0)) { or_problem_destroy(pr); return OR_EGEOM; }
                g->cum[j + 1] = g->cum[j] + g->len[j];
            }
            g->total = g->cum[nv];
            g->area = g->total;
        } else if (g->kind == OR_MESH) {
            if (m != 3 || !in->n_triangles || in->n_vertices[i] < 4 || in->n_triangles[i] < 4) { or_problem_destroy(pr); return OR_EINVAL; }
            int nv = g->nv = in->n_vertices[i], nt = g->ntri = in->n_triangles[i];
            g->v = malloc(sizeof(double) * 3 * nv); g->tri = malloc(sizeof(int) * 3 * nt);
            g->tn = malloc(sizeof(double) * 3 * nt); g->cum = malloc(sizeof(double) * (nt + 1));
            if (!g->v || !g->tri || !g->tn || !g->cum) { or_problem_destroy(pr); return OR_ENOMEM; }
            memcpy(g->v, in->mesh_vertices + 3 * in->mesh_vertex_offset[i], sizeof(double) * 3 * nv);
            memcpy(g->tri, in->triangles + 3 * in->triangle_offset[i], sizeof(int) * 3 * nt);
            double vol = 0;
            g->cum[0] = 0;
            for (int j = 0; j < nt; ++j) {
                const int *t = g->tri + 3 * j;
                for (int k = 0; k < 3; ++k) if (t[k] < 0 || t[k] >= nv) { or_problem_destroy(pr); return OR_EINVAL; }
                const double *a = g->v + 3 * t[0], *b = g->v + 3 * t[1], *c = g->v + 3 * t[2];
                double e1[3], e2[3], cr[3];
                for (int k = 0; k < 3; ++k) { e1[k] = b[k] - a[k]; e2[k] = c[k] - a[k]; }
                cr[0] = e1[1] * e2[2] - e1[2] * e2[1]; cr[1] = e1[2] * e2[0] - e1[0] * e2[2]; cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
                double l = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
                if (!(l > 0)) { or_problem_destroy(pr); return OR_EGEOM; }
                for (int k = 0; k < 3; ++k) g->tn[3 * j + k] = cr[k] / l;
                g->cum[j + 1] = g->cum[j] + 0.5 * l;
                vol += a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) + a[2] * (b[0] * c[1] - b[1] * c[0]);
            }
            if (!(vol > 0)) { or_problem_destroy(pr); return OR_EGEOM; }   /* normals must point outward */
            g->total = g->area = g->cum[nt];
        } else { or_problem_destroy(pr); return OR_EINVAL; }
        if (g->kind == OR_SPHERE && m == 2) g->total = 2 * OR_PI * g->R;
        /* data */
        g->dkind = in->data_kind[i]; g->nt = in->n_terms[i];
        for (int d = 0; d < m; ++d) g->dc[d] = in->data_center[i * m + d];
        int ncoef = g->dkind == OR_DATA_FOURIER2D ? 2 * g->nt + 1 : g->dkind == OR_DATA_ZERO ? 0 : g->dkind == OR_DATA_SOURCE_FLUX ? 1 : g->dkind == OR_DATA_FIELD_FLUX ? m : g->nt;
        if (g->dkind == OR_DATA_FOURIER2D && m != 2) { or_problem_destroy(pr); return OR_EINVAL; }
        g->coef = malloc(sizeof(double) * (ncoef + 1));
        if (ncoef) memcpy(g->coef, in->coef + in->coef_offset[i], sizeof(double) * ncoef);
        if (g->dkind == OR_DATA_DIRPOLY) {
            g->exps = malloc((size_t)g->nt * m + 1);
            memcpy(g->exps, in->exps + (size_t)in->coef_offset[i] * m, (size_t)g->nt * m);
        }
    }
    /* ellipsoid surface measure: det(A)^{-1/2} * integral over S^{m-1} of |A^{1/2} u| */
    for (int i = 0; i < N; ++i) if (pr->r[i].kind == OR_ELLIPSOID) {
        qctx_t c = {pr, i, 0};
        pr->r[i].area = sphere_integral(m, surf_integrand, &c, quad_nodes(m));
        if (m == 2) pr->r[i].total = pr->r[i].area;
    }
    /* alpha_i, beta scale s_i (Eq. unit_coeff_charge_density_sys) */
    pr->alpha_l1 = 0;
    for (int i = 0; i < N; ++i) {
        region_t *g = &pr->r[i];
        if (i == 0) { g->alpha = 2; g->s = 2 / pr->sigma[0]; }
        else {
            double sp = pr->sigma[pr->parent[i]], si = pr->sigma[i];
            g->alpha = 2 * (si - sp) / (sp + si); g->s = -2 / (sp + si);
        }
        pr->alpha_l1 += fabs(g->alpha);
    }
    double acc = 0;
    for (int i = 0; i < N; ++i) { acc += fabs(pr->r[i].alpha); pr->cdf[i] = acc / pr->alpha_l1; }
    /* relation of consecutive scheduled interfaces */
    for (int a = 0; a < N; ++a) for (int b = 0; b < N; ++b) {
        int rel = REL_OTHER;
        if (a == b) rel = REL_SAME;
        else { for (int p = pr->parent[a]; p >= 0; p = pr->parent[p]) if (p == b) { rel = REL_DESC; break; } }
        pr->rel[a][b] = rel;
    }
    /* flux integrals of b_i */
    for (int i = 0; i < N; ++i) {
        region_t *g = &pr->r[i];
        if (g->kind == OR_POLYLINE) {
            static const double gx[4] = {-0.8611363115940526, -0.3399810435848563, 0.3399810435848563, 0.8611363115940526};
            static const double gw[4] = {0.3478548451374538, 0.6521451548625461, 0.6521451548625461, 0.3478548451374538};
            double s = 0;
            for (int j = 0; j < g->nv; ++j) for (int k = 0; k < 4; ++k) {
                const double *a = g->v + 2 * j, *b = g->v + 2 * ((j + 1) % g->nv);
                double f = 0.5 * (gx[k] + 1), y[2] = {a[0] + f * (b[0] - a[0]), a[1] + f * (b[1] - a[1])};
                s += 0.5 * gw[k] * g->len[j] * data_b(g, m, y, j);
            }
            g->flux = s;
        } else if (g->kind == OR_MESH) {
            /* edge-midpoint rule per triangle (exact for quadratics) */
            double s = 0;
            for (int j = 0; j < g->ntri; ++j) {
                const int *t = g->tri + 3 * j;
                const double *a = g->v + 3 * t[0], *b = g->v + 3 * t[1], *c = g->v + 3 * t[2];
                double ar = g->cum[j + 1] - g->cum[j];
                for (int k = 0; k < 3; ++k) {
                    const double *p0 = k == 0 ? a : k == 1 ? b : c, *p1 = k == 0 ? b : k == 1 ? c : a;
                    double y[3] = {0.5 * (p0[0] + p1[0]), 0.5 * (p0[1] + p1[1]), 0.5 * (p0[2] + p1[2])};
                    s += ar / 3 * data_b(g, m, y, j);
                }
            }
            g->flux = s;
        } else {
            qctx_t c = {pr, i, 1};
            g->flux = sphere_integral(m, surf_integrand, &c, quad_nodes(m));
        }
    }
    /* VR halves */
    pr->vr_ok = m <= 3;
    for (int i = 0; i < N; ++i) if (pr->r[i].kind == OR_MESH) pr->vr_ok = 0;   /* no VR halves on meshes */
    /* 2D halves are arclength intervals, built for circles and polylines only */
    for (int i = 0; i < N; ++i) if (m == 2 && pr->r[i].kind == OR_ELLIPSOID) pr->vr_ok = 0;
    for (int i = 0; i < N; ++i) {
        region_t *g = &pr->r[i];
        if (!pr->vr_ok) {
            g->meas[0] = g->meas[1] = NAN;
        } else if (m == 2) {
            int rc = vr_prepare_2d(pr, i);
            if (rc) { or_problem_destroy(pr); return rc; }
        } else if (m == 3) {
            for (int cls = 0; cls < 2; ++cls) {
                g->meas[cls] = simpson_uniform_then_adaptive(pr, i, cls, 1e-11 * g->area);
            }
        } else {
            g->meas[0] = g->meas[1] = NAN;
        }
    }
    *out = pr;
    return OR_OK;
}

void or_problem_destroy(or_problem *pr)
{
    if (!pr) return;
    for (int i = 0; i < OR_MAX_REGIONS; ++i) {
        region_t *g = &pr->r[i];
        free(g->v); free(g->len); free(g->cum); free(g->coef); free(g->exps); free(g->brk); free(g->tri); free(g->tn);
    }
    free(pr);
}

int or_problem_info(const or_problem *pr, double *alpha, double *beta_scale, double *area, double *area_plus,
                    double *area_minus, double *flux, double *alpha_l1)
{
    for (int i = 0; i < pr->N; ++i) {
        const region_t *g = &pr->r[i];
        if (alpha) alpha[i] = g->alpha;
        if (beta_scale) beta_scale[i] = g->s;
        if (area) area[i] = g->area;
        if (area_plus) area_plus[i] = g->meas[0];
        if (area_minus) area_minus[i] = g->meas[1];
        if (flux) flux[i] = g->flux;
    }
    if (alpha_l1) *alpha_l1 = pr->alpha_l1;
    return OR_OK;
}

/* ---------------------------------------------------------------- surrogate training points */
/* Training data of the neural-network surrogate (Sec. 5, Eq. MLP_loss).  Interior points: the
   cell centres x_d = lo_d + (i_d + 1/2) (hi_d - lo_d) / n of an n^m grid over the bounding box of
   dOmega (row-major, last coordinate fastest) that lie strictly inside dOmega and, when
   margin > 0, farther than `margin` from every interface (sphere: ||x - c| - R|; ellipsoid: the
   first-order level-set distance |q - 1| / |grad q|, q = (x - c)^T A (x - c); polyline: the
   distance to its nearest segment).  Boundary points: uniform in the angular coordinates of
   dOmega -- 2D: theta_k = 2 pi k / n_bc, the point of dOmega in direction theta_k from its centre
   (circle) or from the vertex mean (polyline: the farthest crossing of that ray); 3D: polar
   angles pi (i + 1/2) / n_bc and azimuths pi j / n_bc (2 n_bc of them) mapped through the
   sphere or ellipsoid parametrisation -- with the outward unit normal and the normal-derivative
   target b_1 / sigma_1 of the Neumann condition sigma_1 d_n u = b_1 (Eq. interface_problem). */
static int training_box(const or_problem *pr, double *lo, double *hi)
{
    const region_t *g = &pr->r[0];
    const int m = pr->m;
    if (g->kind == OR_SPHERE || g->kind == OR_ELLIPSOID) {
        for (int d = 0; d < m; ++d) {
            double half = g->R;
            if (g->kind == OR_ELLIPSOID) {   /* extent along axis d: sqrt((A^-1)_dd), A^-1 = L L */
                double s2 = 0;
                for (int j = 0; j < m; ++j) s2 += g->L[d * m + j] * g->L[d * m + j];
                half = sqrt(s2);
            }
            lo[d] = g->c[d] - half; hi[d] = g->c[d] + half;
        }
        return OR_OK;
    }
    if (g->kind == OR_POLYLINE) {
        lo[0] = hi[0] = g->v[0]; lo[1] = hi[1] = g->v[1];
        for (int j = 1; j < g->nv; ++j)
            for (int d = 0; d < 2; ++d) {
                if (g->v[2 * j + d] < lo[d]) lo[d] = g->v[2 * j + d];
                if (g->v[2 * j + d] > hi[d]) hi[d] = g->v[2 * j + d];
            }
        return OR_OK;
    }
    return OR_EUNSUP;
}

static int inside_region(const region_t *g, int m, const double *x)
{
    if (g->kind == OR_SPHERE) {
        double r2 = 0; for (int i = 0; i < m; ++i) r2 += (x[i] - g->c[i]) * (x[i] - g->c[i]);
        return r2 < g->R * g->R;
    }
    if (g->kind == OR_ELLIPSOID) {
        double q = 0;
        for (int i = 0; i < m; ++i) for (int j = 0; j < m; ++j) q += (x[i] - g->c[i]) * g->A[i * m + j] * (x[j] - g->c[j]);
        return q < 1.0;
    }
    /* polyline: crossing number of the ray x + t e_1, t > 0 */
    int in = 0;
    for (int j = 0; j < g->nv; ++j) {
        const double *a = g->v + 2 * j, *b = g->v + 2 * ((j + 1) % g->nv);
        if ((a[1] > x[1]) != (b[1] > x[1])) {
            double xi = a[0] + (x[1] - a[1]) / (b[1] - a[1]) * (b[0] - a[0]);
            if (x[0] < xi) in = !in;
        }
    }
    return in;
}

static double distance_to_region(const region_t *g, int m, const double *x)
{
    if (g->kind == OR_SPHERE) {
        double r2 = 0; for (int i = 0; i < m; ++i) r2 += (x[i] - g->c[i]) * (x[i] - g->c[i]);
        return fabs(sqrt(r2) - g->R);
    }
    if (g->kind == OR_ELLIPSOID) {
        double q = 0, gn = 0;
        for (int i = 0; i < m; ++i) {
            double t = 0; for (int j = 0; j < m; ++j) t += g->A[i * m + j] * (x[j] - g->c[j]);
            q += (x[i] - g->c[i]) * t; gn += t * t;
        }
        return fabs(q - 1.0) / (2.0 * sqrt(gn));
    }
    double best = INFINITY;
    for (int j = 0; j < g->nv; ++j) {
        const double *a = g->v + 2 * j, *b = g->v + 2 * ((j + 1) % g->nv);
        double ex = b[0] - a[0], ey = b[1] - a[1], l2 = ex * ex + ey * ey;
        double s = ((x[0] - a[0]) * ex + (x[1] - a[1]) * ey) / l2;
        s = s < 0 ? 0 : (s > 1 ? 1 : s);
        double dx = x[0] - (a[0] + s * ex), dy = x[1] - (a[1] + s * ey), dd = sqrt(dx * dx + dy * dy);
        if (dd < best) best = dd;
    }
    return best;
}

int or_training_points(const or_problem *pr, int grid_n, double margin, int bc_n, double *interior, int64_t cap,
                       int64_t *n_interior, double *bc_points, double *bc_normals, double *bc_flux, int64_t *n_bc)
{
    const int m = pr->m;
    if (grid_n < 1 || bc_n < 0 || (m != 2 && m != 3 && bc_n > 0)) return OR_EINVAL;
    for (int i = 0; i < pr->N; ++i) if (pr->r[i].kind == OR_MESH) return OR_EUNSUP;
    double lo[OR_MAX_DIM], hi[OR_MAX_DIM], step[OR_MAX_DIM];
    int rc = training_box(pr, lo, hi);
    if (rc) return rc;
    for (int d = 0; d < m; ++d) step[d] = (hi[d] - lo[d]) / grid_n;
    uint64_t nodes = 1;
    for (int d = 0; d < m; ++d) nodes *= (uint64_t)grid_n;
    int64_t count = 0;
    for (uint64_t k = 0; k < nodes; ++k) {
        double x[OR_MAX_DIM];
        uint64_t r = k;
        for (int d = m - 1; d >= 0; --d) { x[d] = lo[d] + ((double)(r % (uint64_t)grid_n) + 0.5) * step[d]; r /= (uint64_t)grid_n; }
        if (!inside_region(&pr->r[0], m, x)) continue;
        int keep = 1;
        if (margin > 0)
            for (int i = 0; i < pr->N && keep; ++i) keep = distance_to_region(&pr->r[i], m, x) > margin;
        if (!keep) continue;
        if (count < cap) memcpy(interior + (size_t)count * m, x, sizeof(double) * m);
        ++count;
    }
    *n_interior = count;
    /* boundary */
    const region_t *g = &pr->r[0];
    int64_t nb = m == 2 ? bc_n : 2 * (int64_t)bc_n * bc_n;
    if (n_bc) *n_bc = nb;
    if (!bc_points || bc_n == 0) return OR_OK;
    const double sigma1 = pr->sigma[0];
    for (int64_t k = 0; k < nb; ++k) {
        double y[3] = {0, 0, 0}, n[3] = {0, 0, 0};
        int seg = 0;
        if (m == 2) {
            const double th = 2 * OR_PI * (double)k / bc_n, d[2] = {cos(th), sin(th)};
            if (g->kind == OR_SPHERE) {
                for (int i = 0; i < 2; ++i) y[i] = g->c[i] + g->R * d[i];
            } else {   /* polyline: farthest crossing of the ray from the vertex mean */
                double z[2] = {0, 0}, tbest = -1;
                for (int j = 0; j < g->nv; ++j) { z[0] += g->v[2 * j] / g->nv; z[1] += g->v[2 * j + 1] / g->nv; }
                for (int j = 0; j < g->nv; ++j) {
                    const double *a = g->v + 2 * j, *b = g->v + 2 * ((j + 1) % g->nv);
                    double ex = b[0] - a[0], ey = b[1] - a[1], den = d[0] * ey - d[1] * ex;
                    if (den == 0) continue;
                    double t = ((a[0] - z[0]) * ey - (a[1] - z[1]) * ex) / den;
                    double sp = ((a[0] - z[0]) * d[1] - (a[1] - z[1]) * d[0]) / den;
                    if (sp < 0 || sp >= 1 || !(t > 0) || t <= tbest) continue;
                    tbest = t; seg = j;
                    y[0] = a[0] + sp * ex; y[1] = a[1] + sp * ey;
                }
                if (tbest < 0) return OR_EGEOM;
            }
        } else {
            const int64_t i = k / (2 * bc_n), j = k % (2 * bc_n);
            const double th = OR_PI * ((double)i + 0.5) / bc_n, ph = OR_PI * (double)j / bc_n;
            const double u[3] = {sin(th) * cos(ph), sin(th) * sin(ph), cos(th)};
            if (g->kind == OR_SPHERE) {
                for (int a = 0; a < 3; ++a) y[a] = g->c[a] + g->R * u[a];
            } else {
                for (int a = 0; a < 3; ++a) { double t = 0; for (int b = 0; b < 3; ++b) t += g->L[a * 3 + b] * u[b]; y[a] = g->c[a] + t; }
            }
        }
        normal_at(g, m, y, seg, n);
        for (int a = 0; a < m; ++a) { bc_points[k * m + a] = y[a]; bc_normals[k * m + a] = n[a]; }
        bc_flux[k] = data_b(g, m, y, seg) / sigma1;
    }
    return OR_OK;
}

int or_sample_surface(const or_problem *pr, int h, uint64_t seed, uint64_t n, double *y)
{
    if (h < 0 || h >= pr->N) return OR_EINVAL;
    const region_t *g = &pr->r[h];
    int nb = (surf_words(g, pr->m) + 3) / 4;
    for (uint64_t j = 0; j < n; ++j) {
        words_t w; int seg;
        words_init(&w, seed, (uint32_t)j, 0, 1u, 0);
        for (int att = 0; att < OR_MAX_ATTEMPTS; ++att) {
            words_seek(&w, (uint32_t)(att * nb));
            if (surf_attempt(g, pr->m, &w, y + j * pr->m, &seg)) break;
        }
    }
    return OR_OK;
}

/* ---------------------------------------------------------------- drivers */
typedef struct {
    const or_problem *pr; const double *x; const or_query *q;
    int64_t p0, p1; uint64_t n;
    double *F, *G; uint32_t *trace;            /* trace mode */
    double *mean, *se, *grad, *grad_se;        /* estimate mode */
    const uint32_t *groups;                    /* explicit stream group per point, or NULL */
    or_counters cnt;
} job_t;

static uint32_t group_of(const job_t *j, int64_t p, int B) { return j->groups ? j->groups[p] : (uint32_t)(p / B); }

static uint64_t n_samples_of(const or_query *q) { return q->estimator == 1 ? q->walks / 2 : q->walks; }
static uint64_t first_sample(const or_query *q) { return q->estimator == 1 ? q->walk_offset / 2 : q->walk_offset; }

/* one observation: walker values (K = 2 for VR) or, for the naive estimator, one tree's value */
static void observation(const or_problem *pr, const double *x, const or_query *q, uint64_t s, uint32_t group,
                        double *Fk, double *Gk, uint32_t *trk, or_counters *cnt)
{
    if (q->estimator == 2) naive_tree(pr, x, q, s, group, Fk, Gk, cnt);
    else one_sample(pr, x, q, s, group, Fk, Gk, trk, cnt);
}

static void *trace_job(void *arg)
{
    job_t *j = arg;
    const or_problem *pr = j->pr;
    int m = pr->m, K = j->q->estimator == 1 ? 2 : 1, M = j->q->M;
    int B = j->q->batch_share > 0 ? j->q->batch_share : 1;
    for (int64_t p = j->p0; p < j->p1; ++p)
        for (uint64_t s = 0; s < j->n; ++s) {
            size_t idx = (size_t)p * j->n + s;
            double Fk[2], Gk[2 * OR_MAX_DIM];
            observation(pr, j->x + p * m, j->q, first_sample(j->q) + s, group_of(j, p, B), Fk, Gk,
                        j->trace ? j->trace + idx * K * (M + 1) : NULL, &j->cnt);
            for (int k = 0; k < K; ++k) {
                j->F[idx * K + k] = Fk[k];
                if (j->G) for (int d = 0; d < m; ++d) j->G[(idx * K + k) * m + d] = Gk[k * m + d];
            }
        }
    return NULL;
}

static void *estimate_job(void *arg)
{
    job_t *j = arg;
    const or_problem *pr = j->pr;
    int m = pr->m, K = j->q->estimator == 1 ? 2 : 1;
    int B = j->q->batch_share > 0 ? j->q->batch_share : 1;
    uint64_t n = n_samples_of(j->q);
    for (int64_t p = j->p0; p < j->p1; ++p) {
        double mu = 0, m2 = 0, gmu[OR_MAX_DIM] = {0}, gm2[OR_MAX_DIM] = {0};
        for (uint64_t s = 0; s < n; ++s) {
            double Fk[2], Gk[2 * OR_MAX_DIM];
            observation(pr, j->x + p * m, j->q, first_sample(j->q) + s, group_of(j, p, B), Fk, Gk, NULL, &j->cnt);
            double f = 0, g[OR_MAX_DIM] = {0};
            for (int k = 0; k < K; ++k) { f += Fk[k]; for (int d = 0; d < m; ++d) g[d] += Gk[k * m + d]; }
            /* Welford, as in Alg. 1 */
            double dl = f - mu; mu += dl / (double)(s + 1); m2 += dl * (f - mu);
            for (int d = 0; d < m; ++d) { double e = g[d] - gmu[d]; gmu[d] += e / (double)(s + 1); gm2[d] += e * (g[d] - gmu[d]); }
        }
        j->mean[p] = mu;
        j->se[p] = n > 1 ? sqrt(m2 / (double)(n - 1) / (double)n) : NAN;
        for (int d = 0; d < m; ++d) {
            if (j->grad) j->grad[p * m + d] = gmu[d];
            if (j->grad_se) j->grad_se[p * m + d] = n > 1 ? sqrt(gm2[d] / (double)(n - 1) / (double)n) : NAN;
        }
        j->cnt.walks += n * K;
    }
    return NULL;
}

static int check_query(const or_problem *pr, const or_query *q)
{
    if (!q || q->M < 0 || q->M > OR_MAX_M || q->walks == 0 || q->estimator < 0 || q->estimator > 2) return OR_EINVAL;
    if (q->estimator == 1 && (!pr->vr_ok || (q->walks & 1) || (q->walk_offset & 1))) return pr->vr_ok ? OR_EINVAL : OR_EUNSUP;
    if (q->estimator == 2) {   /* node ids (N+1)^(M+1) below 2^31; no instance; one tree stream per point */
        double ids = pow(pr->N + 1.0, q->M + 1.0);
        if (ids > 2147483648.0 || q->instance != 0 || q->batch_share > 1) return OR_EINVAL;
    }
    return OR_OK;
}

static int run_jobs(const or_problem *pr, const double *x, int64_t P, const or_query *q, int nth, job_t *tmpl,
                    void *(*fn)(void *), or_counters *cnt)
{
    if (nth < 1) nth = 1;
    if (nth > 256) nth = 256;
    if (nth > P) nth = (int)(P > 0 ? P : 1);
    job_t jobs[256];
    pthread_t th[256];
    for (int t = 0; t < nth; ++t) {
        jobs[t] = *tmpl;
        jobs[t].pr = pr; jobs[t].x = x; jobs[t].q = q;
        jobs[t].p0 = P * t / nth; jobs[t].p1 = P * (t + 1) / nth;
        memset(&jobs[t].cnt, 0, sizeof(or_counters));
        if (nth > 1) pthread_create(&th[t], NULL, fn, &jobs[t]);
    }
    if (nth == 1) fn(&jobs[0]);
    else for (int t = 0; t < nth; ++t) pthread_join(th[t], NULL);
    if (cnt) {
        memset(cnt, 0, sizeof(*cnt));
        for (int t = 0; t < nth; ++t) {
            cnt->walks += jobs[t].cnt.walks; cnt->walk_steps += jobs[t].cnt.walk_steps;
            cnt->redraws += jobs[t].cnt.redraws; cnt->rejections += jobs[t].cnt.rejections;
            cnt->cap_hits += jobs[t].cnt.cap_hits; cnt->zero_dist += jobs[t].cnt.zero_dist;
        }
    }
    return OR_OK;
}

int or_trace(const or_problem *pr, const double *x, int64_t P, const or_query *q, uint64_t n, int nth,
             double *F, double *G, uint32_t *trace)
{
    int rc = check_query(pr, q);
    if (rc) return rc;
    job_t t; memset(&t, 0, sizeof t);
    t.n = n; t.F = F; t.G = G; t.trace = trace;
    return run_jobs(pr, x, P, q, nth, &t, trace_job, NULL);
}

int or_estimate(const or_problem *pr, const double *x, int64_t P, const or_query *q, int nth,
                double *mean, double *se, double *grad, double *grad_se, or_counters *cnt)
{
    return or_estimate_groups(pr, x, P, q, NULL, nth, mean, se, grad, grad_se, cnt);
}

int or_estimate_groups(const or_problem *pr, const double *x, int64_t P, const or_query *q, const uint32_t *groups,
                       int nth, double *mean, double *se, double *grad, double *grad_se, or_counters *cnt)
{
    int rc = check_query(pr, q);
    if (rc) return rc;
    job_t t; memset(&t, 0, sizeof t);
    t.mean = mean; t.se = se; t.grad = grad; t.grad_se = grad_se; t.groups = groups;
    return run_jobs(pr, x, P, q, nth, &t, estimate_job, cnt);
}
