/*
 * woi_oracle.h -- slow FP64 CPU oracle for the Walk-on-Interfaces estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header,
 * table or constant with the GPU library; both implement Philox4x32-10 from its
 * published definition (Salmon, Moraes, Dror, Shaw, SC'11).
 *
 * Paper: Ding & Stinchcombe, "Walk-on-Interfaces", arXiv 2508.16767.
 *   problem            Sec. 1, Eq. (interface_problem)
 *   alpha_i, beta_i    Sec. 3, Eq. (unit_coeff_charge_density_sys)
 *   transition pdfs    Sec. 4.2.1, Eqs. (naive_woi_p0), (naive_woi_p)
 *   Q / T factors      Sec. 4.2.2, Eqs. (naive_woi_Q), (naive_woi_T)
 *   naive estimator    Sec. 4.2.2-4.2.4, Eq. (naive_woi_estimator): Markov trees
 *   schedules          Sec. 4.3.1, Theorem 2, Eq. (scheduled_interface_pdf)
 *   estimator          Eq. (woi_estimator), Algorithms 1 and 2
 *   variance reduction Sec. 4.4, Eq. (variance_reduced_woi_estimator), Alg. 3
 *   gradient           Sec. 4.5, Eqs. (naive_woi_grad_estimator),
 *                      (variance_reduced_woi_grad_estimator)
 *
 * Flat problem arrays (N regions, dimension m); region 0 is the root, whose
 * interface is the outer boundary.  All arrays are read during create only.
 */
#ifndef WOI_ORACLE_H
#define WOI_ORACLE_H
#include <stdint.h>

#define OR_MAX_DIM 8
#define OR_MAX_REGIONS 64
#define OR_MAX_M 64

enum { OR_SPHERE = 0, OR_ELLIPSOID = 1, OR_POLYLINE = 2, OR_MESH = 3 };
enum { OR_DATA_ZERO = 0, OR_DATA_FOURIER2D = 1, OR_DATA_DIRPOLY = 2, OR_DATA_SOURCE_FLUX = 3, OR_DATA_FIELD_FLUX = 4 };
enum { OR_OK = 0, OR_EINVAL = -1, OR_EGEOM = -2, OR_EINCOMPAT = -3, OR_EUNSUP = -4, OR_ENOMEM = -6 };

typedef struct {
    int dim, n_regions;
    const int *parent;            /* [N], parent[0] = -1, parent[i] < i            */
    const double *sigma;          /* [N]                                             */
    const int *shape_kind;        /* [N]                                             */
    const double *center;         /* [N*dim] sphere / ellipsoid centre              */
    const double *radius;         /* [N] sphere radius                              */
    const double *A;              /* [N*dim*dim] ellipsoid matrix, (y-c)^T A (y-c)=1 */
    const int *n_vertices;        /* [N] polyline vertex count (0 otherwise)        */
    const int64_t *vertex_offset; /* [N] offset (in vertices) into vertices[]       */
    const double *vertices;       /* [sum n_vertices * 2], counter-clockwise         */
    const int *data_kind;         /* [N]                                             */
    const double *data_center;    /* [N*dim] expansion centre / source position    */
    const int *n_terms;           /* [N]                                             */
    const int64_t *coef_offset;   /* [N]                                             */
    const double *coef;           /* FOURIER2D: a0,a1,c1,..,aK,cK; DIRPOLY: one per term; SOURCE_FLUX: kappa; FIELD_FLUX: g[dim] */
    const unsigned char *exps;    /* DIRPOLY exponents, [sum n_terms * dim] (offset coef_offset*dim) */
    /* MESH (dim 3): closed triangle mesh, n_vertices[i] vertices and n_triangles[i] triangles,
       each triangle's vertices counter-clockwise seen from outside (outward normal
       (b - a) x (c - a)); indices are local to the mesh */
    const int *n_triangles;       /* [N] (0 otherwise)                               */
    const int64_t *mesh_vertex_offset; /* [N] offset (in vertices) into mesh_vertices[] */
    const double *mesh_vertices;  /* [sum * 3]                                       */
    const int64_t *triangle_offset;    /* [N] offset (in triangles) into triangles[]   */
    const int *triangles;         /* [sum * 3]                                       */
} or_problem_in;

typedef struct {
    uint64_t seed;
    uint64_t walks;        /* walkers per point; VR uses walks/2 two-walker samples  */
    uint64_t walk_offset;  /* first walker index (even for VR)                         */
    int M;                 /* truncation: steps 0..M                                  */
    int estimator;         /* 0 plain (Alg. 2), 1 variance reduced (Alg. 3), 2 naive
                              Markov trees (Sec. 4.2; walks = trees, instance 0,
                              batch_share 1, (N+1)^(M+1) <= 2^31)                     */
    int schedule_mode;     /* 0: schedule keyed by (walk, point group), 1: by walk    */
    int batch_share;       /* B >= 1: points p with equal p/B share trajectories      */
    uint32_t instance;     /* instance id (< 2^24) mixed into every counter           */
} or_query;

typedef struct {
    uint64_t walks, walk_steps, redraws, rejections, cap_hits, zero_dist;
} or_counters;

typedef struct or_problem or_problem;

int  or_problem_create(const or_problem_in *in, or_problem **out);
void or_problem_destroy(or_problem *p);
/* alpha, beta scale s_i, |dOmega_i|, |dOmega_i^+|, |dOmega_i^-| (VR, NaN if unsupported),
   integral of b_i over dOmega_i, and ||alpha||_1 */
int  or_problem_info(const or_problem *p, double *alpha, double *beta_scale, double *area,
                     double *area_plus, double *area_minus, double *flux, double *alpha_l1);
/* one sample of the point-x estimator per walk: F[(p*n + j)*K + k] is walker k's value
   (times N), G the matching gradient, trace the decision words [.. *(M+1) + i]. */
int  or_trace(const or_problem *p, const double *x, int64_t P, const or_query *q,
              uint64_t n_samples, int n_threads, double *F, double *G, uint32_t *trace);
/* mean, standard error, gradient and its standard error per point (Alg. 1 with one
   schedule per walk; Welford accumulation). */
int  or_estimate(const or_problem *p, const double *x, int64_t P, const or_query *q, int n_threads,
                 double *mean, double *se, double *grad, double *grad_se, or_counters *cnt);
/* as or_estimate, with an explicit random-stream group per point (groups[p]) instead of p / B */
int  or_estimate_groups(const or_problem *p, const double *x, int64_t P, const or_query *q, const uint32_t *groups,
                        int n_threads, double *mean, double *se, double *grad, double *grad_se, or_counters *cnt);
/* Philox4x32-10 block, exported for the known-answer test. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Training data of the neural-network surrogate (Sec. 5, Eq. MLP_loss): the interior grid nodes
   inside dOmega clear of the interfaces by `margin` (count in *n_interior, the first `cap`
   written), and 2D n_bc / 3D 2 n_bc^2 boundary points with outward normals and b_1 / sigma_1. */
int  or_training_points(const or_problem *p, int grid_n, double margin, int bc_n, double *interior, int64_t cap,
                        int64_t *n_interior, double *bc_points, double *bc_normals, double *bc_flux, int64_t *n_bc);
/* Uniform point on interface `region` from one attempt's words (for histogram tests). */
int  or_sample_surface(const or_problem *p, int region, uint64_t seed, uint64_t n, double *y);

#endif
