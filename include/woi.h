/*
 * woi.h -- C ABI of the MI355X (gfx950) Walk-on-Interfaces library.
 *
 * Walk-on-Interfaces (WoI) is a Monte Carlo estimator of u(x) and grad u(x) for the
 * Neumann elliptic interface problem div(sigma grad u) = 0 with piecewise-constant
 * sigma over a tree of nested regions and flux-jump data b_i on every interface
 * (Ding & Stinchcombe, arXiv 2508.16767, Sec. 1, Eq. interface_problem).
 *
 * Conventions shared by every entry point
 *   - All calls return woi_status (0 = WOI_OK, negative = error).  On error, a
 *     thread-local message is available from woi_last_error(); outputs are then
 *     unspecified.
 *   - Point and output arrays are DEVICE pointers (HIP global memory on the current
 *     device) owned by the caller; the library never frees or retains them.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream) and is
 *     stream-ordered; calls return once the work is enqueued.
 *   - Problems are immutable after creation and may be shared across threads and
 *     streams of the device they were created on.
 *   - Region 0 is the root: its interface is the outer boundary dOmega (Neumann data
 *     b_1 in the paper's 1-based numbering); every other region i has parent[i] < i.
 *   - Deliberately absent: host-array outputs (results stay in device memory; copying them
 *     to the host is the caller's, on its own stream) and cancellation (every call only
 *     enqueues bounded work; a caller stops by enqueuing no more).
 */
#ifndef WOI_H
#define WOI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WOI_MAX_DIM 8
#define WOI_MAX_REGIONS 32
#define WOI_MAX_M 32
#define WOI_COUNTERS 9
#define WOI_NAIVE_MAX_LEAVES (1 << 24)

typedef enum {
    WOI_OK = 0,
    WOI_E_INVALID_ARG = -1,   /* bad pointer, size, dimension, query field            */
    WOI_E_GEOMETRY = -2,      /* not a tree, degenerate or non-nested shapes          */
    WOI_E_INCOMPATIBLE = -3,  /* flux data violate the compatibility condition        */
    WOI_E_UNSUPPORTED = -4,   /* valid request the library does not implement         */
    WOI_E_DEVICE = -5,        /* a HIP call failed                                    */
    WOI_E_OOM = -6            /* device allocation or workspace too small             */
} woi_status;

/* Interface geometry (Sec. 4.6: implicit surfaces with exact sampling and
 * intersection, and 2D polylines as surface meshes). */
typedef enum {
    WOI_SHAPE_SPHERE = 0,     /* |y - center| = radius, any dimension                   */
    WOI_SHAPE_ELLIPSOID = 1,  /* (y - c)^T A (y - c) = 1, A symmetric positive definite  */
    WOI_SHAPE_POLYLINE2D = 2, /* closed counter-clockwise polygon, dimension 2 only      */
    WOI_SHAPE_MESH3D = 3      /* closed triangle mesh, dimension 3 only: every edge shared by
                                 two triangles in opposite directions, outward normals
                                 (b - a) x (c - a); no variance-reduced estimator         */
} woi_shape_kind;

typedef struct {
    int kind;                 /* woi_shape_kind                                        */
    int n_vertices;           /* POLYLINE2D: vertex count (>= 3); MESH3D (>= 4)        */
    double center[WOI_MAX_DIM];
    double radius;            /* SPHERE                                                */
    const double *A;          /* ELLIPSOID: dim*dim row-major, host memory             */
    const double *vertices;   /* POLYLINE2D: n_vertices*2 (x, y), host memory, CCW;
                                 MESH3D: n_vertices*3 (x, y, z)                          */
    int n_triangles;          /* MESH3D: triangle count (>= 4)                           */
    const int *triangles;     /* MESH3D: n_triangles*3 vertex indices, host memory       */
} woi_shape;

/* Flux-jump / Neumann data b_i on an interface (Eq. interface_problem). */
typedef enum {
    WOI_DATA_ZERO = 0,
    WOI_DATA_FOURIER2D = 1,   /* a0 + sum_k a_k cos(k th) + c_k sin(k th), th = angle about center;
                                 coef = [a0, a1, c1, ..., aK, cK], n_terms = K           */
    WOI_DATA_DIRPOLY = 2,     /* sum_t coef_t prod_d e_d^{exps[t*dim+d]}, e = (y-center)/|y-center|;
                                 n_terms terms, exponents <= 15                         */
    WOI_DATA_SOURCE_FLUX = 3, /* coef[0] (y - center).n(y) / |y - center|^dim            */
    WOI_DATA_FIELD_FLUX = 4   /* n(y) . coef[0..dim-1] (flux of a uniform field)        */
} woi_data_kind;

typedef struct {
    int kind;                 /* woi_data_kind                                          */
    int n_terms;
    double center[WOI_MAX_DIM];
    const double *coef;       /* host memory                                            */
    const uint8_t *exps;      /* DIRPOLY: n_terms*dim exponents, host memory            */
} woi_data;

/* Compatibility of the data (Sec. 1 requires zero flux through every interface). */
typedef enum {
    WOI_COMPAT_PER_INTERFACE = 0, /* |int b_i dA| <= tol * int |b_i| dA for every i      */
    WOI_COMPAT_GLOBAL = 1,        /* int b_1 = sum_{i>1} int b_i (global flux balance)   */
    WOI_COMPAT_NONE = 2
} woi_compat_mode;

typedef struct {
    int dim;                  /* 2 .. WOI_MAX_DIM                                       */
    int n_regions;            /* N, 1 .. WOI_MAX_REGIONS                                */
    const int *parent;        /* [N], parent[0] = -1, 0 <= parent[i] < i               */
    const double *sigma;      /* [N] conductivities, sigma_i >= 0, sigma_i + sigma_parent > 0 */
    const woi_shape *shapes;  /* [N] shapes[i] is the interface dOmega_i               */
    const woi_data *data;     /* [N] b_i                                                */
    int compat_mode;          /* woi_compat_mode                                        */
    double compat_tol;        /* relative tolerance, e.g. 1e-8                          */
} woi_problem_desc;

typedef struct woi_problem woi_problem;

/* Compile a problem on the host (validation, alpha_i / beta scalings of Eq.
 * unit_coeff_charge_density_sys, schedule distribution of Eq. scheduled_interface_pdf,
 * region relations for the transition pdfs of Eq. naive_woi_p, surface measures,
 * polyline arclength tables and bounding-volume trees, VR half-surface tables of
 * Sec. 4.4, compatibility check).  Deep-copies everything it needs: the descriptor
 * and its arrays may be freed after return.  Makes no HIP call.
 * Errors: INVALID_ARG, GEOMETRY, INCOMPATIBLE, UNSUPPORTED, OOM. */
woi_status woi_problem_create(const woi_problem_desc *desc, woi_problem **out);
/* Copy the compiled tables to the current device (hipMalloc + hipMemcpy, synchronous).
 * Called implicitly by the first woi_estimate / woi_trace; call it explicitly before
 * capturing those calls in a HIP graph.  Idempotent; the problem is then bound to that
 * device (INVALID_ARG if used from another).  Errors: DEVICE, OOM, INVALID_ARG. */
woi_status woi_problem_upload(woi_problem *p);
/* Frees host and device memory of the problem (no stream synchronisation: the caller
 * must ensure no enqueued work still reads it). */
void woi_problem_destroy(woi_problem *p);

typedef struct {
    int dim, n_regions;
    double alpha_l1;                          /* ||alpha||_1                          */
    double alpha[WOI_MAX_REGIONS];            /* alpha_i                              */
    double beta_scale[WOI_MAX_REGIONS];       /* beta_i = beta_scale[i] * b_i         */
    double area[WOI_MAX_REGIONS];             /* |dOmega_i|                           */
    double area_plus[WOI_MAX_REGIONS];        /* |{beta_i >= 0}| (NaN if unsupported) */
    double area_minus[WOI_MAX_REGIONS];       /* |{beta_i <  0}|                      */
    double flux[WOI_MAX_REGIONS];             /* integral of b_i over dOmega_i        */
    size_t device_bytes;                      /* size of the uploaded tables          */
} woi_problem_info;
woi_status woi_problem_get_info(const woi_problem *p, woi_problem_info *out);

/* PLAIN: Alg. 2; VR: Alg. 3; NAIVE: the naive estimator of Sec. 4.2 (Eq. naive_woi_estimator),
 * one observation per Markov tree: every interface tuple (h_0..h_i), i <= M, of the tree is
 * summed with weight w_i prod_{m=1}^{i} alpha_{h_m} instead of being scheduled (Theorem 2 gives
 * both the same expectation).  A tree has sum_{i=0}^{M} N^{i+1} interface points, drawn with the
 * transitions of Eq. naive_woi_p; node (h_0..h_i) draws from its own counter, so a branch is
 * reused by all its extensions.  For NAIVE, walks = trees per point (walk_offset = first tree);
 * it requires batch_share = 1 and instance = 0 (WOI_E_UNSUPPORTED otherwise) and
 * (N + 1)^(M + 1) <= 2^31 and N^(M + 1) <= WOI_NAIVE_MAX_LEAVES leaves per tree, which bounds the
 * work of one tree (WOI_E_INVALID_ARG otherwise); FP32 walks keep FP64 tree sums; schedule_mode and
 * block_size are ignored. */
typedef enum { WOI_EST_PLAIN = 0, WOI_EST_VR = 1, WOI_EST_NAIVE = 2 } woi_estimator;
typedef enum { WOI_PREC_FP64 = 0, WOI_PREC_FP32 = 1 } woi_precision;
typedef enum { WOI_SCHED_PER_GROUP = 0, WOI_SCHED_SHARED = 1 } woi_schedule_mode;

typedef struct {
    uint64_t seed;            /* Philox4x32-10 key                                      */
    uint64_t walks;           /* W walkers per point; VR uses W/2 two-walker samples (W even) */
    uint64_t walk_offset;     /* first walker index (resume; even for VR)               */
    int M;                    /* truncation, steps 0..M, 0 <= M <= WOI_MAX_M            */
    int estimator;            /* woi_estimator                                          */
    int precision;            /* woi_precision: FP64 everywhere, or FP32 walks with FP64 sums */
    int schedule_mode;        /* PER_GROUP: schedule keyed by (walk, point group);
                                 SHARED: keyed by walk only (wave-uniform, Alg. 1)      */
    int batch_share;          /* B >= 1: points p with equal p/B share trajectories (Sec. 4.6) */
    uint32_t instance;        /* < 2^24, mixed into every random-number counter         */
    int samples_per_thread;   /* 0 = automatic                                          */
    int block_size;           /* 0 = automatic (64 or 256)                              */
    void *event_begin;        /* optional hipEvent_t recorded on `stream` right before the walk
                                 kernel, and event_end right after it (NULL = none)     */
    void *event_end;
} woi_query;

/* Device workspace (bytes) woi_estimate needs for P points with this query. */
woi_status woi_workspace_size(const woi_problem *p, int64_t P, const woi_query *q, size_t *bytes);

/* Estimate u, its standard error, grad u and the gradient's standard error at P points
 * (Eq. woi_estimator / variance_reduced_woi_estimator and their gradient versions,
 * Alg. 1 with one schedule per sample).
 *   points   [P*dim] row-major doubles (device)
 *   mean, se [P] doubles (device); grad, grad_se [P*dim] (device) or NULL
 *   workspace/workspace_bytes: device scratch of at least woi_workspace_size() bytes
 *   counters: NULL or device uint64[WOI_COUNTERS] that the call adds to: [0] walker-steps,
 *             [1] redraws (q = 0), [2] rejections, [3] attempt-cap hits, [4] zero distances,
 *             [5] search node tests (polyline blocks, mesh BVH nodes), [6] segment or triangle
 *             tests, [7] uniform ("other") transitions, [8] FP64 rechecks of FP32 decisions
 *             (crossing and sign tests whose FP32 value fell in the rounding band; see
 *             woi_stats)
 * Errors: INVALID_ARG (sizes, NULL, VR with odd walks, naive with (N+1)^(M+1) > 2^31),
 *         UNSUPPORTED (VR in dim > 3 or with meshes; naive with batch_share > 1 or instance != 0),
 *         OOM (workspace), DEVICE. */
woi_status woi_estimate(const woi_problem *p, const double *points, int64_t P, const woi_query *q,
                        double *mean, double *se, double *grad, double *grad_se,
                        void *workspace, size_t workspace_bytes, uint64_t *counters, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): woi_estimate without a workspace.  The partial sums go
 * to a library-owned device array of WOI_NOALLOC_SCRATCH_BYTES (16 MiB, one per device, held
 * until the process ends); the sample chunks are capped so that they fit, which bounds P at
 * WOI_NOALLOC_SCRATCH_BYTES / ((2 + 2 dim) 8) points per call (349525 in 2D).  The call makes no
 * allocation: the problem must already be on the current device (woi_problem_upload).
 * Plain and VR estimators with batch_share = 1 only.  Results equal woi_estimate's up to the
 * summation order of the chunk sums.  All calls on one device share the array: calls that
 * overlap on a device race (order them on one stream).
 * Errors: INVALID_ARG (as woi_estimate; problem not uploaded; P too large), UNSUPPORTED (naive
 * estimator, batch_share > 1), DEVICE. */
#define WOI_NOALLOC_SCRATCH_BYTES (16u << 20)
woi_status woi_estimate_noalloc(const woi_problem *p, const double *points, int64_t P, const woi_query *q,
                                double *mean, double *se, double *grad, double *grad_se,
                                uint64_t *counters, void *stream);

/* Per-sample values and per-step decisions of Alg. 2 / Alg. 3 (the scheduled interface, the
 * transition case of Eq. naive_woi_p, the hit count q and the uniform pick among the hits of
 * Sec. 4.2.3, and the sign of Eq. naive_woi_T), for parity checks: samples
 * [walk_offset, walk_offset + n_samples) of every point.  F[(p*n + j)*K + k] = N * (walker k's sum), K = 1 (plain) or 2 (VR); for NAIVE,
 * F[p*n + j] = tree j's value and trace must be NULL (WOI_E_INVALID_ARG otherwise);
 * G[((p*n + j)*K + k)*dim + d]; trace[((p*n + j)*K + k)*(M+1) + i] = decision word
 * (bits 0-5 region, 6-7 case 0 first/1 same/2 descendant/3 other, 8-15 q,
 * 16-23 pick, 24 negative sign, 25-31 attempts).  All device pointers; G, trace may be NULL. */
woi_status woi_trace(const woi_problem *p, const double *points, int64_t P, const woi_query *q,
                     uint64_t n_samples, double *F, double *G, uint32_t *trace, void *stream);

/* Many independent problem instances in one persistent launch (uneven N, P, W; the
 * batching of Sec. 4.6 taken across problems).  Every sample is the sample woi_estimate
 * draws for the same query (same Philox keys), so an instance's results match a
 * woi_estimate call up to the summation order of the per-point sums.
 *
 * Work: items (instance, tile of 64 points, chunk of samples), largest first, pulled by a
 * grid of resident workgroups from one atomic queue; the waves of a workgroup split an item,
 * add their sums in wave order and write the item's one partial slot, and the reduction
 * merges the slots in sample order (deterministic results).
 *
 * Items with batch_share = 1 run in the persistent kernel; items with batch_share B > 1 (shared
 * trajectories, Sec. 4.6: points with equal p / B share every trajectory) run in the same graph
 * after it, each as the trajectory-generation and evaluation launches of woi_estimate with that
 * query, so their results equal woi_estimate's exactly.  Triangle meshes only in the latter.
 * Requirements: all items share dim, estimator and precision; fewer than 2^32 samples per
 * point; samples_per_thread is ignored; block_size is the same for all items: 0 (tuned) or
 * 256 / 512 (64 x waves per workgroup).  Per-item arrays are host
 * arrays of length n; the pointers inside are device pointers.
 * Events: items[0].query.event_begin / event_end, if set, are recorded on `stream` around
 * the graph launch. */
typedef struct {
    const woi_problem *problem;
    const double *points;     /* device [P*dim]                                         */
    int64_t P;
    woi_query query;
    double *mean, *se, *grad, *grad_se;  /* device; grad/grad_se may be NULL            */
} woi_batch_item;

/* Device workspace (bytes) woi_estimate_batch needs: 256 bytes of queue head, then one
 * running-sum record per resident workgroup and the partial slots (one per work item) of the
 * largest plan the tuner may choose, then the largest shared-trajectory item's workspace
 * (woi_workspace_size of its query; the shared items run one after another).  Uploads the problems and
 * queries the current device.  Errors: INVALID_ARG, UNSUPPORTED, DEVICE. */
woi_status woi_batch_workspace_size(const woi_batch_item *items, int n, size_t *bytes);

/* Enqueue the whole batch on `stream` as one HIP graph: a fill kernel zeroes the queue
 * head, the persistent walk kernel drains the queue, the reduction writes every item's
 * mean / se / grad / grad_se.
 * The first call with a given (items, workspace, counters, device) builds the plan in
 * library-owned device memory and captures the graph; with block_size 0 it also times the
 * candidate launch shapes on a scaled-down copy of the batch, which synchronizes `stream`
 * and the device.  Later calls with the same arguments only launch the cached graph (up
 * to 8 cached batches per process, least recently used evicted); the seeds are not part
 * of that key: changed seeds are copied into the library's seed table on `stream` before
 * the launch.  A cached graph reads the current contents of the points and problems; a
 * problem must stay alive while a batch that uses it can run.  Calls that share a
 * workspace or an item list must be ordered on one stream.
 * counters: NULL or device uint64[WOI_COUNTERS], added to as in woi_estimate.
 * Errors: INVALID_ARG, UNSUPPORTED, OOM (workspace too small or plan allocation), DEVICE. */
woi_status woi_estimate_batch(const woi_batch_item *items, int n, void *workspace, size_t workspace_bytes,
                              uint64_t *counters, void *stream);

/* Training data of the neural-network surrogate of Sec. 5 (Eq. MLP_loss: a mean squared misfit to
 * the WoI estimates at interior points plus one to the Neumann data at boundary points).
 *   interior: cell centres x_d = lo_d + (i_d + 1/2)(hi_d - lo_d) / grid_n of a grid_n^dim grid over
 *     the bounding box of dOmega, in row-major order (last coordinate fastest), strictly inside
 *     dOmega and, when margin > 0, farther than `margin` from every interface (sphere: distance;
 *     ellipsoid: first-order level-set distance |q - 1| / |grad q|; polyline: distance to the
 *     nearest segment).  The first `cap` are written to interior [cap*dim] (device); the count of
 *     all of them to *n_interior (host).  Estimate u, its SE and grad u there with woi_estimate.
 *   boundary (bc_n > 0, dim 2 or 3): n_bc = bc_n (2D: angles 2 pi k / bc_n about the circle's
 *     centre, or the polyline's vertex mean -- the farthest crossing of that ray) or 2 bc_n^2 (3D:
 *     polar angles pi (i + 1/2) / bc_n, azimuths pi j / bc_n, through the sphere or ellipsoid
 *     parametrisation) points bc_points [n_bc*dim], outward unit normals bc_normals [n_bc*dim] and
 *     targets bc_flux [n_bc] = b_1 / sigma_1, the normal derivative the Neumann condition
 *     sigma_1 d_n u = b_1 prescribes (device arrays; *n_bc, host, may be NULL).
 * Synchronizes `stream` (the interior count is copied to the host); allocates 8 bytes of device
 * memory per call.  Errors: INVALID_ARG (sizes, NULL, grid_n^dim > 1e10), UNSUPPORTED (triangle
 * meshes; boundary points for dim > 3), DEVICE, OOM. */
typedef struct {
    int grid_n;               /* grid nodes per axis (>= 1)                            */
    int bc_n;                 /* boundary resolution (0: no boundary points)          */
    double margin;            /* minimum distance of interior points from interfaces  */
} woi_training_spec;
woi_status woi_training_points(const woi_problem *p, const woi_training_spec *spec, double *interior, int64_t cap,
                               int64_t *n_interior, double *bc_points, double *bc_normals, double *bc_flux,
                               int64_t *n_bc, void *stream);

/* Statistics of one or more calls: the counter array they added to (see woi_estimate) and the
 * time between the query's event_begin and event_end.
 *   counters     device uint64[WOI_COUNTERS] (read with a synchronous copy) or NULL (zeros)
 *   event_begin, event_end   hipEvent_t recorded by a call (query.event_begin / event_end), or
 *                NULL: then seconds = -1.  Waits for event_end.
 * walks = walker-steps / (M + 1) is left to the caller (steps per walker vary with M).
 * Errors: INVALID_ARG (NULL out), DEVICE. */
typedef struct {
    uint64_t walker_steps, redraws, rejections, cap_hits, zero_distances;
    uint64_t search_node_tests, segment_tests, other_transitions;
    uint64_t fp64_fallbacks;  /* FP32 decisions recomputed in FP64 because their FP32 value
                                 fell inside the rounding band (crossing parameters near the
                                 self-hit threshold, near-zero vertex distances, near-tangent
                                 discriminants and signs)                               */
    double seconds;
} woi_stats;
woi_status woi_stats_read(const uint64_t *counters, void *event_begin, void *event_end, woi_stats *out);

const char *woi_status_string(woi_status s);
const char *woi_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WOI_H */
