// woi_launch.h -- kernel parameter blocks and launchers (host <-> device boundary inside
// the library; not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "woi_device.h"

namespace woi {

// One estimation launch: grid.x covers points (one lane per point), grid.y covers
// chunks of `samples_per_thread` consecutive samples.
struct KParams {
    const DevProblem* dp;
    const double* points;          // [P*dim]
    int64_t P;
    uint64_t n_samples;            // samples per point (walkers, or walker pairs for VR)
    uint64_t first_sample;         // index of the first sample
    uint32_t samples_per_thread;
    uint32_t k0, k1;               // Philox key (seed)
    int M;
    int batch_share;
    int shared_sched;
    int mesh;                      // 3D problem with triangle-mesh interfaces: the mesh-capable kernels
    uint32_t instance;
    double* partials;              // [chunks][P][2 + 2 dim] or null
    const uint64_t* seed_tab;      // trajectory generation: the Philox key read from here (device) when
                                   // not null, else k0, k1 (a cached graph whose seed may change)
    double* traceF;                // per-walker values (trace mode) or null
    double* traceG;
    uint32_t* trace;
    uint64_t* counters;
};

// Reduction of n_chunks partial slots per point ([slot][P][2 + 2 dim] doubles); slot c holds
// full + min(samples_per_thread, max(0, tail - c samples_per_thread)) samples.
struct RParams {
    const double* partials;
    int64_t P;
    int dim;
    int n_chunks;
    uint32_t samples_per_thread;
    uint64_t full, tail;
    double *mean, *se, *grad, *grad_se;
};

// Shared trajectories (batch_share B > 1).  Generation: lane = point group g < ng; rows of
// `lg` lanes walk runs of `spt` samples of the chunk's `ns`; trajectories go to `traj`
// (planes of ns * K * (M + 1) * ng elements, see StoreSink).  Evaluation: lane = point,
// grid.y = piece of `spt_e` samples, staged through LDS `tile_rows` (sample, walker, step)
// rows at a time; writes (accumulate = 0) or adds to (accumulate = 1) the partials of slot
// blockIdx.y, so slot y collects piece y of every chunk.
struct TParams {
    void* traj;                    // R-typed planes
    size_t plane;                  // elements per plane
    int ng;                        // point groups
    uint32_t ns;                   // samples in this chunk
    uint64_t chunk_first;          // first sample index of the chunk
    uint32_t spt;                  // generation: samples per thread
    int lg;                        // generation: lanes per row (multiple of 64, divides the block)
    uint32_t spt_e;                // evaluation: samples per piece
    int tile_rows;                 // evaluation: rows per LDS tile
    int accumulate;                // evaluation: add to the slots (every chunk after the first)
};

constexpr int EVAL_BLOCK = 256;            // points per evaluation workgroup
constexpr int EVAL_LDS = 32 * 1024;        // LDS tile budget of the evaluation kernel
// Groups one evaluation workgroup can touch, and the LDS its tile of `rows` rows takes.
inline int eval_groups(int B, int64_t P) {
    const int64_t g = (EVAL_BLOCK + B - 1) / B + 1, ng = (P + B - 1) / B;
    return (int)(g < ng ? g : ng);
}
inline size_t eval_lds_bytes(int B, int64_t P, int dim, int rows, size_t elem) {
    return (size_t)rows * eval_groups(B, P) * (size_t)((dim + 2 + 3) & ~3) * elem;
}

hipError_t launch_traj(const KParams& kp, const TParams& tp, int dim, bool vr, bool fp32, unsigned lds_bytes,
                       hipStream_t s);
hipError_t launch_eval(const KParams& kp, const TParams& tp, int dim, bool vr, bool fp32, hipStream_t s);

// lds_bytes > 0 (dimension 2, at most lds_budget()): polyline tables are staged in LDS;
// block must then be 512 threads
hipError_t launch_walk(const KParams& kp, int dim, bool vr, bool fp32, unsigned lds_bytes, dim3 grid, dim3 block,
                       hipStream_t s);
hipError_t launch_reduce(const RParams& rp, hipStream_t s);

// Naive estimator (Markov trees): wave = (point, chunk of samples_per_thread trees), lane = leaf;
// grid = (ceil(P / 4), chunks), 256 threads.  FP64 or FP32 walks (FP64 tree sums); partials and
// trace values as launch_walk (K = 1, one value per tree).
struct NParams {
    uint32_t leaves;               // N^(M+1) leaves per tree
    uint32_t span0;                // N^M: leaves under one root
};
hipError_t launch_naive(const KParams& kp, const NParams& np, int dim, bool fp32, dim3 grid, hipStream_t s);

// ----------------------------------------------------------------------------- surrogate training data
// Interior nodes x_d = lo_d + (i_d + 1/2) step_d of an n^dim grid (last coordinate fastest) inside
// region 0 and farther than `margin` from every interface (when margin > 0), written in grid order
// to `out` (the first `cap`; the total to *count, device); boundary nodes k < n_bc (2D: angle
// 2 pi k / bc_n; 3D: bc_n polar x 2 bc_n azimuthal angles) with normals and b_1 / sigma_1.
struct TrainParams {
    const DevProblem* dp;
    int n;
    double lo[WOI_MAX_DIM], step[WOI_MAX_DIM];
    double margin;
    uint64_t nodes;
    double* out;
    int64_t cap;
    int64_t* count;
    int bc_n;
    int64_t n_bc;
    double *bc_points, *bc_normals, *bc_flux;
};
hipError_t launch_training(const TrainParams& tp, int dim, hipStream_t s);

// ----------------------------------------------------------------------------- batches
// Many instances in one persistent launch.  A work item is (instance, tile of 64 points,
// chunk of samples); the workgroup that pulls it splits the chunk's samples evenly over
// its WV waves, adds their sums in wave order through its record wg_sums[blockIdx.x] and
// writes partial slot slot0 + tile * n_chunks + chunk (64 lanes x (2 + 2 dim) doubles,
// field f of lane l at f * 64 + l).  Chunk k of an instance covers samples
// [ctab[c0 + k], ctab[c0 + k + 1]) counted from first_sample; every tile of the instance
// has the same chunks.
struct BInst {
    const DevProblem* dp;
    const double* points;
    int64_t P;
    uint64_t first_sample;
    uint64_t slot0;
    int64_t out0;              // index of the instance's first point in the flattened point list
    double *mean, *se, *grad, *grad_se;
    int M, shared_sched;
    uint32_t instance;
    uint32_t lds;              // bytes of polyline tables staged in LDS (0: read from global memory)
    uint32_t c0, n_chunks;
};

struct BItem {                 // 16 bytes
    uint32_t inst, tile, chunk, cost;
};

struct BParams {
    const BInst* inst;
    const BItem* items;
    const uint32_t* ctab;
    const uint64_t* seeds;     // Philox key of every instance (refreshed before each launch)
    uint32_t n_items;
    uint32_t* head;            // queue head, zeroed before the launch
    double* wg_sums;           // [grid][2 + 2 dim][64]: each workgroup's running sum of its waves
    double* partials;
    uint64_t* counters;
};

struct BRParams {
    const BInst* inst;
    const uint32_t* ctab;
    const double* partials;
    int n_inst;
    int64_t n_points;          // total points over all instances
    int dim;
};

// Persistent walk kernel: grid = resident workgroups, 64 * waves threads each (waves 4 or 8).
// smem > 0: polyline tables are staged in LDS (dimension 2; every instance with polylines
// then needs lds <= smem bytes).  shared: every instance takes the shared schedule (the
// kernel is then compiled for it).
hipError_t launch_batch(const BParams& bp, int dim, bool vr, bool fp32, bool shared, int waves, unsigned grid,
                        unsigned smem, hipStream_t s);
hipError_t launch_batch_reduce(const BRParams& rp, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s);
// Resident workgroups per CU of the batch kernel for this configuration (0 on error).
int batch_blocks_per_cu(int dim, bool vr, bool fp32, bool shared, int waves, unsigned smem);
// Bytes of LDS one workgroup may stage on the current device: the device's per-workgroup
// limit, at most LDS_BUDGET_MAX.
int lds_budget();

}  // namespace woi
