// woi_batch_host.cpp -- host side of batched estimation: validation, the work-item plan,
// the launch-shape autotuner and the cached HIP graph (queue reset, persistent walk kernel,
// reduction).
//
// Partial sums.  The waves of the workgroup that runs an item add their per-lane sums in wave
// order (through the workgroup's record in the workspace) and write one slot per item, so the
// partial traffic is (2 + 2 dim) doubles per (tile lane, chunk), whatever the launch shape.
//
// Plan.  Instance i has T_i = ceil(P_i / 64) tiles and S_i samples (walkers, or walker
// pairs for VR).  A model cost e_i per sample and lane, (M_i + 1) K (1 + 3 f_i) with f_i the
// schedule mass on polylines (Theorem 2: H ~ |alpha| / ||alpha||_1), converts samples into
// workgroup time.  With the batch's total cost C spread over G resident workgroups, big
// chunks take about C / (G g) each (g = grain), and the last eighth of every instance's
// samples is cut into chunks eight times smaller; the item list is sorted by decreasing
// cost (longest-processing-time first), so the queue ends on small items and workgroups
// finish together.
//
// Autotuner.  With block_size 0 the first call with a new item list times every candidate
// (waves per workgroup 4 or 8) x (grain 4, 8, 16) on a miniature of the batch -- the same
// instances and tiles with the sample counts scaled down to about 1.5e8 lane-steps -- and
// keeps the fastest.  That call synchronizes the device; later calls replay the graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <numeric>
#include <vector>

#include "woi.h"
#include "woi_device.h"
#include "woi_internal.h"
#include "woi_launch.h"

using woi::set_error;

namespace {

struct Tune {
    int waves;   // waves per workgroup (64 * waves threads): walkers of one tile in flight
    int grain;   // big items per resident workgroup
};

const Tune kCandidates[] = {{4, 4}, {4, 8}, {4, 16}, {8, 4}, {8, 8}, {8, 16}};
constexpr Tune kDefault{8, 8};

// Validated batch, independent of the launch shape.
struct Spec {
    int dim = 0;
    bool vr = false, f32 = false;
    bool shared = true;                // every item takes the shared schedule
    int n = 0;
    std::vector<woi::ProblemRef> ref;
    std::vector<uint64_t> ns, first;   // samples per point, first sample index
    std::vector<double> cost;          // model cost of one sample in one lane
    std::vector<int64_t> P;
    unsigned smem = 0;                 // LDS staging bytes (0: tables read from global memory)
};

struct Plan {
    Tune t{};
    unsigned grid = 0;
    std::vector<woi::BInst> inst;
    std::vector<woi::BItem> items;
    std::vector<uint32_t> ctab;
    uint64_t n_slots = 0;
    int64_t n_points = 0;
    // workspace after the queue head: the workgroups' running sums, then the partial slots
    size_t wg_bytes(int dim) const { return ((size_t)grid * 64 * (2 + 2 * dim) * sizeof(double) + 255) & ~size_t(255); }
    size_t partial_bytes(int dim) const {
        return wg_bytes(dim) + (size_t)n_slots * 64 * (2 + 2 * dim) * sizeof(double);
    }
    size_t table_bytes(size_t n_seeds) const {   // [BInst][BItem][ctab][pad to 8][seeds]
        const size_t a = inst.size() * sizeof(woi::BInst) + items.size() * sizeof(woi::BItem) + ctab.size() * sizeof(uint32_t);
        return ((a + 7) & ~size_t(7)) + n_seeds * sizeof(uint64_t);
    }
};

constexpr size_t kHead = 256;   // the queue head sits at the start of the workspace

woi_status validate(const woi_batch_item* items, int n, Spec& sp) {
    if (!items || n < 1) return set_error(WOI_E_INVALID_ARG, "empty batch");
    if (n > (1 << 24)) return set_error(WOI_E_INVALID_ARG, "at most 2^24 instances per batch");
    sp = Spec{};
    sp.n = n;
    for (int i = 0; i < n; ++i) {
        const woi_batch_item& it = items[i];
        woi_status st = woi::check_query(it.problem, it.P, &it.query);
        if (st != WOI_OK) return set_error(st, "item %d: %s", i, woi_last_error());
        if (!it.points || !it.mean || !it.se) return set_error(WOI_E_INVALID_ARG, "item %d: NULL points/mean/se", i);
        if (it.query.estimator == WOI_EST_NAIVE)
            return set_error(WOI_E_UNSUPPORTED, "item %d: batched estimation does not take the naive estimator", i);
        if (woi::problem_has_mesh(it.problem) && it.query.batch_share == 1)
            return set_error(WOI_E_UNSUPPORTED,
                             "item %d: the persistent kernel does not take triangle meshes (batch_share > 1 does)", i);
        const bool vr = it.query.estimator == WOI_EST_VR, f32 = it.query.precision == WOI_PREC_FP32;
        if (i == 0) { sp.vr = vr; sp.f32 = f32; }
        sp.shared = sp.shared && it.query.schedule_mode == WOI_SCHED_SHARED;
        if (vr != sp.vr || f32 != sp.f32)
            return set_error(WOI_E_INVALID_ARG, "item %d: every item needs the same estimator and precision", i);
        if (i > 0 && it.query.block_size != items[0].query.block_size)
            return set_error(WOI_E_INVALID_ARG, "item %d: every item needs the same block_size", i);
        const uint64_t ns = vr ? it.query.walks / 2 : it.query.walks;
        if (ns >= (1ull << 32)) return set_error(WOI_E_INVALID_ARG, "item %d: at most 2^32 - 1 samples per point", i);
        if ((it.P + 63) / 64 >= (1ll << 32)) return set_error(WOI_E_INVALID_ARG, "item %d: too many points", i);
        sp.ns.push_back(ns);
        sp.first.push_back(vr ? it.query.walk_offset / 2 : it.query.walk_offset);
        sp.P.push_back(it.P);
    }
    const int bs = items[0].query.block_size;
    if (bs != 0 && bs != 256 && bs != 512)
        return set_error(WOI_E_INVALID_ARG, "batched block_size must be 0 (tuned), 256 or 512");
    return WOI_OK;
}

// Device-side part of the validation: upload the problems, check dimensions, cost model,
// LDS staging decision.
woi_status resolve(const woi_batch_item* items, Spec& sp) {
    unsigned need = 0;
    bool all_fit = true;
    const int budget = woi::lds_budget();
    for (int i = 0; i < sp.n; ++i) {
        woi::ProblemRef r{};
        woi_status st = woi::problem_ref(const_cast<woi_problem*>(items[i].problem), &r);
        if (st != WOI_OK) return set_error(st, "item %d: %s", i, woi_last_error());
        if (i == 0) sp.dim = r.dim;
        if (r.dim != sp.dim) return set_error(WOI_E_INVALID_ARG, "item %d: every problem needs the same dimension", i);
        sp.ref.push_back(r);
        const woi::DevProblem* h = r.host;
        double poly = 0;
        for (int j = 0; j < h->N; ++j)
            if (h->reg[j].kind == WOI_SHAPE_POLYLINE2D) poly += std::fabs(h->reg[j].alpha);
        const double f = h->alpha_l1 > 0 ? poly / h->alpha_l1 : 0.0;
        sp.cost.push_back((sp.vr ? 2.0 : 1.0) * (items[i].query.M + 1) * (1.0 + 3.0 * f));
        if (h->lds_bytes > 0) {
            need = std::max(need, (unsigned)h->lds_bytes);
            if (h->lds_bytes > budget) all_fit = false;
        }
    }
    sp.smem = sp.dim == 2 && need > 0 && all_fit ? need : 0u;
    return WOI_OK;
}

// Work items for a launch shape; `scale` < 1 shrinks every sample count (tuning probe).
Plan make_plan(const woi_batch_item* items, const Spec& sp, Tune t, unsigned grid, double scale) {
    Plan pl;
    pl.t = t;
    pl.grid = grid;
    const int n = sp.n;
    std::vector<uint64_t> ns(n);
    double total = 0;
    for (int i = 0; i < n; ++i) {
        ns[i] = scale >= 1.0 ? sp.ns[i] : std::max<uint64_t>(1, (uint64_t)std::llround((double)sp.ns[i] * scale));
        total += (double)((sp.P[i] + 63) / 64) * (double)ns[i] * sp.cost[i] / t.waves;
    }
    const double c_big = std::max(1e-30, total / ((double)grid * t.grain)), c_small = c_big / 8;
    struct Tmp { uint32_t inst, tile, chunk; double cost; };
    std::vector<Tmp> tmp;
    int64_t out0 = 0;
    for (int i = 0; i < n; ++i) {
        const woi_batch_item& it = items[i];
        const double u = sp.cost[i] / t.waves;   // workgroup time of one sample of the tile
        const uint64_t S = ns[i];
        const uint64_t nb = std::min<uint64_t>(S, std::max<uint64_t>(t.waves, (uint64_t)std::llround(c_big / u)));
        const uint64_t nsm = std::min<uint64_t>(nb, std::max<uint64_t>(t.waves, (uint64_t)std::llround(c_small / u)));
        const uint64_t nbig = (uint64_t)(0.875 * (double)S) / nb;
        woi::BInst b{};
        b.c0 = (uint32_t)pl.ctab.size();
        uint64_t pos = 0;
        pl.ctab.push_back(0);
        for (uint64_t k = 0; k < nbig; ++k) { pos += nb; pl.ctab.push_back((uint32_t)pos); }
        while (pos < S) { pos = std::min(S, pos + nsm); pl.ctab.push_back((uint32_t)pos); }
        b.n_chunks = (uint32_t)(pl.ctab.size() - b.c0 - 1);
        const uint64_t tiles = (uint64_t)((it.P + 63) / 64);
        b.dp = sp.ref[i].dev;
        b.points = it.points;
        b.P = it.P;
        b.first_sample = sp.first[i];
        b.slot0 = pl.n_slots;
        b.out0 = out0;
        b.mean = it.mean;
        b.se = it.se;
        b.grad = it.grad;
        b.grad_se = it.grad_se;
        b.M = it.query.M;
        b.shared_sched = it.query.schedule_mode == WOI_SCHED_SHARED;
        b.instance = it.query.instance;
        b.lds = sp.smem ? (uint32_t)sp.ref[i].host->lds_bytes : 0u;
        pl.n_slots += tiles * b.n_chunks;
        out0 += it.P;
        for (uint64_t tile = 0; tile < tiles; ++tile)
            for (uint32_t k = 0; k < b.n_chunks; ++k) {
                const uint32_t len = pl.ctab[b.c0 + k + 1] - pl.ctab[b.c0 + k];
                tmp.push_back({(uint32_t)i, (uint32_t)tile, k, len * u});
            }
        pl.inst.push_back(b);
    }
    pl.n_points = out0;
    std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp& a, const Tmp& b) { return a.cost > b.cost; });
    pl.items.reserve(tmp.size());
    for (const Tmp& x : tmp) {
        const double c = x.cost / c_small * 1024.0;
        pl.items.push_back({x.inst, x.tile, x.chunk, (uint32_t)std::min(c, 4294967295.0)});
    }
    return pl;
}

struct Device {
    int cus = 0;
    hipStream_t capture = nullptr;   // private stream the graphs are captured on
};

woi_status device_info(Device*& out) {
    static std::mutex mu;
    static Device devs[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return set_error(WOI_E_DEVICE, "no HIP device");
    std::lock_guard<std::mutex> lk(mu);
    Device& d = devs[dev];
    if (!d.cus) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return set_error(WOI_E_DEVICE, "hipGetDeviceProperties failed");
        if (hipStreamCreateWithFlags(&d.capture, hipStreamNonBlocking) != hipSuccess)
            return set_error(WOI_E_DEVICE, "hipStreamCreate failed");
        d.cus = prop.multiProcessorCount;
    }
    out = &d;
    return WOI_OK;
}

unsigned grid_for(const Spec& sp, const Device& d, int waves) {
    const int per_cu = woi::batch_blocks_per_cu(sp.dim, sp.vr, sp.f32, sp.shared, waves, sp.smem);
    return (unsigned)std::max(1, per_cu) * (unsigned)d.cus;
}

// Tables of a plan in one device buffer: [BInst][BItem][ctab][seeds].
struct DevTables {
    void* buf = nullptr;
    woi::BInst* inst = nullptr;
    woi::BItem* items = nullptr;
    uint32_t* ctab = nullptr;
    uint64_t* seeds = nullptr;
};

woi_status upload(const Plan& pl, const std::vector<uint64_t>& seeds, void* buf, DevTables& t) {
    char* b = static_cast<char*>(buf);
    t.buf = buf;
    t.inst = reinterpret_cast<woi::BInst*>(b);
    t.items = reinterpret_cast<woi::BItem*>(b + pl.inst.size() * sizeof(woi::BInst));
    t.ctab = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(t.items) + pl.items.size() * sizeof(woi::BItem));
    const size_t a = reinterpret_cast<char*>(t.ctab + pl.ctab.size()) - b;
    t.seeds = reinterpret_cast<uint64_t*>(b + ((a + 7) & ~size_t(7)));
    auto put = [](void* dst, const void* src, size_t bytes) {
        return bytes == 0 || hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!put(t.inst, pl.inst.data(), pl.inst.size() * sizeof(woi::BInst)) ||
        !put(t.items, pl.items.data(), pl.items.size() * sizeof(woi::BItem)) ||
        !put(t.ctab, pl.ctab.data(), pl.ctab.size() * sizeof(uint32_t)) ||
        !put(t.seeds, seeds.data(), seeds.size() * sizeof(uint64_t)))
        return set_error(WOI_E_DEVICE, "plan upload failed");
    return WOI_OK;
}

// Items of a batch by path: `one` (batch_share 1) run in the persistent kernel, `shared` (batch_share
// > 1) as shared-trajectory launches after it.  `order` lists the item indices in the order of the
// device seed table: the persistent kernel's instances first, then the shared items.
struct Split {
    std::vector<woi_batch_item> one;
    std::vector<int> shared, order;
};

Split split_items(const woi_batch_item* items, int n) {
    Split sp;
    for (int i = 0; i < n; ++i)
        if (items[i].query.batch_share == 1) { sp.one.push_back(items[i]); sp.order.push_back(i); }
    for (int i = 0; i < n; ++i)
        if (items[i].query.batch_share > 1) { sp.shared.push_back(i); sp.order.push_back(i); }
    return sp;
}

std::vector<uint64_t> seeds_of(const woi_batch_item* items, const std::vector<int>& order) {
    std::vector<uint64_t> s(order.size());
    for (size_t i = 0; i < order.size(); ++i) s[i] = items[order[i]].query.seed;
    return s;
}

// Workspace of the shared items (run one after another): the largest one's.
size_t shared_bytes(const woi_batch_item* items, const Split& sl) {
    size_t b = 0;
    for (int i : sl.shared) b = std::max(b, woi::shared_workspace_bytes(items[i].problem, items[i].P, &items[i].query));
    return (b + 255) & ~size_t(255);
}

woi::BParams batch_params(const Plan& pl, const DevTables& t, void* ws, uint64_t* counters, int dim) {
    woi::BParams bp{};
    bp.inst = t.inst;
    bp.items = t.items;
    bp.ctab = t.ctab;
    bp.seeds = t.seeds;
    bp.n_items = (uint32_t)pl.items.size();
    bp.head = static_cast<uint32_t*>(ws);
    bp.wg_sums = reinterpret_cast<double*>(static_cast<char*>(ws) + kHead);
    bp.partials = reinterpret_cast<double*>(static_cast<char*>(ws) + kHead + pl.wg_bytes(dim));
    bp.counters = counters;
    return bp;
}

// Times every candidate on the miniature batch and returns the fastest.  The caller's
// stream is synchronized first: the probes run on the library's own stream and read the
// points.
woi_status autotune(const woi_batch_item* items, const Spec& sp, const Device& d, hipStream_t caller, Tune& best) {
    if (hipStreamSynchronize(caller) != hipSuccess) return set_error(WOI_E_DEVICE, "hipStreamSynchronize failed");
    double full = 0;
    for (int i = 0; i < sp.n; ++i) full += (double)((sp.P[i] + 63) / 64) * 64.0 * (double)sp.ns[i] * sp.cost[i];
    const double scale = std::min(1.0, 1.5e8 / std::max(1.0, full));
    std::vector<Plan> plans;
    size_t tab = 0, part = 0;
    for (const Tune& t : kCandidates) {
        plans.push_back(make_plan(items, sp, t, grid_for(sp, d, t.waves), scale));
        tab = std::max(tab, plans.back().table_bytes((size_t)sp.n));
        part = std::max(part, plans.back().partial_bytes(sp.dim));
    }
    void *tbuf = nullptr, *ws = nullptr;
    if (hipMalloc(&tbuf, tab) != hipSuccess) return set_error(WOI_E_OOM, "tuning: hipMalloc(%zu) failed", tab);
    if (hipMalloc(&ws, kHead + part) != hipSuccess) {
        (void)hipFree(tbuf);
        return set_error(WOI_E_OOM, "tuning: hipMalloc(%zu) failed", kHead + part);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    woi_status st = WOI_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = set_error(WOI_E_DEVICE, "hipEventCreate failed");
    float best_ms = 0;
    for (size_t c = 0; c < plans.size() && st == WOI_OK; ++c) {
        DevTables t;
        std::vector<int> ident((size_t)sp.n);
        std::iota(ident.begin(), ident.end(), 0);
        st = upload(plans[c], seeds_of(items, ident), tbuf, t);
        if (st != WOI_OK) break;
        const woi::BParams bp = batch_params(plans[c], t, ws, nullptr, sp.dim);
        float ms = 0;
        for (int rep = 0; rep < 2 && st == WOI_OK; ++rep) {   // the first run loads the code object
            hipError_t e = woi::launch_fill_u32(bp.head, 1, 0, d.capture);
            if (e == hipSuccess) e = hipEventRecord(e0, d.capture);
            if (e == hipSuccess) e = woi::launch_batch(bp, sp.dim, sp.vr, sp.f32, sp.shared, plans[c].t.waves, plans[c].grid, sp.smem,
                                                 d.capture);
            if (e == hipSuccess) e = hipEventRecord(e1, d.capture);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) st = set_error(WOI_E_DEVICE, "tuning launch failed: %s", hipGetErrorString(e));
        }
        if (st == WOI_OK && (c == 0 || ms < best_ms)) { best_ms = ms; best = plans[c].t; }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(ws);
    (void)hipFree(tbuf);
    return st;
}

// ---------------------------------------------------------------------------- graph cache
struct Entry {
    std::vector<uint64_t> key;
    int device = -1;
    Plan plan;
    DevTables tab;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t need = 0;
    // Seeds are not part of the graph: the device seed table is refreshed on the caller's
    // stream before a launch whose seeds differ, from one of two pinned staging buffers
    // (each reused only after the copy that last read it has completed).
    std::vector<int> order;               // item of every seed-table entry (Split::order)
    std::vector<uint64_t> seeds;          // what the device table holds once queued copies land
    uint64_t* pinned[2] = {nullptr, nullptr};
    hipEvent_t copied[2] = {nullptr, nullptr};
    int next = 0;
    ~Entry() {
        for (int b = 0; b < 2; ++b) {
            if (copied[b]) (void)hipEventDestroy(copied[b]);
            if (pinned[b]) (void)hipHostFree(pinned[b]);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (tab.buf) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(device);
            (void)hipFree(tab.buf);
            (void)hipSetDevice(cur);
        }
    }
};

std::mutex g_mu;
std::list<std::unique_ptr<Entry>> g_cache;   // most recently used first
constexpr size_t kCacheSize = 8;

std::vector<uint64_t> make_key(const woi_batch_item* items, int n, const Spec& sp, const void* ws,
                               const uint64_t* counters, int device) {
    std::vector<uint64_t> k;
    k.reserve(4 + (size_t)n * 20);
    k.push_back((uint64_t)n);
    k.push_back((uint64_t)(uintptr_t)ws);
    k.push_back((uint64_t)(uintptr_t)counters);
    k.push_back((uint64_t)device);
    for (int i = 0; i < n; ++i) {
        const woi_batch_item& it = items[i];
        const woi_query& q = it.query;
        const uint64_t f[] = {sp.ref.empty() ? 0 : sp.ref[i].serial, (uint64_t)(uintptr_t)it.problem,
                              (uint64_t)(uintptr_t)it.points, (uint64_t)it.P, q.walks, q.walk_offset,
                              (uint64_t)q.M, (uint64_t)q.estimator, (uint64_t)q.precision, (uint64_t)q.schedule_mode,
                              (uint64_t)q.batch_share, (uint64_t)q.instance, (uint64_t)q.block_size,
                              (uint64_t)(uintptr_t)it.mean, (uint64_t)(uintptr_t)it.se, (uint64_t)(uintptr_t)it.grad,
                              (uint64_t)(uintptr_t)it.grad_se};
        k.insert(k.end(), std::begin(f), std::end(f));
    }
    return k;
}

// Plan for the batch as it will run: tuned (block_size 0) or the given shape.
woi_status choose_plan(const woi_batch_item* items, const Spec& sp, const Device& d, hipStream_t caller, Plan& pl) {
    Tune t = kDefault;
    const int bs = items[0].query.block_size;
    if (bs) t.waves = bs / 64;
    else {
        const woi_status st = autotune(items, sp, d, caller, t);
        if (st != WOI_OK) return st;
    }
    pl = make_plan(items, sp, t, grid_for(sp, d, t.waves), 1.0);
    if (pl.items.size() >= (1ull << 32)) return set_error(WOI_E_INVALID_ARG, "batch has more than 2^32 work items");
    return WOI_OK;
}

// Validated spec of the persistent kernel's items (batch_share 1).
woi_status spec_of(const std::vector<woi_batch_item>& one, Spec& sp1) {
    woi_status st = validate(one.data(), (int)one.size(), sp1);
    if (st == WOI_OK) st = resolve(one.data(), sp1);
    return st;
}

woi_status build_entry(const woi_batch_item* items, int n, const Spec& sp, Device& d, void* ws, size_t ws_bytes,
                       uint64_t* counters, hipStream_t caller, Entry& e) {
    const Split sl = split_items(items, n);
    const int n1 = (int)sl.one.size();
    Spec sp1;
    if (n1) {
        woi_status st = spec_of(sl.one, sp1);
        if (st == WOI_OK) st = choose_plan(sl.one.data(), sp1, d, caller, e.plan);
        if (st != WOI_OK) return st;
    }
    const size_t part = n1 ? ((e.plan.partial_bytes(sp.dim) + 255) & ~size_t(255)) : 0;
    const size_t shb = shared_bytes(items, sl);
    char* const wsc = static_cast<char*>(ws);
    e.need = kHead + part + shb;
    if (!ws || ws_bytes < e.need)
        return set_error(WOI_E_OOM, "workspace of %zu bytes is smaller than the %zu bytes needed", ws_bytes, e.need);
    if (hipMalloc(&e.tab.buf, e.plan.table_bytes((size_t)n)) != hipSuccess)
        return set_error(WOI_E_OOM, "hipMalloc(%zu) for the work items failed", e.plan.table_bytes((size_t)n));
    e.order = sl.order;
    e.seeds = seeds_of(items, e.order);
    woi_status st = upload(e.plan, e.seeds, e.tab.buf, e.tab);
    if (st != WOI_OK) return st;
    for (int b = 0; b < 2; ++b) {
        if (hipHostMalloc(reinterpret_cast<void**>(&e.pinned[b]), e.seeds.size() * sizeof(uint64_t)) != hipSuccess)
            return set_error(WOI_E_OOM, "hipHostMalloc for the seed table failed");
        if (hipEventCreateWithFlags(&e.copied[b], hipEventDisableTiming) != hipSuccess)
            return set_error(WOI_E_DEVICE, "hipEventCreate failed");
    }
    const woi::BParams bp = batch_params(e.plan, e.tab, ws, counters, sp.dim);
    woi::BRParams rp{};
    rp.inst = e.tab.inst;
    rp.ctab = e.tab.ctab;
    rp.partials = bp.partials;
    rp.n_inst = n1;
    rp.n_points = e.plan.n_points;
    rp.dim = sp.dim;
    // set the kernels' LDS limits before capturing
    if (n1 && woi::batch_blocks_per_cu(sp.dim, sp1.vr, sp1.f32, sp1.shared, e.plan.t.waves, sp1.smem) <= 0)
        return set_error(WOI_E_DEVICE, "batch kernel cannot be resident");
    if (hipStreamBeginCapture(d.capture, hipStreamCaptureModeRelaxed) != hipSuccess)
        return set_error(WOI_E_DEVICE, "hipStreamBeginCapture failed");
    hipError_t err = hipSuccess;
    if (n1) {
        err = woi::launch_fill_u32(bp.head, 1, 0, d.capture);
        if (err == hipSuccess)
            err = woi::launch_batch(bp, sp.dim, sp1.vr, sp1.f32, sp1.shared, e.plan.t.waves, e.plan.grid, sp1.smem,
                                    d.capture);
        if (err == hipSuccess) err = woi::launch_batch_reduce(rp, d.capture);
    }
    // shared-trajectory items, one after another in the workspace after the persistent kernel's
    for (size_t j = 0; j < sl.shared.size() && err == hipSuccess && st == WOI_OK; ++j) {
        const woi_batch_item& it = items[sl.shared[j]];
        woi_query q = it.query;
        q.event_begin = q.event_end = nullptr;
        st = woi::enqueue_shared(it.problem, it.points, it.P, &q, it.mean, it.se, it.grad, it.grad_se,
                                 wsc + kHead + part, shb, counters, e.tab.seeds + n1 + j, d.capture);
    }
    const hipError_t ec = hipStreamEndCapture(d.capture, &e.graph);
    if (st != WOI_OK) return st;
    if (err != hipSuccess || ec != hipSuccess)
        return set_error(WOI_E_DEVICE, "graph capture failed: %s", hipGetErrorString(err != hipSuccess ? err : ec));
    if (hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0) != hipSuccess)
        return set_error(WOI_E_DEVICE, "hipGraphInstantiate failed");
    return WOI_OK;
}

}  // namespace

extern "C" {

woi_status woi_batch_workspace_size(const woi_batch_item* items, int n, size_t* bytes) {
    if (!bytes) return set_error(WOI_E_INVALID_ARG, "NULL bytes");
    Spec sp;
    woi_status st = validate(items, n, sp);
    if (st != WOI_OK) return st;
    st = resolve(items, sp);
    if (st != WOI_OK) return st;
    Device* d = nullptr;
    st = device_info(d);
    if (st != WOI_OK) return st;
    // the largest over the shapes the tuner may pick (or the one given), then the shared items'
    const Split sl = split_items(items, n);
    size_t part = 0;
    if (!sl.one.empty()) {
        Spec sp1;
        st = spec_of(sl.one, sp1);
        if (st != WOI_OK) return st;
        const int bs = items[0].query.block_size;
        for (const Tune& t : kCandidates) {
            if (bs && t.waves != bs / 64) continue;
            if (bs && t.grain != kDefault.grain) continue;
            const Plan pl = make_plan(sl.one.data(), sp1, t, grid_for(sp1, *d, t.waves), 1.0);
            part = std::max(part, (pl.partial_bytes(sp.dim) + 255) & ~size_t(255));
        }
    }
    *bytes = kHead + part + shared_bytes(items, sl);
    return WOI_OK;
}

woi_status woi_estimate_batch(const woi_batch_item* items, int n, void* workspace, size_t workspace_bytes,
                              uint64_t* counters, void* stream) {
    Spec sp;
    woi_status st = validate(items, n, sp);
    if (st != WOI_OK) return st;
    st = resolve(items, sp);
    if (st != WOI_OK) return st;
    Device* d = nullptr;
    st = device_info(d);
    if (st != WOI_OK) return st;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const std::vector<uint64_t> key = make_key(items, n, sp, workspace, counters, dev);
    std::lock_guard<std::mutex> lk(g_mu);
    Entry* e = nullptr;
    for (auto it = g_cache.begin(); it != g_cache.end(); ++it)
        if ((*it)->key == key) {
            g_cache.splice(g_cache.begin(), g_cache, it);
            e = g_cache.front().get();
            break;
        }
    if (!e) {
        auto fresh = std::make_unique<Entry>();
        fresh->key = key;
        fresh->device = dev;
        st = build_entry(items, n, sp, *d, workspace, workspace_bytes, counters, static_cast<hipStream_t>(stream), *fresh);
        if (st != WOI_OK) return st;
        g_cache.push_front(std::move(fresh));
        while (g_cache.size() > kCacheSize) g_cache.pop_back();
        e = g_cache.front().get();
    }
    if (workspace_bytes < e->need)
        return set_error(WOI_E_OOM, "workspace of %zu bytes is smaller than the %zu bytes needed", workspace_bytes, e->need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<uint64_t> seeds = seeds_of(items, e->order);
    if (seeds != e->seeds) {   // new seeds: refresh the device table on the caller's stream
        const int b = e->next;
        if (hipEventSynchronize(e->copied[b]) != hipSuccess) return set_error(WOI_E_DEVICE, "hipEventSynchronize failed");
        std::memcpy(e->pinned[b], seeds.data(), seeds.size() * sizeof(uint64_t));
        if (hipMemcpyAsync(e->tab.seeds, e->pinned[b], seeds.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipEventRecord(e->copied[b], s) != hipSuccess)
            return set_error(WOI_E_DEVICE, "seed table update failed");
        e->next ^= 1;
        e->seeds.swap(seeds);
    }
    const woi_query& q0 = items[0].query;
    if (q0.event_begin && hipEventRecord(static_cast<hipEvent_t>(q0.event_begin), s) != hipSuccess)
        return set_error(WOI_E_DEVICE, "hipEventRecord(begin) failed");
    const hipError_t err = hipGraphLaunch(e->exec, s);
    if (err != hipSuccess) return set_error(WOI_E_DEVICE, "hipGraphLaunch failed: %s", hipGetErrorString(err));
    if (q0.event_end && hipEventRecord(static_cast<hipEvent_t>(q0.event_end), s) != hipSuccess)
        return set_error(WOI_E_DEVICE, "hipEventRecord(end) failed");
    return WOI_OK;
}

}  // extern "C"
