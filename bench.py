#!/usr/bin/env python3
"""Walk-on-Interfaces benchmark on one MI355X.

Headline workload (the batched uneven 2D instances): 512 independent problems, each the unit
disk with 1-16 circle or star interfaces (stars r0 (1 + 0.2 cos k t) as 512-vertex polylines) in
a random nesting tree, sigma = 10^U(-1, 3), 5-mode random Fourier flux data with zero mean,
P = 2^U(4, 10) points and W = 10^U(3, 6) walkers per point, M = 4.  One step = the whole batch
estimated once (values and gradients of every point), inputs resident in HBM, as ONE persistent
graph launch (queue reset, persistent walk kernel, reduction) with FP32 walks and FP64
per-point sums; the same batch in FP64 gives the equal-standard-error comparison and the paired
FP32 - FP64 difference on identical random streams.

Beside it, one record per configuration ("configs") and, as the last key, a compact
"summary" of every configuration's ms per step, roofline fraction, speed-up at equal SE, paired
z and flip rate: the concentric
disk (FP64 plain, W = 1e4), the 2D star tree (FP32 batched / per point / VR / shared
trajectories against FP64 plain), the 3D sphere + ellipsoid tree (VR), the 6D nested spheres,
the point-charge ellipsoids (3-6D), the triangle-mesh tree and the naive Markov trees; each with
its FP32-vs-FP64 decision-flip rate on identical streams.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walk-steps/s and eval-points/s at fixed std. error, FP32-batched vs FP64 plain"

# Algorithmic FP work per event of the 2D walk kernels (counted from the kernel source; a
# transcendental counts as one flop, an FMA as two, compares and integer work count zero).
FLOPS_PER_WALKER_STEP = 29      # Phi + grad Phi + accumulation (19) and the Q/T/sign update (10)
FLOPS_PER_OTHER = 18            # uniform re-sample + |K*| |dOmega| factor
FLOPS_PER_NODE_TEST = 4         # distance of a block end vertex from the line (two FMAs)
FLOPS_PER_SEGMENT_TEST = 4      # distance of the segment end vertex (crossings add ~10, rare)
FLOPS_PER_WALKER = 57           # step-0 datum b(y_0) (5-mode Fourier) and Q_0
PEAK_FP32_TFLOPS = 157.3        # MI355X vector FP32 peak (packed FMA)
# HBM bytes per launch of the headline batch kernel (512 instances), from the FETCH_SIZE and
# WRITE_SIZE passes summarised in profiles/, each scaled by what the same counter reads for a
# 1 GiB device copy.  None whenever the kernel has changed since those passes were taken.
BATCH_TRAFFIC_BYTES = 4.477e8   # FETCH 394.3 MB + WRITE 53.4 MB (profiles/batch_kernel_instances_2d_counters.md)


def log(msg):
    """Progress of the run on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def sig(x, n=4):
    """Round every float of a nested record to n significant digits (keeps the line short)."""
    if isinstance(x, float):
        if not math.isfinite(x) or x == 0.0:
            return x
        return round(x, n - 1 - int(math.floor(math.log10(abs(x)))))
    if isinstance(x, dict):
        return {k: sig(v, n) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [sig(v, n) for v in x]
    return x


def eval_flops_per_pair(m):
    """Algorithmic flops of one (point, trajectory step) pair of the evaluation kernel:
    x - y with the low part of x (2m), r^2 (2m - 1), the kernel powers, c_F phi accumulated
    (2), c_G r^-m (2) and the gradient FMAs (2m); a transcendental counts as one."""
    if m == 2:
        return 2 * m + (2 * m - 1) + 2 + 2 + 1 + 2 * m          # log2 and rcp
    return 2 * m + (2 * m - 1) + 1 + 1 + (m - 2) // 2 + m % 2 + 2 + 2 + 2 * m


class HipEvents:
    """hipEvent_t handles from libamdhip64 (events on the stream the kernels run on)."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]

    def create(self):
        e = ctypes.c_void_p()
        assert self.hip.hipEventCreate(ctypes.byref(e)) == 0
        return e.value

    def ms(self, a, b):
        t = ctypes.c_float()
        assert self.hip.hipEventElapsedTime(ctypes.byref(t), ctypes.c_void_p(a), ctypes.c_void_p(b)) == 0
        return t.value


def flops_of(counts, M=4):
    walker_steps, other, nodes, segs = counts[0], counts[7], counts[5], counts[6]
    walkers = walker_steps / (M + 1.0)
    return (FLOPS_PER_WALKER_STEP * walker_steps + FLOPS_PER_OTHER * other + FLOPS_PER_NODE_TEST * nodes +
            FLOPS_PER_SEGMENT_TEST * segs + FLOPS_PER_WALKER * walkers)


def timed(torch, ev, fn, steps, warmup):
    """Warm-up calls, then `steps` timed calls fn(k, events); returns wall seconds per call
    and the per-call HIP-event milliseconds (events recorded by the library on the launch
    stream around its kernels)."""
    for w in range(warmup):
        fn(1000 + w, None)
    evs = [(ev.create(), ev.create()) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        fn(k, evs[k])
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, [ev.ms(a, b) for a, b in evs]


class Path:
    """One estimator configuration on resident points: per-point (B = 1) or shared
    trajectories (B > 1).  Step k uses seed seed0 + k, so two precisions with the same
    seed0 run on identical random streams."""

    def __init__(self, woi, torch, prob, pts, walks, M, precision, estimator=0, B=1, seed0=1):
        self.woi, self.torch, self.prob, self.pts = woi, torch, prob, pts
        self.walks, self.M, self.precision, self.estimator, self.B, self.seed0 = walks, M, precision, estimator, B, seed0
        P, m = pts.shape
        self.out = tuple(torch.empty(*s, dtype=torch.float64, device="cuda") for s in ((P,), (P,), (P, m), (P, m)))
        q = woi.make_query(walks, M, precision=precision, estimator=estimator, schedule_mode=woi.SCHED_SHARED,
                           batch_share=B)
        self.ws = torch.empty(woi.workspace_size(prob, P, q), dtype=torch.uint8, device="cuda")
        self.first = None

    def __call__(self, k, events=None, counters=None):
        self.woi.estimate(self.prob, self.pts, self.walks, self.M, seed=self.seed0 + k, precision=self.precision,
                          estimator=self.estimator, schedule_mode=self.woi.SCHED_SHARED, batch_share=self.B,
                          out=self.out, workspace=self.ws, events=events, counters=counters)
        if k == 0 and events is not None:
            self.first = (self.out[0].clone(), self.out[1].clone())

    def run(self, ev, steps, warmup):
        wall, ms = timed(self.torch, ev, self, steps, warmup)
        mean, se = (t.cpu().numpy() for t in self.first)
        return {"wall": wall, "ms": ms, "mean": mean, "se": se}

    def counts(self):
        cnt = self.woi.new_counters()
        self(999, counters=cnt)
        return cnt.cpu().numpy().astype(float)


class BatchPath:
    """The same estimate as a one-item batch: woi_estimate_batch, one persistent graph launch
    (fill, persistent walk kernel, reduction) with the tuned launch shape.  Step k replays
    the cached graph with seed seed0 + k (the library refreshes its seed table first)."""

    def __init__(self, woi, torch, prob, pts, walks, M, precision, seed0=1, counters=None, estimator=0, B=1):
        self.torch, self.seed0 = torch, seed0
        self.b = woi.Batch([dict(problem=prob, points=pts, walks=walks, M=M, seed=seed0, precision=precision,
                                 estimator=estimator, schedule_mode=woi.SCHED_SHARED, batch_share=B)],
                           counters=counters)
        self.first = None

    def __call__(self, k, events=None):
        self.b.run(events=events, seed=self.seed0 + k)
        if k == 0 and events is not None:
            self.first = (self.b.outputs[0][0].clone(), self.b.outputs[0][1].clone())

    def run(self, ev, steps, warmup):
        wall, ms = timed(self.torch, ev, self, steps, warmup)
        mean, se = (t.cpu().numpy() for t in self.first)
        return {"wall": wall, "ms": ms, "mean": mean, "se": se}


def fixed_se(r, eps):
    """Time per step rescaled to standard error eps (SE ~ 1/sqrt(W))."""
    import numpy as np
    return r["wall"] * float(np.mean(r["se"] ** 2)) / eps ** 2


def paired(r32, r64):
    """FP32 - FP64 means on identical streams, in units of the FP64 standard error."""
    import numpy as np
    z = (r32["mean"] - r64["mean"]) / r64["se"]
    return {"mean_z": float(np.mean(z)), "mean_abs_z": float(np.mean(np.abs(z))), "max_abs_z": float(np.max(np.abs(z)))}


def flips(woi, torch, prob, pts, n, M, estimator=0, instance=0):
    """FP32 against FP64 walks on identical streams (shared schedule): the fraction of walkers
    whose decision words (region, case, q, pick, sign, attempts) differ in some step, and the
    FP64 rechecks per walker-step of the FP32 walks."""
    import numpy as np
    kw = dict(seed=31, estimator=estimator, schedule_mode=woi.SCHED_SHARED, instance=instance)
    _, _, t64 = woi.trace(prob, pts, n, M, precision=woi.FP64, **kw)
    _, _, t32 = woi.trace(prob, pts, n, M, precision=woi.FP32, **kw)
    c = woi.new_counters()
    woi.estimate(prob, pts, n * (2 if estimator == woi.VR else 1), M, precision=woi.FP32, counters=c, **kw)
    same = torch.all(t64 == t32, dim=-1).cpu().numpy()
    cn = c.cpu().numpy().astype(float)
    return {"walkers": int(same.size), "flip_rate": float(1.0 - same.mean()),
            "fp64_rechecks_per_walker_step": float(cn[8] / max(cn[0], 1.0))}


def config_block(woi, torch, ev, prob_desc, pts_np, walks, M, estimator, B, steps, flip_pts=64, flip_walks=2000):
    """FP32 per point, FP64 plain and FP32 shared trajectories for one configuration."""
    import numpy as np
    prob = woi.Problem(prob_desc)
    woi._lib.woi_problem_upload(prob.handle)
    pts = torch.tensor(pts_np, dtype=torch.float64, device="cuda")
    P, m = pts.shape
    K = 2 if estimator else 1
    point_steps = P * walks * (M + 1)                           # (point, walker, step) contributions
    r32 = Path(woi, torch, prob, pts, walks, M, woi.FP32, estimator).run(ev, steps, 1)
    r64 = Path(woi, torch, prob, pts, walks, M, woi.FP64, estimator).run(ev, 1, 0)
    rsh = BatchPath(woi, torch, prob, pts, walks, M, woi.FP32, estimator=estimator, B=B).run(ev, steps, 1)
    eps = float(np.median(r64["se"]))
    t64 = fixed_se(r64, eps)
    pairs = P * (walks // K) * K * (M + 1)
    ev_fl = pairs * eval_flops_per_pair(m) / (float(np.mean(rsh["ms"])) * 1e-3) / 1e12
    z = paired(r32, r64)
    fl = flips(woi, torch, prob, pts[:flip_pts], flip_walks, M, estimator)
    return {
        "fp32_ms": r32["wall"] * 1e3, "fp32_walk_steps_per_s": point_steps / r32["wall"],
        "fp64_ms": r64["wall"] * 1e3, "fp64_points_per_s_fixed_se": P / t64,
        "fp32_speedup_fixed_se": t64 / fixed_se(r32, eps),
        "shared": {"B": B, "ms": rsh["wall"] * 1e3, "walk_steps_per_s": point_steps / rsh["wall"],
                   "points_per_s_fixed_se": P / fixed_se(rsh, eps), "speedup_fixed_se": t64 / fixed_se(rsh, eps),
                   "pair_tflops": ev_fl},
        "paired_z": [z["mean_abs_z"], z["max_abs_z"]], "flip_rate": fl["flip_rate"],
        "fp64_rechecks_per_step": fl["fp64_rechecks_per_walker_step"],
    }


def disk_block(woi, torch, W, ev, steps):
    """Concentric disk (sigma 10 around 1, b = cos theta on both): 64 polar-grid points, W = 1e4,
    FP64 plain at M = 4, 8, 12, and FP32 at M = 4."""
    import numpy as np
    p, xs = W.concentric_disk_2d()
    prob = woi.Problem(p)
    woi._lib.woi_problem_upload(prob.handle)
    pts = torch.tensor(xs, dtype=torch.float64, device="cuda")
    out = {}
    for M in (4, 8, 12):
        r = Path(woi, torch, prob, pts, 10000, M, woi.FP64).run(ev, steps, 1)
        out[f"fp64_M{M}_ms"] = r["wall"] * 1e3
        out[f"fp64_M{M}_walk_steps_per_s"] = len(xs) * 10000 * (M + 1) / r["wall"]
    r32 = Path(woi, torch, prob, pts, 10000, 4, woi.FP32).run(ev, steps, 1)
    out["fp32_M4_ms"] = r32["wall"] * 1e3
    fl = flips(woi, torch, prob, pts, 4000, 4)
    out["flip_rate"] = fl["flip_rate"]
    out["fp64_rechecks_per_step"] = fl["fp64_rechecks_per_walker_step"]
    return out


def star_tree_block(woi, torch, W, ev, steps, walks):
    """2D star tree: FP32 batched (one-item batch graph), FP32 per point, FP64 plain, VR (FP32 and
    FP64) and shared trajectories (B = 16 <= 0.5 % of the points, Sec. 4.6)."""
    import numpy as np
    prob_desc, pts_np = W.star_tree_2d()
    M = 4
    prob = woi.Problem(prob_desc)
    woi._lib.woi_problem_upload(prob.handle)
    pts = torch.tensor(pts_np, dtype=torch.float64, device="cuda")
    P = pts.shape[0]
    steps_all = P * walks * (M + 1)
    cnt = woi.new_counters()
    BatchPath(woi, torch, prob, pts, walks, M, woi.FP32, seed0=999, counters=cnt)(0)
    c32 = cnt.cpu().numpy().astype(float)
    rb = BatchPath(woi, torch, prob, pts, walks, M, woi.FP32).run(ev, steps, 1)
    r64 = Path(woi, torch, prob, pts, walks, M, woi.FP64).run(ev, 1, 1)
    rpp = Path(woi, torch, prob, pts, walks, M, woi.FP32).run(ev, steps, 1)
    rvr = Path(woi, torch, prob, pts, walks, M, woi.FP32, woi.VR).run(ev, steps, 1)
    rvr64 = Path(woi, torch, prob, pts, walks, M, woi.FP64, woi.VR).run(ev, 1, 0)
    rsh = BatchPath(woi, torch, prob, pts, walks, M, woi.FP32, B=16).run(ev, steps, 1)
    eps = float(np.median(r64["se"]))
    t64 = fixed_se(r64, eps)
    kms = float(np.mean(rb["ms"]))
    ach = flops_of(c32, M) / (kms * 1e-3) / 1e12
    z = paired(rb, r64)
    zvr = paired(rvr, rvr64)
    fl = flips(woi, torch, prob, pts[::64], 2000, M)
    flv = flips(woi, torch, prob, pts[::64], 1000, M, woi.VR)
    return {
        "fp32_batched_ms": rb["wall"] * 1e3, "fp32_batched_walk_steps_per_s": c32[0] / rb["wall"],
        "fp32_batched_frac": ach / PEAK_FP32_TFLOPS, "fp32_batched_speedup_fixed_se": t64 / fixed_se(rb, eps),
        "fp32_per_point_ms": rpp["wall"] * 1e3,
        "fp64_ms": r64["wall"] * 1e3, "fp64_points_per_s_fixed_se": P / t64,
        "vr_fp32_ms": rvr["wall"] * 1e3, "vr_fp64_ms": rvr64["wall"] * 1e3,
        "vr_fp32_speedup_fixed_se": t64 / fixed_se(rvr, eps),
        "shared": {"B": 16, "ms": rsh["wall"] * 1e3, "walk_steps_per_s": steps_all / rsh["wall"],
                   "speedup_fixed_se": t64 / fixed_se(rsh, eps),
                   "pair_tflops": steps_all * eval_flops_per_pair(2) / (float(np.mean(rsh["ms"])) * 1e-3) / 1e12},
        "paired_z": [z["mean_abs_z"], z["max_abs_z"]], "vr_paired_z": [zvr["mean_abs_z"], zvr["max_abs_z"]],
        "flip_rate": fl["flip_rate"], "vr_flip_rate": flv["flip_rate"],
        "fp64_rechecks_per_step": fl["fp64_rechecks_per_walker_step"],
    }


def naive_block(woi, torch, W, ev, steps):
    """Naive Markov-tree estimator (FP64) against the scheduled FP64 estimator on the star tree
    (N = 9), M = 1..3: per tree sum_{i=0}^{M} 9^{i+1} interface points, against M + 1 per
    scheduled walker.  Cost at the same standard error, and the two means in combined SEs
    (Theorem 2: same expectation)."""
    import numpy as np
    prob_desc, pts_np = W.star_tree_2d()
    prob = woi.Problem(prob_desc)
    pts = torch.tensor(pts_np, dtype=torch.float64, device="cuda")
    P = pts.shape[0]
    N = prob.N
    out = {}
    for M, trees in ((1, 400), (2, 100), (3, 12)):
        nodes = sum(N ** (i + 1) for i in range(M + 1))
        rn = Path(woi, torch, prob, pts, trees, M, woi.FP64, woi.NAIVE).run(ev, steps, 1)
        rs = Path(woi, torch, prob, pts, 100000, M, woi.FP64).run(ev, 1, 1)
        eps = float(np.median(rs["se"]))
        z = (rn["mean"] - rs["mean"]) / np.sqrt(rn["se"] ** 2 + rs["se"] ** 2)
        out[f"M{M}"] = {"trees": trees, "ms": rn["wall"] * 1e3, "tree_points_per_s": P * trees * nodes / rn["wall"],
                        "scheduled_speedup_fixed_se": fixed_se(rn, eps) / fixed_se(rs, eps),
                        "z_mean_abs": float(np.mean(np.abs(z)))}
    return out


def training_block(woi, torch, W, ev, steps):
    """Training data of the neural-network surrogate (Sec. 5, Eq. MLP_loss) for the paper's Example 3
    set-ups: interior grid points inside dOmega (2D: 100^2 grid, about the paper's 7845 points; 3D:
    25^3, about its 8326) with the WoI estimate (value, SE, gradient; W = 1e5, M = 4 / 6, FP32 walks)
    at each, and boundary points with normals and b_1 / sigma_1 targets (2D: 500; 3D: 51 x 102).
    Points/s of the whole generation, and at the fixed SE of the FP64 path."""
    import numpy as np
    out = {}
    for name, prob_desc, grid_n, bc_n, M in (("ex3_2d", W.bower_ex3_2d(), 100, 500, 4),
                                             ("ex3_3d", W.zheng_ex3_3d(), 25, 51, 6)):
        gp = woi.Problem(prob_desc)
        woi._lib.woi_problem_upload(gp.handle)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, yb, nb, fb, cnt = woi.training_points(gp, grid_n, bc_n=bc_n)
        t_pts = time.perf_counter() - t0
        r32 = Path(woi, torch, gp, x, 100000, M, woi.FP32).run(ev, steps, 1)
        r64 = Path(woi, torch, gp, x, 100000, M, woi.FP64).run(ev, 1, 0)
        eps = float(np.median(r64["se"]))
        out[name] = {"interior_points": cnt, "boundary_points": int(yb.shape[0]), "points_ms": t_pts * 1e3,
                     "fp32_estimate_ms": r32["wall"] * 1e3, "fp64_estimate_ms": r64["wall"] * 1e3,
                     "points_per_s": cnt / (t_pts + r32["wall"]),
                     "points_per_s_fixed_se": cnt / (t_pts + fixed_se(r32, eps)),
                     "fp64_points_per_s_fixed_se": cnt / (t_pts + fixed_se(r64, eps))}
    return out


def summary(rec):
    """The last key of the line, short enough for a log tail: per configuration and path, ms per
    step, the roofline fraction where its flops are counted (2D walks; shared-trajectory pairs),
    the speed-up over FP64 plain at equal SE, FP32-vs-FP64 paired mean |z| and the decision-flip
    rate."""
    out = {}

    def put(key, ms, frac=None, x=None, z=None, flip=None):
        e = {"ms": ms}
        for k, v in (("frac", frac), ("x_fp64", x), ("z", z), ("flip", flip)):
            if v is not None:
                e[k] = v
        out[key] = e

    c = rec.get("configs", {})
    h = c.get("instances_2d", {})
    put("c3_batch", h.get("ms"), h.get("frac"), h.get("speedup_fixed_se"), (h.get("paired_z") or [None])[0],
        h.get("flip_rate"))
    sh = rec.get("shared_trajectories_b_0p5pct")
    if sh:
        put("c3_shared", sh["ms_per_step"], x=sh.get("speedup_vs_fp64_fixed_se"))
    d = c.get("disk_2d")
    if d:
        put("c1_fp64_M4", d["fp64_M4_ms"], flip=d["flip_rate"])
    t = c.get("star_tree_2d")
    if t:
        put("c2_batch", t["fp32_batched_ms"], t["fp32_batched_frac"], t["fp32_batched_speedup_fixed_se"],
            t["paired_z"][0], t["flip_rate"])
        put("c2_vr", t["vr_fp32_ms"], x=t["vr_fp32_speedup_fixed_se"], z=t["vr_paired_z"][0], flip=t["vr_flip_rate"])
        put("c2_shared", t["shared"]["ms"], t["shared"]["pair_tflops"] / PEAK_FP32_TFLOPS, t["shared"]["speedup_fixed_se"])
    for key, name in (("c4_vr", "ellipsoid_tree_3d_vr"), ("c5_6d", "spheres_6d"), ("pc3", "point_charge_3d"),
                      ("pc4", "point_charge_4d"), ("pc5", "point_charge_5d"), ("pc6", "point_charge_6d"),
                      ("mesh", "mesh_tree_3d")):
        b = c.get(name)
        if b:
            put(key, b["fp32_ms"], x=b["fp32_speedup_fixed_se"], z=b["paired_z"][0], flip=b["flip_rate"])
            put(key + "_shared", b["shared"]["ms"], b["shared"]["pair_tflops"] / PEAK_FP32_TFLOPS,
                b["shared"]["speedup_fixed_se"])
    n = c.get("naive_markov_trees")
    if n:
        for M in (1, 2, 3):
            if f"M{M}" in n:
                put(f"naive_M{M}", n[f"M{M}"]["ms"], x=1.0 / n[f"M{M}"]["scheduled_speedup_fixed_se"])
    tr = c.get("surrogate_training_data")
    if tr:
        for k, v in tr.items():
            put("train_" + k, v["points_ms"] + v["fp32_estimate_ms"], x=v["points_per_s_fixed_se"] / v["fp64_points_per_s_fixed_se"])
    return out


def run_instances(woi, torch, inst, probs, precision, steps, warmup, ev, counters=None, shared=False):
    """The 512-instance 2D batch in one persistent graph launch (tuned launch shape); the timed
    graph replays the whole batch (same seed: every replay recomputes it).  shared: every instance
    takes shared trajectories with B = floor(0.5 % of its points) (Sec. 4.6), B = 1 below 400 points."""
    entries = [dict(problem=g, points=x, walks=w, M=4, seed=4242, precision=precision, schedule_mode=woi.SCHED_SHARED,
                    instance=i, batch_share=max(1, int(0.005 * len(x))) if shared else 1)
               for i, (g, (_, x, w)) in enumerate(zip(probs, inst))]
    b = woi.Batch(entries, counters=counters)
    if counters is not None:
        b.run()
        return None
    wall, ms = timed(torch, ev, lambda k, e: b.run(events=e), steps, warmup)
    se = [o[1].cpu().numpy() for o in b.outputs]
    mean = [o[0].cpu().numpy() for o in b.outputs]
    return {"wall": wall, "ms": ms, "se": se, "mean": mean}


def cpu_baseline(inst, budget_s):
    """The FP64 oracle on the host cores over a fixed spread of the batch's instances, every point
    of each, with W scaled down by one factor so that the run takes about budget_s seconds."""
    import numpy as np
    from oracle import oracle as O
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = min(16, ncpu)   # the CPU share of one GPU on the benchmark box
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    idx = np.linspace(0, len(inst) - 1, 32).round().astype(int)
    ops = {int(i): O.OracleProblem(inst[i][0]) for i in idx}
    # probe: the same instances at W = 64
    t = time.perf_counter()
    steps = 0
    for i in idx[:8]:
        _, _, _, _, c = O.estimate(ops[int(i)], inst[i][1], 64, 4, seed=5, schedule_mode=1, threads=threads,
                                   instance=int(i))
        steps += c["walk_steps"]
    rate = steps / (time.perf_counter() - t)
    full = sum(len(inst[i][1]) * inst[i][2] * 5 for i in idx)
    f = min(1.0, budget_s * rate / full)
    t = time.perf_counter()
    steps = 0
    for i in idx:
        w = max(2, int(round(inst[i][2] * f)))
        _, _, _, _, c = O.estimate(ops[int(i)], inst[i][1], w, 4, seed=6, schedule_mode=1, threads=threads,
                                   instance=int(i))
        steps += c["walk_steps"]
    dt = time.perf_counter() - t
    return {"value": steps / dt, "unit": "walk-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"32 of the 512 instances (every 16th), all their points, each W scaled by {f:.3g}; "
                      f"FP64 oracle, {steps} walker-steps in {dt:.1f} s; host: {ncpu} CPUs available, "
                      f"{os.cpu_count()} online, {model}"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="measure only the headline batch")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison of the headline batch")
    ap.add_argument("--extra-steps", type=int, default=2, help="timed steps of the other configurations")
    ap.add_argument("--blocks", default="all",
                    help="comma-separated configurations to run besides the headline batch (instances_2d_shared: "
                         "the same batch with shared trajectories; disk_2d, star_tree_2d, ellipsoid_tree_3d_vr, "
                         "spheres_6d, point_charge_ellipsoids, mesh_tree_3d, naive_markov_trees, "
                         "surrogate_training_data), default all")
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--detail", default="", help="also write the full record to this JSON file")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after the run, copy this many bytes device-to-device three times (a plain copy "
                         "kernel of known size, to scale the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the walk ranges would shard with one all-reduce of per-point sums)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2508_16767_amd import woi

    torch.cuda.set_device(0)
    ev = HipEvents()

    # ---- headline: the 512 instances, FP32 walks, one persistent graph launch
    inst = W.star_tree_instances_2d()
    probs = [woi.Problem(p) for p, _, _ in inst]
    cnt = woi.new_counters()
    run_instances(woi, torch, inst, probs, woi.FP32, 0, 0, ev, counters=cnt)      # counting graph (untimed)
    counts = cnt.cpu().numpy().astype(float)
    log("headline: counting graph done")
    b32 = run_instances(woi, torch, inst, probs, woi.FP32, args.steps, args.warmup, ev)
    log(f"headline: FP32 batch {b32['wall'] * 1e3:.1f} ms per step")
    kms = float(np.mean(b32["ms"]))
    flops = flops_of(counts)
    achieved = flops / (kms * 1e-3) / 1e12
    n_points = sum(x.shape[0] for _, x, _ in inst)
    rec = {
        "metric": METRIC,
        "value": counts[0] / b32["wall"],
        "unit": "walk-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": b32["wall"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched uneven 2D instances: 512 problems, each the unit disk with 1-16 circle / "
                               "512-vertex star interfaces in a random nesting tree, sigma 10^U(-1,3), 5-mode Fourier "
                               "flux data; P = 2^U(4,10) points, W = 10^U(3,6) walkers, M = 4; values + gradients",
                   "instances": len(inst), "points": n_points, "walker_steps": counts[0],
                   "precision": "FP32 walks, FP64 per-point sums", "schedule": "shared",
                   "path": "one persistent graph launch (woi_estimate_batch: queue reset, batch_kernel, reduction)"},
        "graph_ms": kms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": BATCH_TRAFFIC_BYTES,
                     "kernel": "batch_kernel<float, 2, false, false, WV, true, true> (time: the whole graph)",
                     "flops_per_launch": flops},
    }
    if not args.no_fp64:
        b64 = run_instances(woi, torch, inst, probs, woi.FP64, 1, 0, ev)
        log(f"headline: FP64 batch {b64['wall'] * 1e3:.1f} ms")
        # fixed SE per instance: median SE of the FP64 batch, time rescaled by the mean SE^2 ratio
        bt32 = b32["wall"] * np.mean([np.mean(a ** 2) / np.median(c) ** 2 for a, c in zip(b32["se"], b64["se"])])
        bt64 = b64["wall"] * np.mean([np.mean(c ** 2) / np.median(c) ** 2 for c in b64["se"]])
        z = np.concatenate([(a - c) / s for a, c, s in zip(b32["mean"], b64["mean"], b64["se"])])
        rec["eval_points_per_s_fixed_se"] = n_points / bt32
        rec["fp64_batch"] = {"ms_per_step": b64["wall"] * 1e3, "walk_steps_per_s": counts[0] / b64["wall"],
                             "eval_points_per_s_fixed_se": n_points / bt64}
        rec["speedup_fp32_vs_fp64_fixed_se"] = bt64 / bt32
        rec["fp32_vs_fp64_paired_z"] = {"mean_z": float(np.mean(z)), "mean_abs_z": float(np.mean(np.abs(z))),
                                        "max_abs_z": float(np.max(np.abs(z)))}
    blocks = set(args.blocks.split(",")) if args.blocks != "all" else None

    def want(name):
        return not args.no_extra and (blocks is None or name in blocks)

    # the same batch with shared trajectories where the paper's batch size allows it (B <= 0.5 % of P)
    if want("instances_2d_shared"):
        bsh = run_instances(woi, torch, inst, probs, woi.FP32, args.extra_steps, 1, ev, shared=True)
        rec["shared_trajectories_b_0p5pct"] = {
            "ms_per_step": bsh["wall"] * 1e3, "walk_steps_per_s": counts[0] / bsh["wall"],
            "instances_shared": int(sum(1 for _, x, _ in inst if int(0.005 * len(x)) > 1))}
        if "fp64_batch" in rec:
            bts = bsh["wall"] * np.mean([np.mean(a ** 2) / np.median(c) ** 2 for a, c in zip(bsh["se"], b64["se"])])
            rec["shared_trajectories_b_0p5pct"]["speedup_vs_fp64_fixed_se"] = bt64 / bts
        log(f"headline: shared-trajectory batch {bsh['wall'] * 1e3:.1f} ms")
    sel = np.linspace(0, len(inst) - 1, 16).round().astype(int)
    fr = [flips(woi, torch, probs[i], inst[i][1][:64], 500, 4, instance=int(i)) for i in sel]
    rec["flips"] = {"instances": 16, "walkers": sum(f["walkers"] for f in fr),
                    "flip_rate": float(np.average([f["flip_rate"] for f in fr], weights=[f["walkers"] for f in fr])),
                    "fp64_rechecks_per_walker_step": float(counts[8] / max(counts[0], 1.0))}
    rec["counts_per_launch"] = {n: float(v) for n, v in zip(woi.COUNTER_NAMES, counts)}
    log("headline: flip rates done")
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
        log("cpu baseline done")

    cfg = {}
    es = args.extra_steps
    if want("disk_2d"):
        cfg["disk_2d"] = disk_block(woi, torch, W, ev, es)
        log("disk_2d done")
    if want("star_tree_2d"):
        cfg["star_tree_2d"] = star_tree_block(woi, torch, W, ev, es, 100000)
        log("star_tree_2d done")
    if want("ellipsoid_tree_3d_vr"):
        p4, x4 = W.ellipsoid_tree_3d()
        cfg["ellipsoid_tree_3d_vr"] = config_block(woi, torch, ev, p4, x4, 100000, 6, 1, 64, es)
        log("ellipsoid_tree_3d_vr done")
    if want("spheres_6d"):
        p5, x5 = W.nested_spheres_6d()
        cfg["spheres_6d"] = config_block(woi, torch, ev, p5, x5, 1000000, 8, 0, 4, es, flip_walks=1000)
        log("spheres_6d done")
    if want("point_charge_ellipsoids"):
        # three nested ellipsoids around the potential |x|^(2-m) of a point charge, m = 3..6
        # (1e4 points; M = m + 2 as the paper walks them; W = 2e5: the rates do not depend on W)
        for m in (3, 4, 5, 6):
            pm, xm = W.point_charge_ellipsoids(m)
            cfg[f"point_charge_{m}d"] = config_block(woi, torch, ev, pm, xm, 200000, m + 2, 0, 32, es, flip_walks=500)
            log(f"point_charge_{m}d done")
    if want("mesh_tree_3d"):
        p6, x6 = W.mesh_tree_3d()
        cfg["mesh_tree_3d"] = config_block(woi, torch, ev, p6, x6, 20000, 4, 0, 16, es, flip_walks=500)
        log("mesh_tree_3d done")
    if want("naive_markov_trees"):
        cfg["naive_markov_trees"] = naive_block(woi, torch, W, ev, es)
    if want("surrogate_training_data"):
        cfg["surrogate_training_data"] = training_block(woi, torch, W, ev, es)
        log("surrogate_training_data done")
    log("configurations done: " + ", ".join(cfg))
    headline_cfg = {"instances_2d": {
        "ms": rec["ms_per_step"], "walk_steps_per_s": rec["value"], "frac": rec["roofline"]["frac"],
        "speedup_fixed_se": rec.get("speedup_fp32_vs_fp64_fixed_se"),
        "paired_z": ([rec["fp32_vs_fp64_paired_z"]["mean_abs_z"], rec["fp32_vs_fp64_paired_z"]["max_abs_z"]]
                     if "fp32_vs_fp64_paired_z" in rec else None),
        "flip_rate": rec["flips"]["flip_rate"]}}
    rec["configs"] = {**headline_cfg, **cfg}
    rec["summary"] = summary(rec)
    rec["configs"], rec["summary"] = sig(rec["configs"], 3), sig(rec["summary"], 3)
    rec = sig(rec)
    if args.detail:
        with open(args.detail, "w") as f:
            json.dump(rec, f, indent=1)
    print(json.dumps(rec, separators=(",", ":")), flush=True)
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
