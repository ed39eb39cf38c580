#!/usr/bin/env python3
"""Walk-on-Interfaces benchmark on one MI355X.

Headline workload (the 2D star tree): unit disk containing 3 nested star
interfaces r0 (1 + 0.2 cos k t) with (r0, k) = (0.7, 3), (0.4, 5), (0.2, 7) as 2048-vertex
polylines and 5 circular inclusions (N = 9 regions, depth 3), sigma = 10^U(-1, 2), 5-mode
random Fourier flux data with zero mean; 4096 evaluation points (25 % within 1e-3 of an
interface); W = 1e5 walkers per point, M = 4; values and gradients.

One step = one full estimate of all points, inputs resident in HBM.  The headline path is
FP32-batched: FP32 walks with FP64 per-point sums and the wave-uniform shared schedule, run
as one persistent batched graph launch (queue reset, persistent walk kernel, reduction);
the FP64 plain path (the per-point walk kernel in FP64) gives the equal-standard-error
comparison, and the FP32 per-point kernel is reported beside it.  Beside it the line reports, at their full sizes: the star tree
with shared trajectories (B = 16 <= 0.5 % of the points, Sec. 4.6), the 512-instance batch
(one persistent graph launch), 3D spheres + ellipsoids with the variance-reduced estimator,
and the 6D nested spheres; each with its FP64 plain comparison at equal SE and the paired
FP32 - FP64 difference on identical random streams.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walk-steps/s and eval-points/s at fixed std. error, FP32-batched vs FP64 plain"

# Algorithmic FP work per event of the 2D walk kernel (counted from the kernel source; a
# transcendental counts as one flop, an FMA as two, compares and integer work count zero).
FLOPS_PER_WALKER_STEP = 29      # Phi + grad Phi + accumulation (19) and the Q/T/sign update (10)
FLOPS_PER_OTHER = 18            # uniform re-sample + |K*| |dOmega| factor
FLOPS_PER_NODE_TEST = 4         # distance of a block end vertex from the line (two FMAs)
FLOPS_PER_SEGMENT_TEST = 4      # distance of the segment end vertex (crossings add ~10, rare)
FLOPS_PER_WALKER = 57           # step-0 datum b(y_0) (5-mode Fourier) and Q_0
PEAK_FP32_TFLOPS = 157.3        # MI355X vector FP32 (packed) peak
# HBM bytes per launch of the timed FP32 walk kernel at W = 1e5, from the FETCH_SIZE and
# WRITE_SIZE passes in profiles/headline_kernels_star_tree_2d_counters.md, scaled by what the same
# counters read for a 1 GiB device copy.  None whenever the kernel has changed since those
# passes were taken.
TRAFFIC_BYTES = 858 * 1024 * 2.0 + 49152 * 1024 * 1.0
# The same for the persistent batch kernel of the headline graph.
BATCH_TRAFFIC_BYTES = 1790 * 1024 * 2.0 + 249172 * 1024 * 1.0


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


def flops_of(counts):
    walker_steps, other, nodes, segs = counts[0], counts[7], counts[5], counts[6]
    walkers = walker_steps / 5.0
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

    def __init__(self, woi, torch, prob, pts, walks, M, precision, seed0=1, counters=None):
        self.torch, self.seed0 = torch, seed0
        self.b = woi.Batch([dict(problem=prob, points=pts, walks=walks, M=M, seed=seed0, precision=precision,
                                 schedule_mode=woi.SCHED_SHARED)], counters=counters)
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


def config_block(woi, torch, ev, name, prob_desc, pts_np, walks, M, estimator, B, steps):
    """Per-point FP32 and FP64 and shared-trajectory FP32 for one configuration."""
    import numpy as np
    prob = woi.Problem(prob_desc)
    woi._lib.woi_problem_upload(prob.handle)
    pts = torch.tensor(pts_np, dtype=torch.float64, device="cuda")
    P, m = pts.shape
    K = 2 if estimator else 1
    point_steps = P * walks * (M + 1)                           # (point, walker, step) contributions
    r32 = Path(woi, torch, prob, pts, walks, M, woi.FP32, estimator).run(ev, steps, 1)
    r64 = Path(woi, torch, prob, pts, walks, M, woi.FP64, estimator).run(ev, 1, 0)
    rsh = Path(woi, torch, prob, pts, walks, M, woi.FP32, estimator, B).run(ev, steps, 1)
    eps = float(np.median(r64["se"]))
    t64 = fixed_se(r64, eps)
    pairs = P * (walks // K) * K * (M + 1)
    ev_fl = pairs * eval_flops_per_pair(m) / (float(np.mean(rsh["ms"])) * 1e-3) / 1e12
    return {
        "workload": name, "points": P, "walkers": walks, "M": M, "estimator": "VR" if estimator else "plain",
        "fixed_se": eps,
        "fp32_per_point": {"walk_steps_per_s": point_steps / r32["wall"], "ms_per_step": r32["wall"] * 1e3,
                           "speedup_vs_fp64_plain_fixed_se": t64 / fixed_se(r32, eps)},
        "fp64_plain": {"walk_steps_per_s": point_steps / r64["wall"], "ms_per_step": r64["wall"] * 1e3,
                       "eval_points_per_s_fixed_se": P / t64},
        "fp32_shared_trajectories": {"batch_share": B, "walk_steps_per_s": point_steps / rsh["wall"],
                                     "ms_per_step": rsh["wall"] * 1e3,
                                     "eval_points_per_s_fixed_se": P / fixed_se(rsh, eps),
                                     "speedup_vs_fp64_plain_fixed_se": t64 / fixed_se(rsh, eps),
                                     "pair_eval_tflops_over_traj_plus_eval": ev_fl},
        "fp32_vs_fp64_paired_z": paired(r32, r64),
    }


def naive_block(woi, torch, ev, prob, pts, steps):
    """Naive Markov-tree estimator (FP64) against the scheduled FP64 estimator on the star tree
    (N = 9), M = 1..3: per tree sum_{i=0}^{M} 9^{i+1} interface points, against M + 1 per
    scheduled walker.  Cost at the same standard error, and the two means in combined SEs
    (Theorem 2: same expectation)."""
    import numpy as np
    P = pts.shape[0]
    N = prob.N
    out = {"workload": "star tree 2D (N = 9: unit disk, 3 nested 2048-segment stars, 5 circles), 4096 points",
           "M": {}}
    for M, trees in ((1, 400), (2, 100), (3, 12)):
        nodes = sum(N ** (i + 1) for i in range(M + 1))
        rn = Path(woi, torch, prob, pts, trees, M, woi.FP64, woi.NAIVE).run(ev, steps, 1)
        rs = Path(woi, torch, prob, pts, 100000, M, woi.FP64).run(ev, 1, 1)
        eps = float(np.median(rs["se"]))
        z = (rn["mean"] - rs["mean"]) / np.sqrt(rn["se"] ** 2 + rs["se"] ** 2)
        out["M"][str(M)] = {
            "trees_per_point": trees, "tree_points": nodes, "lane_node_draws_per_tree": (M + 1) * N ** (M + 1),
            "ms_per_step": rn["wall"] * 1e3, "kernel_ms": float(np.mean(rn["ms"])),
            "tree_points_per_s": P * trees * nodes / rn["wall"],
            "eval_points_per_s_fixed_se": P / fixed_se(rn, eps),
            "scheduled_fp64_eval_points_per_s_fixed_se": P / fixed_se(rs, eps),
            "scheduled_speedup_fixed_se": fixed_se(rn, eps) / fixed_se(rs, eps),
            "naive_vs_scheduled_z": {"mean_abs": float(np.mean(np.abs(z))), "max_abs": float(np.max(np.abs(z)))}}
    return out


def run_batch(woi, torch, W, precision, steps, warmup, ev):
    """The 512-instance 2D batch in one persistent graph launch (tuned launch shape).  An
    untimed graph of the counting kernel gives the event counts; the timed graph replays
    the non-counting kernel (same seed: the whole batch is recomputed every replay)."""
    inst = W.star_tree_instances_2d()
    probs = [woi.Problem(p) for p, _, _ in inst]
    entries = [dict(problem=g, points=x, walks=w, M=4, seed=4242, precision=precision, schedule_mode=woi.SCHED_SHARED,
                    instance=i) for i, (g, (_, x, w)) in enumerate(zip(probs, inst))]
    cnt = woi.new_counters()
    woi.Batch(entries, counters=cnt).run()
    b = woi.Batch(entries)
    wall, ms = timed(torch, ev, lambda k, e: b.run(events=e), steps, warmup)
    counts = cnt.cpu().numpy().astype(float)
    se = [o[1].cpu().numpy() for o in b.outputs]
    mean = [o[0].cpu().numpy() for o in b.outputs]
    return {"wall": wall, "ms": ms, "counts": counts, "se": se, "mean": mean,
            "points": sum(x.shape[0] for _, x, _ in inst), "walkers": sum(x.shape[0] * w for _, x, w in inst)}


def batch_block(woi, torch, W, ev, steps):
    import numpy as np
    b32 = run_batch(woi, torch, W, woi.FP32, steps, 1, ev)
    b64 = run_batch(woi, torch, W, woi.FP64, 1, 0, ev)
    # fixed SE per instance: median SE of the FP64 batch, time rescaled by the mean SE^2 ratio
    bt32 = b32["wall"] * np.mean([np.mean(a ** 2) / np.median(c) ** 2 for a, c in zip(b32["se"], b64["se"])])
    bt64 = b64["wall"] * np.mean([np.mean(c ** 2) / np.median(c) ** 2 for c in b64["se"]])
    z = np.concatenate([(a - c) / s for a, c, s in zip(b32["mean"], b64["mean"], b64["se"])])
    kms = float(np.mean(b32["ms"]))
    bfl = flops_of(b32["counts"])
    return {
        "workload": "512 independent 2D instances: 1-16 circle/512-vertex star interfaces in random nesting trees, "
                    "sigma 10^U(-1,3), P = 2^U(4,10), W = 10^U(3,6), M = 4; one persistent graph launch",
        "points": b32["points"], "walkers": b32["walkers"],
        "walk_steps_per_s": b32["counts"][0] / b32["wall"], "ms_per_step": b32["wall"] * 1e3, "graph_ms": kms,
        "fp64_walk_steps_per_s": b64["counts"][0] / b64["wall"], "fp64_ms_per_step": b64["wall"] * 1e3,
        "speedup_fp32_vs_fp64_fixed_se": bt64 / bt32,
        "fp32_vs_fp64_paired_z": {"mean_z": float(np.mean(z)), "mean_abs_z": float(np.mean(np.abs(z))),
                                  "max_abs_z": float(np.max(np.abs(z)))},
        "roofline": {"bound": "alu", "achieved": bfl / (kms * 1e-3) / 1e12, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": bfl / (kms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "batch_kernel<float, 2, false, false, WV, true> + fill + reduce (graph)",
                     "counts_per_launch": {n: float(v) for n, v in zip(woi.COUNTER_NAMES, b32["counts"])}}}


def cpu_baseline(prob, pts, walks, M, budget_s):
    import numpy as np
    from oracle import oracle as O
    threads = min(16, os.cpu_count() or 1)
    op = O.OracleProblem(prob)
    idx = np.linspace(0, len(pts) - 1, 64).astype(int)
    t = time.perf_counter()
    _, _, _, _, c = O.estimate(op, pts[idx], 2000, M, seed=5, schedule_mode=1, threads=threads, groups=idx)
    rate = c["walk_steps"] / (time.perf_counter() - t)
    # points spread over the set, each with the full W, sized to the time budget
    n_pts = int(max(threads, min(len(pts), budget_s * rate / (walks * (M + 1)))))
    idx = np.linspace(0, len(pts) - 1, n_pts).astype(int)
    t = time.perf_counter()
    _, _, _, _, c = O.estimate(op, pts[idx], walks, M, seed=6, schedule_mode=1, threads=threads, groups=idx)
    dt = time.perf_counter() - t
    return {"value": c["walk_steps"] / dt, "unit": "walk-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_pts} of the 4096 points spread over the set, W = {walks} walkers each, FP64 oracle, "
                      f"{c['walk_steps']} walker-steps in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--walks", type=int, default=100000)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="measure only the headline path (skip shared trajectories, the instance batch, 3D and 6D)")
    ap.add_argument("--extra-steps", type=int, default=2, help="timed steps of the other configurations")
    ap.add_argument("--blocks", default="all",
                    help="comma-separated other configurations to run (shared_trajectories, batched_star_tree_instances, "
                         "ellipsoid_tree_3d_vr, nested_spheres_6d, point_charge_ellipsoids, mesh_tree_3d, "
                         "naive_markov_trees), default all")
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after the run, copy this many bytes device-to-device three times (a plain copy "
                         "kernel of known size, to scale the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the walk ranges would shard with one all-reduce of per-point sums)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2508_16767_amd import woi

    torch.cuda.set_device(0)
    ev = HipEvents()
    prob_desc, pts_np = W.star_tree_2d()
    M = 4
    prob = woi.Problem(prob_desc)
    woi._lib.woi_problem_upload(prob.handle)
    pts = torch.tensor(pts_np, dtype=torch.float64, device="cuda")
    P = pts.shape[0]

    # headline: FP32 walks through the persistent batched graph; an untimed graph of the
    # counting kernel on the same workload gives the event counts
    cnt = woi.new_counters()
    BatchPath(woi, torch, prob, pts, args.walks, M, woi.FP32, seed0=999, counters=cnt)(0)
    c32 = cnt.cpu().numpy().astype(float)
    r32 = BatchPath(woi, torch, prob, pts, args.walks, M, woi.FP32).run(ev, args.steps, args.warmup)
    # FP64 plain: the per-point walk kernel in FP64
    p64 = Path(woi, torch, prob, pts, args.walks, M, woi.FP64)
    c64 = p64.counts()
    r64 = p64.run(ev, args.fp64_steps, min(args.warmup, 1))
    # FP32 per-point walk kernel (same samples, one launch per estimate)
    pp = Path(woi, torch, prob, pts, args.walks, M, woi.FP32)
    cpp = pp.counts()
    rpp = pp.run(ev, args.steps, args.warmup)

    eps = float(np.median(r64["se"]))                  # fixed SE: median per-point SE of FP64 plain
    t32_eps, t64_eps = fixed_se(r32, eps), fixed_se(r64, eps)
    kern_ms = float(np.mean(r32["ms"]))
    flops = flops_of(c32)
    achieved = flops / (kern_ms * 1e-3) / 1e12
    kern64_ms = float(np.mean(r64["ms"]))
    kpp_ms = float(np.mean(rpp["ms"]))
    rec = {
        "metric": METRIC,
        "value": c32[0] / r32["wall"],
        "unit": "walk-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["wall"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D tree: unit disk, 3 nested 2048-vertex star polylines (k=3,5,7) + 5 circles, "
                               "sigma 10^U(-1,2), 5-mode Fourier jump data; 4096 points (25% within 1e-3 of an "
                               "interface); W=1e5 walkers, M=4; values + gradients",
                   "points": P, "walkers": args.walks, "M": M, "estimator": "plain", "schedule": "shared",
                   "precision": "FP32 walks, FP64 per-point sums",
                   "path": "persistent batched graph launch (woi_estimate_batch, one instance, tuned shape)"},
        "eval_points_per_s_fixed_se": P / t32_eps,
        "fixed_se": eps,
        "fp64_plain": {"walk_steps_per_s": c64[0] / r64["wall"], "ms_per_step": r64["wall"] * 1e3,
                       "eval_points_per_s_fixed_se": P / t64_eps, "walk_kernel_ms": kern64_ms,
                       "fp64_tflops": flops_of(c64) / (kern64_ms * 1e-3) / 1e12},
        "speedup_fp32_vs_fp64_fixed_se": t64_eps / t32_eps,
        "fp32_vs_fp64_paired_z": paired(r32, r64),
        "graph_ms": kern_ms,
        "fp32_per_point": {"walk_steps_per_s": cpp[0] / rpp["wall"], "ms_per_step": rpp["wall"] * 1e3,
                           "walk_kernel_ms": kpp_ms, "speedup_vs_fp64_plain_fixed_se": t64_eps / fixed_se(rpp, eps),
                           "tflops": flops_of(cpp) / (kpp_ms * 1e-3) / 1e12,
                           "traffic": TRAFFIC_BYTES if args.walks == 100000 else None},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": BATCH_TRAFFIC_BYTES if args.walks == 100000 else None,
                     "kernel": "batch_kernel<float, 2, false, false, WV, true> (FP32, 2D, plain, LDS-staged polylines; "
                               "time over the whole graph: fill + persistent kernel + reduction)",
                     "flops_per_launch": flops,
                     "counts_per_launch": {n: float(v) for n, v in zip(woi.COUNTER_NAMES, c32)}},
    }
    blocks = set(args.blocks.split(",")) if args.blocks != "all" else None

    def want(name):
        return not args.no_extra and (blocks is None or name in blocks)

    B = 16                                              # <= 0.5 % of the 4096 points
    if want("shared_trajectories"):
        rsh = Path(woi, torch, prob, pts, args.walks, M, woi.FP32, 0, B).run(ev, args.steps, args.warmup)
        pairs = P * args.walks * (M + 1)
        rec["shared_trajectories"] = {
            "batch_share": B, "walk_steps_per_s": pairs / rsh["wall"], "ms_per_step": rsh["wall"] * 1e3,
            "traj_plus_eval_ms": float(np.mean(rsh["ms"])),
            "eval_points_per_s_fixed_se": P / fixed_se(rsh, eps),
            "speedup_vs_fp64_plain_fixed_se": t64_eps / fixed_se(rsh, eps),
            "pair_eval_tflops_over_traj_plus_eval":
                pairs * eval_flops_per_pair(2) / (float(np.mean(rsh["ms"])) * 1e-3) / 1e12}
    if want("batched_star_tree_instances"):
        rec["batched_star_tree_instances"] = batch_block(woi, torch, W, ev, args.extra_steps)
    if want("ellipsoid_tree_3d_vr"):
        p4, x4 = W.ellipsoid_tree_3d()
        rec["ellipsoid_tree_3d_vr"] = config_block(
            woi, torch, ev, "unit ball, spheres 0.6 > 0.3, 10 ellipsoids (semi-axes 0.03-0.08), sigma 10^U(log .5, "
            "log 50), real SH l <= 4 data; 16384 points; VR, W = 1e5 walkers, M = 6", p4, x4, 100000, 6, 1, 64,
            args.extra_steps)
    if want("nested_spheres_6d"):
        p5, x5 = W.nested_spheres_6d()
        rec["nested_spheres_6d"] = config_block(
            woi, torch, ev, "unit 6-ball, spheres 0.7 > 0.35, sigma (1, 5, 0.2), c + lambda x1/|x| data; 1024 points; "
            "W = 1e6, M = 8", p5, x5, 1000000, 8, 0, 4, args.extra_steps)
    if want("point_charge_ellipsoids"):
        # three nested ellipsoids around the potential |x|^(2-m) of a point charge, m = 3..6
        # (1e4 points; M = m + 2 as the paper walks them; W = 2e5 keeps the run short, the rates
        # do not depend on W)
        rec["point_charge_ellipsoids"] = {}
        for m in (3, 4, 5, 6):
            pm, xm = W.point_charge_ellipsoids(m)
            rec["point_charge_ellipsoids"][f"{m}d"] = config_block(
                woi, torch, ev, f"{m}D: 3 nested ellipsoids (centres 1.3/1.4/1.6 e1), sigma (1.1, 1.3, 0.9), data "
                f"from u = |x|^(2-m); 10000 points; W = 2e5, M = {m + 2}", pm, xm, 200000, m + 2, 0, 32,
                args.extra_steps)
    if want("mesh_tree_3d"):
        # triangle-mesh interfaces (BVH line/ray hits over 1280 triangles per mesh)
        p6, x6 = W.mesh_tree_3d()
        rec["mesh_tree_3d"] = config_block(
            woi, torch, ev, "3D: jittered icosphere (R 1, 1280 triangles) around a jittered icosphere (R 0.45, 1280 "
            "triangles) and a sphere; sigma (1, 4, 0.5); quadratic direction-polynomial data; 4096 points; W = 2e4, "
            "M = 4", p6, x6, 20000, 4, 0, 16, args.extra_steps)
    if want("naive_markov_trees"):
        rec["naive_markov_trees"] = naive_block(woi, torch, ev, prob, pts, args.extra_steps)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(prob_desc, pts_np, args.walks, M, args.cpu_seconds)
    print(json.dumps(rec), flush=True)
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
