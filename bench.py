#!/usr/bin/env python3
"""Walk-on-Interfaces benchmark on one MI355X.

Workload (the 2D tree configuration): unit disk containing 3 nested star interfaces
r0 (1 + 0.2 cos k t) with (r0, k) = (0.7, 3), (0.4, 5), (0.2, 7) as 2048-vertex polylines
and 5 circular inclusions (N = 9 regions, depth 3), sigma = 10^U(-1, 2), 5-mode random
Fourier flux data with zero mean; 4096 evaluation points (25 % within 1e-3 of an
interface); W = 1e5 walkers per point, M = 4; values and gradients.

One step = one full estimate of all points: the walk kernel plus the per-point reduction,
inputs resident in HBM.  The headline path is FP32 walks with FP64 per-point sums and the
wave-uniform shared schedule; the FP64 plain path (same kernel in FP64) is measured for the
equal-standard-error comparison.  Prints one JSON line.
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

# Algorithmic FP work per event of the walk kernel (2D, counted from the kernel source; a
# transcendental counts as one flop, an FMA as two, compares and integer work count zero).
FLOPS_PER_WALKER_STEP = 29      # Phi + grad Phi + accumulation (19) and the Q/T/sign update (10)
FLOPS_PER_OTHER = 18            # uniform re-sample + |K*| |dOmega| factor
FLOPS_PER_NODE_TEST = 7         # signed distance of a block end vertex to the line (5) +- bound (2)
FLOPS_PER_SEGMENT_TEST = 5      # signed distance of the segment end vertex (crossings add ~10, rare)
FLOPS_PER_WALKER = 57           # step-0 datum b(y_0) (5-mode Fourier) and Q_0
PEAK_FP32_TFLOPS = 157.3        # MI355X vector FP32 (packed) peak
PEAK_HBM_GBS = 8000.0
# HBM bytes per launch of the timed FP32 walk kernel at W = 1e5, from the FETCH_SIZE and
# WRITE_SIZE passes in profiles/walk_kernel_config2_hbm_counters.md, scaled by what the same
# counters read for a 1 GiB device copy.  None whenever the kernel has changed since those
# passes were taken.
TRAFFIC_BYTES = None


class HipEvents:
    """hipEvent_t handles from libamdhip64 (events on the stream the kernels run on)."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

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


def run_path(woi, torch, prob, pts, walks, M, precision, steps, warmup, ev, seed0):
    """Untimed counting launch (same workload, its own seed) for the work counts, warm-up
    launches, then `steps` timed launches of the non-counting kernel."""
    P = pts.shape[0]
    out = (torch.empty(P, dtype=torch.float64, device="cuda"), torch.empty(P, dtype=torch.float64, device="cuda"),
           torch.empty(P, 2, dtype=torch.float64, device="cuda"), torch.empty(P, 2, dtype=torch.float64, device="cuda"))
    q = woi.make_query(walks, M, precision=precision, schedule_mode=woi.SCHED_SHARED)
    ws = torch.empty(woi.workspace_size(prob, P, q), dtype=torch.uint8, device="cuda")
    cnt = woi.new_counters()
    woi.estimate(prob, pts, walks, M, seed=seed0 + 999, precision=precision, schedule_mode=woi.SCHED_SHARED,
                 out=out, workspace=ws, counters=cnt)
    for w in range(warmup):
        woi.estimate(prob, pts, walks, M, seed=seed0 + 1000 + w, precision=precision, schedule_mode=woi.SCHED_SHARED,
                     out=out, workspace=ws)
    evs = [(ev.create(), ev.create()) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        woi.estimate(prob, pts, walks, M, seed=seed0 + k, precision=precision, schedule_mode=woi.SCHED_SHARED,
                     out=out, workspace=ws, events=evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [ev.ms(a, b) for a, b in evs]
    se = out[1].cpu().numpy()
    return wall, kern_ms, cnt.cpu().numpy().astype(float) * steps, se, out[0].cpu().numpy()


def timed(torch, ev, fn, steps, warmup):
    """Warm-up calls, then `steps` timed calls of fn(events); returns wall seconds and the
    per-call HIP-event milliseconds (events recorded by the library on the launch stream)."""
    for _ in range(warmup):
        fn(None)
    evs = [(ev.create(), ev.create()) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        fn(evs[k])
    torch.cuda.synchronize()
    return time.perf_counter() - t0, [ev.ms(a, b) for a, b in evs]


def run_shared(woi, torch, prob, pts, walks, M, B, steps, warmup, ev):
    """Config 2 with shared trajectories (Sec. 4.6): points p with equal p // B share one
    trajectory set.  Walk-steps here are (point, walk, step) contributions, as for the
    per-point path."""
    P = pts.shape[0]
    out = (torch.empty(P, dtype=torch.float64, device="cuda"), torch.empty(P, dtype=torch.float64, device="cuda"),
           torch.empty(P, 2, dtype=torch.float64, device="cuda"), torch.empty(P, 2, dtype=torch.float64, device="cuda"))
    q = woi.make_query(walks, M, precision=woi.FP32, schedule_mode=woi.SCHED_SHARED, batch_share=B)
    ws = torch.empty(woi.workspace_size(prob, P, q), dtype=torch.uint8, device="cuda")
    fn = lambda e: woi.estimate(prob, pts, walks, M, seed=77, precision=woi.FP32, schedule_mode=woi.SCHED_SHARED,
                                batch_share=B, out=out, workspace=ws, events=e)
    wall, ms = timed(torch, ev, fn, steps, warmup)
    return wall / steps, ms, out[1].cpu().numpy()


def run_batch(woi, torch, W, precision, steps, warmup, ev):
    """Config 3: 512 instances in one persistent graph launch (tuned launch shape).  An
    untimed graph of the counting kernel gives the event counts; the timed graph replays
    the non-counting kernel (same seed: the whole batch is recomputed every replay)."""
    inst = W.config3_instances()
    probs = [woi.Problem(p) for p, _, _ in inst]
    entries = [dict(problem=g, points=x, walks=w, M=4, seed=4242, precision=precision, schedule_mode=woi.SCHED_SHARED,
                    instance=i) for i, (g, (_, x, w)) in enumerate(zip(probs, inst))]
    cnt = woi.new_counters()
    woi.Batch(entries, counters=cnt).run()
    b = woi.Batch(entries)
    wall, ms = timed(torch, ev, lambda e: b.run(events=e), steps, warmup)
    counts = cnt.cpu().numpy().astype(float)
    se = [o[1].cpu().numpy() for o in b.outputs]
    return {"wall": wall / steps, "ms": ms, "counts": counts, "se": se,
            "points": sum(x.shape[0] for _, x, _ in inst), "walkers": sum(x.shape[0] * w for _, x, w in inst)}


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
                    help="measure only the headline path (skip config 3 batched and shared trajectories)")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
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
    prob_desc, pts_np = W.config2()
    M = 4
    prob = woi.Problem(prob_desc)
    woi._lib.woi_problem_upload(prob.handle)
    pts = torch.tensor(pts_np, dtype=torch.float64, device="cuda")
    P = pts.shape[0]
    ev = HipEvents()

    wall32, k32, c32, se32, _ = run_path(woi, torch, prob, pts, args.walks, M, woi.FP32, args.steps, args.warmup, ev, 1)
    wall64, k64, c64, se64, _ = run_path(woi, torch, prob, pts, args.walks, M, woi.FP64, args.fp64_steps,
                                         min(args.warmup, 1), ev, 101)

    steps32 = c32[0] / args.steps                     # walker-steps per step
    value = c32[0] / wall32
    value64 = c64[0] / wall64
    t32, t64 = wall32 / args.steps, wall64 / args.fp64_steps
    eps = float(np.median(se64))                      # fixed SE: median per-point SE of FP64 plain
    t32_eps = t32 * float(np.mean(se32 ** 2)) / eps ** 2
    t64_eps = t64 * float(np.mean(se64 ** 2)) / eps ** 2
    kern_ms = float(np.mean(k32))
    flops = flops_of(c32 / args.steps)
    achieved = flops / (kern_ms * 1e-3) / 1e12
    kern64_ms = float(np.mean(k64))
    flops64 = flops_of(c64 / args.fp64_steps)
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "walk-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D tree: unit disk, 3 nested 2048-vertex star polylines (k=3,5,7) + 5 circles, "
                               "sigma 10^U(-1,2), 5-mode Fourier jump data; 4096 points (25% within 1e-3 of an "
                               "interface); W=1e5 walkers, M=4; values + gradients",
                   "points": P, "walkers": args.walks, "M": M, "estimator": "plain", "schedule": "shared",
                   "precision": "FP32 walks, FP64 per-point sums"},
        "eval_points_per_s_fixed_se": P / t32_eps,
        "fixed_se": eps,
        "fp64_plain": {"walk_steps_per_s": value64, "ms_per_step": t64 * 1e3,
                       "eval_points_per_s_fixed_se": P / t64_eps, "walk_kernel_ms": kern64_ms,
                       "fp64_tflops": flops64 / (kern64_ms * 1e-3) / 1e12},
        "speedup_fp32_vs_fp64_fixed_se": t64_eps / t32_eps,
        "walk_kernel_ms": kern_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": TRAFFIC_BYTES if args.walks == 100000 else None,
                     "kernel": "walk_kernel<float, 2, false, false, true> (FP32, 2D, plain, LDS-staged polylines)",
                     "flops_per_launch": flops,
                     "counts_per_launch": {n: float(v / args.steps) for n, v in zip(woi.COUNTER_NAMES, c32)}},
    }
    if not args.no_extra:
        B = 16                                            # <= 0.5 % of the 4096 points
        t_sh, ms_sh, se_sh = run_shared(woi, torch, prob, pts, args.walks, M, B, args.steps, args.warmup, ev)
        t_sh_eps = t_sh * float(np.mean(se_sh ** 2)) / eps ** 2
        rec["shared_trajectories"] = {
            "batch_share": B, "walk_steps_per_s": P * args.walks * (M + 1) / t_sh, "ms_per_step": t_sh * 1e3,
            "traj_plus_eval_ms": float(np.mean(ms_sh)), "eval_points_per_s_fixed_se": P / t_sh_eps,
            "speedup_vs_fp64_plain_fixed_se": t64_eps / t_sh_eps}
        b32 = run_batch(woi, torch, W, woi.FP32, args.batch_steps, 1, ev)
        b64 = run_batch(woi, torch, W, woi.FP64, 1, 0, ev)
        # fixed SE per instance: median SE of the FP64 batch; points/s at that SE summed over instances
        bt32 = b32["wall"] * np.mean([np.mean(a ** 2) / np.median(c) ** 2 for a, c in zip(b32["se"], b64["se"])])
        bt64 = b64["wall"] * np.mean([np.mean(c ** 2) / np.median(c) ** 2 for c in b64["se"]])
        kms = float(np.mean(b32["ms"]))
        bfl = flops_of(b32["counts"])
        rec["batched_config3"] = {
            "workload": "512 independent 2D instances: 1-16 circle/512-vertex star interfaces in random nesting "
                        "trees, sigma 10^U(-1,3), P = 2^U(4,10), W = 10^U(3,6), M = 4; one persistent graph launch",
            "points": b32["points"], "walkers": b32["walkers"],
            "walk_steps_per_s": b32["counts"][0] / b32["wall"], "ms_per_step": b32["wall"] * 1e3,
            "graph_ms": kms, "fp64_walk_steps_per_s": b64["counts"][0] / b64["wall"],
            "fp64_ms_per_step": b64["wall"] * 1e3,
            "speedup_fp32_vs_fp64_fixed_se": bt64 / bt32,
            "roofline": {"bound": "alu", "achieved": bfl / (kms * 1e-3) / 1e12, "peak": PEAK_FP32_TFLOPS,
                         "unit": "TFLOP/s", "frac": bfl / (kms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, "traffic": None,
                         "kernel": "batch_kernel<float, 2, false, false, WV, true> + fill + reduce (graph)",
                         "counts_per_launch": {n: float(v) for n, v in zip(woi.COUNTER_NAMES, b32["counts"])}}}
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
