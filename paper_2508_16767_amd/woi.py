"""Python binding of libwoi.so (include/woi.h): argument marshalling only.

Every step of the estimator runs in the HIP kernels behind the C ABI; this module
only converts problem descriptions to the C structs, allocates device buffers with
PyTorch (device memory and streams are PyTorch's job here) and passes pointers.
If the native library is missing the import fails: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libwoi.so")

MAX_DIM, MAX_REGIONS, MAX_M, N_COUNTERS = 8, 32, 32, 9
PLAIN, VR, NAIVE = 0, 1, 2   # estimators: Alg. 2, Alg. 3, naive Markov trees (Sec. 4.2)
FP64, FP32 = 0, 1
SCHED_PER_GROUP, SCHED_SHARED = 0, 1
COUNTER_NAMES = ("walker_steps", "redraws", "rejections", "cap_hits", "zero_distance", "node_tests",
                 "segment_tests", "other_transitions", "fp64_fallbacks")


class WoiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status}: {msg}")
        self.status = status


class _Shape(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_vertices", C.c_int), ("center", C.c_double * MAX_DIM),
                ("radius", C.c_double), ("A", C.POINTER(C.c_double)), ("vertices", C.POINTER(C.c_double)),
                ("n_triangles", C.c_int), ("triangles", C.POINTER(C.c_int))]


class _Data(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_terms", C.c_int), ("center", C.c_double * MAX_DIM),
                ("coef", C.POINTER(C.c_double)), ("exps", C.POINTER(C.c_uint8))]


class _Desc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_regions", C.c_int), ("parent", C.POINTER(C.c_int)),
                ("sigma", C.POINTER(C.c_double)), ("shapes", C.POINTER(_Shape)), ("data", C.POINTER(_Data)),
                ("compat_mode", C.c_int), ("compat_tol", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_regions", C.c_int), ("alpha_l1", C.c_double),
                ("alpha", C.c_double * MAX_REGIONS), ("beta_scale", C.c_double * MAX_REGIONS),
                ("area", C.c_double * MAX_REGIONS), ("area_plus", C.c_double * MAX_REGIONS),
                ("area_minus", C.c_double * MAX_REGIONS), ("flux", C.c_double * MAX_REGIONS),
                ("device_bytes", C.c_size_t)]


class Query(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("walks", C.c_uint64), ("walk_offset", C.c_uint64), ("M", C.c_int),
                ("estimator", C.c_int), ("precision", C.c_int), ("schedule_mode", C.c_int),
                ("batch_share", C.c_int), ("instance", C.c_uint32), ("samples_per_thread", C.c_int),
                ("block_size", C.c_int), ("event_begin", C.c_void_p), ("event_end", C.c_void_p)]


class _BatchItem(C.Structure):
    _fields_ = [("problem", C.c_void_p), ("points", C.c_void_p), ("P", C.c_int64), ("query", Query),
                ("mean", C.c_void_p), ("se", C.c_void_p), ("grad", C.c_void_p), ("grad_se", C.c_void_p)]


class _TrainSpec(C.Structure):
    _fields_ = [("grid_n", C.c_int), ("bc_n", C.c_int), ("margin", C.c_double)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("walker_steps", "redraws", "rejections", "cap_hits", "zero_distances",
                                          "search_node_tests", "segment_tests", "other_transitions",
                                          "fp64_fallbacks")] + [("seconds", C.c_double)]


EXPORTS = ("woi_problem_create", "woi_problem_upload", "woi_problem_destroy", "woi_problem_get_info", "woi_workspace_size",
           "woi_estimate", "woi_estimate_noalloc", "woi_trace", "woi_batch_workspace_size", "woi_estimate_batch",
           "woi_stats_read", "woi_training_points",
           "woi_status_string", "woi_last_error")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2508_16767_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    lib.woi_problem_create.argtypes = [C.POINTER(_Desc), C.POINTER(C.c_void_p)]
    lib.woi_problem_destroy.argtypes = [C.c_void_p]
    lib.woi_problem_upload.argtypes = [C.c_void_p]
    lib.woi_problem_destroy.restype = None
    lib.woi_problem_get_info.argtypes = [C.c_void_p, C.POINTER(_Info)]
    lib.woi_workspace_size.argtypes = [C.c_void_p, C.c_int64, C.POINTER(Query), C.POINTER(C.c_size_t)]
    lib.woi_estimate.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(Query), C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]
    lib.woi_estimate_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(Query), C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.woi_trace.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(Query), C.c_uint64, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p]
    lib.woi_batch_workspace_size.argtypes = [C.POINTER(_BatchItem), C.c_int, C.POINTER(C.c_size_t)]
    lib.woi_estimate_batch.argtypes = [C.POINTER(_BatchItem), C.c_int, C.c_void_p, C.c_size_t, C.c_void_p,
                                       C.c_void_p]
    lib.woi_stats_read.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Stats)]
    lib.woi_training_points.argtypes = [C.c_void_p, C.POINTER(_TrainSpec), C.c_void_p, C.c_int64,
                                        C.POINTER(C.c_int64), C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.POINTER(C.c_int64), C.c_void_p]
    lib.woi_status_string.restype = C.c_char_p
    lib.woi_status_string.argtypes = [C.c_int]
    lib.woi_last_error.restype = C.c_char_p
    return lib


_lib = _load()


def _check(rc):
    if rc != 0:
        raise WoiError(_lib.woi_status_string(rc).decode(), _lib.woi_last_error().decode())


def _dptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Problem:
    """A compiled problem on the current device.

    `desc` is any object with attributes dim, parent, sigma, shapes, data, compat_mode (and
    optionally compat_tol, used when the argument is None):
    shapes[i] has kind (0 sphere, 1 ellipsoid, 2 polyline), center, radius, A, vertices;
    data[i] has kind (0 zero, 1 Fourier, 2 direction polynomial, 3 source flux,
    4 field flux), center, coef, exps -- the fields of woi_shape / woi_data in woi.h.
    """

    def __init__(self, desc, compat_tol=None):
        if compat_tol is None:
            compat_tol = float(getattr(desc, "compat_tol", 1e-8))
        m, N = int(desc.dim), len(desc.parent)
        self.dim, self.N = m, N
        keep = []
        parent = np.ascontiguousarray(desc.parent, dtype=np.int32)
        sigma = np.ascontiguousarray(desc.sigma, dtype=np.float64)
        keep += [parent, sigma]
        shapes = (_Shape * N)()
        datas = (_Data * N)()
        for i, (s, d) in enumerate(zip(desc.shapes, desc.data)):
            shapes[i].kind = int(s.kind)
            c = np.zeros(MAX_DIM); c[:m] = np.asarray(s.center, dtype=np.float64)[:m]
            shapes[i].center[:] = list(c)
            shapes[i].radius = float(getattr(s, "radius", 0.0) or 0.0)
            A = getattr(s, "A", None)
            if A is not None:
                A = np.ascontiguousarray(A, dtype=np.float64).reshape(-1); keep.append(A)
                shapes[i].A = _dptr(A, C.c_double)
            v = getattr(s, "vertices", None)
            if v is not None:
                v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1); keep.append(v)
                shapes[i].vertices = _dptr(v, C.c_double)
                shapes[i].n_vertices = len(v) // (3 if int(s.kind) == 3 else 2)
            t = getattr(s, "triangles", None)
            if t is not None:
                t = np.ascontiguousarray(t, dtype=np.int32).reshape(-1); keep.append(t)
                shapes[i].triangles = _dptr(t, C.c_int)
                shapes[i].n_triangles = len(t) // 3
            datas[i].kind = int(d.kind)
            dc = np.zeros(MAX_DIM); dc[:m] = np.asarray(d.center, dtype=np.float64).reshape(-1)[:m]
            datas[i].center[:] = list(dc)
            coef = np.ascontiguousarray(d.coef, dtype=np.float64).reshape(-1)
            keep.append(coef)
            if coef.size:
                datas[i].coef = _dptr(coef, C.c_double)
            if int(d.kind) == 1:
                datas[i].n_terms = (coef.size - 1) // 2
            else:
                datas[i].n_terms = coef.size
            ex = getattr(d, "exps", None)
            if ex is not None:
                ex = np.ascontiguousarray(ex, dtype=np.uint8).reshape(-1); keep.append(ex)
                datas[i].exps = _dptr(ex, C.c_uint8)
        desc_c = _Desc(m, N, _dptr(parent, C.c_int), _dptr(sigma, C.c_double), shapes, datas,
                       int(getattr(desc, "compat_mode", 0)), float(compat_tol))
        h = C.c_void_p()
        _check(_lib.woi_problem_create(C.byref(desc_c), C.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            try:
                _lib.woi_problem_destroy(h)
            except Exception:
                pass
            self.handle = None

    def info(self):
        inf = _Info()
        _check(_lib.woi_problem_get_info(self.handle, C.byref(inf)))
        N = self.N
        out = {k: np.array(getattr(inf, k)[:N]) for k in
               ("alpha", "beta_scale", "area", "area_plus", "area_minus", "flux")}
        out["alpha_l1"] = inf.alpha_l1
        out["device_bytes"] = inf.device_bytes
        return out


def make_query(walks, M, seed=0, estimator=PLAIN, precision=FP64, schedule_mode=SCHED_PER_GROUP,
               batch_share=1, walk_offset=0, instance=0, samples_per_thread=0, block_size=0, events=None):
    ev = events if events is not None else (None, None)
    return Query(int(seed), int(walks), int(walk_offset), int(M), int(estimator), int(precision),
                 int(schedule_mode), int(batch_share), int(instance), int(samples_per_thread), int(block_size),
                 ev[0], ev[1])


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _points(points, dim):
    x = torch.as_tensor(points, dtype=torch.float64)
    if not x.is_cuda:
        x = x.cuda()
    return x.reshape(-1, dim).contiguous()


def workspace_size(problem, P, q):
    n = C.c_size_t()
    _check(_lib.woi_workspace_size(problem.handle, int(P), C.byref(q), C.byref(n)))
    return n.value


def estimate(problem, points, walks, M, seed=0, estimator=PLAIN, precision=FP64, schedule_mode=SCHED_PER_GROUP,
             batch_share=1, walk_offset=0, instance=0, samples_per_thread=0, block_size=0, counters=None,
             out=None, workspace=None, events=None):
    """Per-point mean, SE, gradient, gradient SE as CUDA float64 tensors (asynchronous).
    events: optional (hipEvent_t, hipEvent_t) handles recorded around the walk kernel."""
    x = _points(points, problem.dim)
    P = x.shape[0]
    q = make_query(walks, M, seed, estimator, precision, schedule_mode, batch_share, walk_offset, instance,
                   samples_per_thread, block_size, events)
    if out is None:
        out = (torch.empty(P, dtype=torch.float64, device=x.device), torch.empty(P, dtype=torch.float64, device=x.device),
               torch.empty(P, problem.dim, dtype=torch.float64, device=x.device),
               torch.empty(P, problem.dim, dtype=torch.float64, device=x.device))
    nbytes = workspace_size(problem, P, q)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 8), dtype=torch.uint8, device=x.device)
    mean, se, g, gse = out
    _check(_lib.woi_estimate(problem.handle, C.c_void_p(x.data_ptr()), P, C.byref(q), C.c_void_p(mean.data_ptr()),
                             C.c_void_p(se.data_ptr()), C.c_void_p(g.data_ptr()), C.c_void_p(gse.data_ptr()),
                             C.c_void_p(workspace.data_ptr()), workspace.numel(),
                             C.c_void_p(counters.data_ptr()) if counters is not None else None, _stream()))
    return mean, se, g, gse


def estimate_noalloc(problem, points, walks, M, seed=0, estimator=PLAIN, precision=FP64,
                     schedule_mode=SCHED_PER_GROUP, walk_offset=0, instance=0, counters=None, out=None):
    """woi_estimate_noalloc: the per-point estimate with the library's own fixed partial-sum
    array (no workspace; the problem must be uploaded first).  Returns (mean, se, grad, grad_se)."""
    x = _points(points, problem.dim)
    P = x.shape[0]
    q = make_query(walks, M, seed, estimator, precision, schedule_mode, 1, walk_offset, instance)
    if out is None:
        out = (torch.empty(P, dtype=torch.float64, device=x.device), torch.empty(P, dtype=torch.float64, device=x.device),
               torch.empty(P, problem.dim, dtype=torch.float64, device=x.device),
               torch.empty(P, problem.dim, dtype=torch.float64, device=x.device))
    mean, se, g, gse = out
    _check(_lib.woi_estimate_noalloc(problem.handle, C.c_void_p(x.data_ptr()), P, C.byref(q),
                                     C.c_void_p(mean.data_ptr()), C.c_void_p(se.data_ptr()), C.c_void_p(g.data_ptr()),
                                     C.c_void_p(gse.data_ptr()),
                                     C.c_void_p(counters.data_ptr()) if counters is not None else None, _stream()))
    return mean, se, g, gse


def upload(problem):
    """woi_problem_upload: copy the compiled problem to the current device now."""
    _check(_lib.woi_problem_upload(problem.handle))


def trace(problem, points, n_samples, M, seed=0, estimator=PLAIN, precision=FP64, schedule_mode=SCHED_PER_GROUP,
          batch_share=1, walk_offset=0, instance=0):
    """Per-walker values F[P, n, K], gradients G[P, n, K, dim] and decision words T[P, n, K, M+1].
    For the naive estimator: one value per tree (K = 1) and no decision words (T is None)."""
    x = _points(points, problem.dim)
    P = x.shape[0]
    K = 2 if estimator == VR else 1
    F = torch.zeros(P, n_samples, K, dtype=torch.float64, device=x.device)
    G = torch.zeros(P, n_samples, K, problem.dim, dtype=torch.float64, device=x.device)
    T = torch.zeros(P, n_samples, K, M + 1, dtype=torch.int32, device=x.device)
    q = make_query(2 * n_samples if estimator == VR else n_samples, M, seed, estimator, precision, schedule_mode,
                   batch_share, walk_offset, instance)
    if estimator == NAIVE:
        T = None
    _check(_lib.woi_trace(problem.handle, C.c_void_p(x.data_ptr()), P, C.byref(q), int(n_samples),
                          C.c_void_p(F.data_ptr()), C.c_void_p(G.data_ptr()),
                          C.c_void_p(None if T is None else T.data_ptr()), _stream()))
    return F, G, T


class Batch:
    """Instances estimated together by woi_estimate_batch (one persistent launch, replayed
    as a cached HIP graph).  `entries` is a list of dicts with keys problem, points, walks,
    M and optionally seed, estimator, precision, schedule_mode, batch_share, walk_offset, instance.  The
    object keeps the points, the outputs and the workspace alive: the graph reads and
    writes them on every run()."""

    def __init__(self, entries, block_size=0, counters=None):
        n = len(entries)
        self.items = (_BatchItem * n)()
        self.points, self.outputs = [], []
        self.counters = counters
        for i, e in enumerate(entries):
            prob = e["problem"]
            x = _points(e["points"], prob.dim)
            P = x.shape[0]
            out = (torch.empty(P, dtype=torch.float64, device=x.device), torch.empty(P, dtype=torch.float64, device=x.device),
                   torch.empty(P, prob.dim, dtype=torch.float64, device=x.device),
                   torch.empty(P, prob.dim, dtype=torch.float64, device=x.device))
            q = make_query(e["walks"], e["M"], e.get("seed", 0), e.get("estimator", PLAIN), e.get("precision", FP64),
                           e.get("schedule_mode", SCHED_SHARED), e.get("batch_share", 1), e.get("walk_offset", 0),
                           e.get("instance", 0), 0, block_size)
            it = self.items[i]
            it.problem, it.points, it.P, it.query = prob.handle, x.data_ptr(), P, q
            it.mean, it.se, it.grad, it.grad_se = (t.data_ptr() for t in out)
            self.points.append(x)
            self.outputs.append(out)
        self.problems = [e["problem"] for e in entries]
        nbytes = C.c_size_t()
        _check(_lib.woi_batch_workspace_size(self.items, n, C.byref(nbytes)))
        self.workspace = torch.empty(max(nbytes.value, 8), dtype=torch.uint8, device="cuda")

    def run(self, events=None, seed=None):
        """Enqueue the batch on the current stream; returns the list of (mean, se, grad, grad_se).
        seed: if given, every item's seed for this and later runs (the cached graph is reused)."""
        if seed is not None:
            for it in self.items:
                it.query.seed = int(seed)
        q0 = self.items[0].query
        q0.event_begin, q0.event_end = events if events is not None else (None, None)
        cnt = C.c_void_p(self.counters.data_ptr()) if self.counters is not None else None
        _check(_lib.woi_estimate_batch(self.items, len(self.items), C.c_void_p(self.workspace.data_ptr()),
                                       self.workspace.numel(), cnt, _stream()))
        return self.outputs


def estimate_batch(entries, block_size=0, counters=None):
    """One batched estimate of every entry (see Batch)."""
    return Batch(entries, block_size, counters).run()


def training_points(problem, grid_n, margin=0.0, bc_n=0, cap=None):
    """woi_training_points: surrogate training data of Sec. 5 on the device -- interior grid points
    inside dOmega (clear of the interfaces by `margin`), and boundary points, outward normals and
    b_1 / sigma_1 targets.  Returns (interior [n, dim], bc_points, bc_normals, bc_flux) tensors."""
    m = problem.dim
    spec = _TrainSpec(int(grid_n), int(bc_n), float(margin))
    if cap is None:
        cap = 1
        for _ in range(m):
            cap *= int(grid_n)
    nb = (bc_n if m == 2 else 2 * bc_n * bc_n) if bc_n else 0
    x = torch.empty(max(cap, 1), m, dtype=torch.float64, device="cuda")
    yb = torch.empty(max(nb, 1), m, dtype=torch.float64, device="cuda")
    nr = torch.empty(max(nb, 1), m, dtype=torch.float64, device="cuda")
    fl = torch.empty(max(nb, 1), dtype=torch.float64, device="cuda")
    n_in, n_bc = C.c_int64(), C.c_int64()
    _check(_lib.woi_training_points(problem.handle, C.byref(spec), C.c_void_p(x.data_ptr()), int(cap), C.byref(n_in),
                                    C.c_void_p(yb.data_ptr()) if nb else None, C.c_void_p(nr.data_ptr()) if nb else None,
                                    C.c_void_p(fl.data_ptr()) if nb else None, C.byref(n_bc), _stream()))
    return x[:min(n_in.value, cap)], yb[:nb], nr[:nb], fl[:nb], n_in.value


def new_counters(device="cuda"):
    return torch.zeros(N_COUNTERS, dtype=torch.int64, device=device)


def stats(counters=None, events=None):
    """woi_stats_read: the counters (a new_counters() tensor) and the seconds between two events
    recorded by a call (-1 without events), as a dict."""
    st = Stats()
    ev = events if events is not None else (None, None)
    _check(_lib.woi_stats_read(C.c_void_p(counters.data_ptr()) if counters is not None else None,
                               C.c_void_p(ev[0]) if ev[0] else None, C.c_void_p(ev[1]) if ev[1] else None,
                               C.byref(st)))
    return {f: getattr(st, f) for f, _ in Stats._fields_}
