"""ctypes wrapper of the FP64 CPU oracle (oracle/woi_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU-baseline
leg of the benchmark.  The product path never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "woi_oracle.c")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, -O2, no fast-math)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(_SRC):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC,
                               "-lm", "-lpthread"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _In(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_regions", C.c_int),
                ("parent", C.POINTER(C.c_int)), ("sigma", C.POINTER(C.c_double)),
                ("shape_kind", C.POINTER(C.c_int)), ("center", C.POINTER(C.c_double)),
                ("radius", C.POINTER(C.c_double)), ("A", C.POINTER(C.c_double)),
                ("n_vertices", C.POINTER(C.c_int)), ("vertex_offset", C.POINTER(C.c_int64)),
                ("vertices", C.POINTER(C.c_double)), ("data_kind", C.POINTER(C.c_int)),
                ("data_center", C.POINTER(C.c_double)), ("n_terms", C.POINTER(C.c_int)),
                ("coef_offset", C.POINTER(C.c_int64)), ("coef", C.POINTER(C.c_double)),
                ("exps", C.POINTER(C.c_ubyte)),
                ("n_triangles", C.POINTER(C.c_int)), ("mesh_vertex_offset", C.POINTER(C.c_int64)),
                ("mesh_vertices", C.POINTER(C.c_double)), ("triangle_offset", C.POINTER(C.c_int64)),
                ("triangles", C.POINTER(C.c_int))]


class _Query(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("walks", C.c_uint64), ("walk_offset", C.c_uint64),
                ("M", C.c_int), ("estimator", C.c_int), ("schedule_mode", C.c_int),
                ("batch_share", C.c_int), ("instance", C.c_uint32)]


class _Counters(C.Structure):
    _fields_ = [("walks", C.c_uint64), ("walk_steps", C.c_uint64), ("redraws", C.c_uint64),
                ("rejections", C.c_uint64), ("cap_hits", C.c_uint64), ("zero_dist", C.c_uint64)]


_lib = None


def build_variant(plant: int, outdir: str) -> str:
    """Build a deliberately wrong oracle (OR_PLANT = plant) for the tests that show the
    pins reject it; never used for reference values."""
    path = os.path.join(outdir, f"liboracle_plant{plant}.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", f"-DOR_PLANT={plant}", "-o", path,
                           _SRC, "-lm", "-lpthread"])
    return path


def load(path):
    _l = C.CDLL(path)
    _declare(_l)
    return _l


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _declare(_lib)
    return _lib


def _declare(_lib):
    _lib.or_problem_create.argtypes = [C.POINTER(_In), C.POINTER(C.c_void_p)]
    _lib.or_problem_destroy.argtypes = [C.c_void_p]
    _lib.or_problem_info.argtypes = [C.c_void_p] + [C.POINTER(C.c_double)] * 7
    _lib.or_trace.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int64, C.POINTER(_Query), C.c_uint64,
                              C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_uint32)]
    _lib.or_estimate.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int64, C.POINTER(_Query), C.c_int,
                                 C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(_Counters)]
    _lib.or_estimate_groups.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int64, C.POINTER(_Query),
                                        C.POINTER(C.c_uint32), C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(_Counters)]
    _lib.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
    _lib.or_sample_surface.argtypes = [C.c_void_p, C.c_int, C.c_uint64, C.c_uint64, C.POINTER(C.c_double)]
    _lib.or_training_points.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_int, C.POINTER(C.c_double), C.c_int64,
                                        C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_int64)]


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32); k = np.asarray(key, dtype=np.uint32); o = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(o, C.c_uint32))
    return o


class OracleProblem:
    """Oracle-side compiled problem (built from a workloads.Problem)."""

    def __init__(self, prob, library=None):
        self.lib = library if library is not None else lib()
        m, N = prob.dim, prob.n_regions
        self.dim, self.N = m, N
        keep = {}
        keep["parent"] = np.asarray(prob.parent, dtype=np.int32)
        keep["sigma"] = np.asarray(prob.sigma, dtype=np.float64)
        keep["kind"] = np.array([s.kind for s in prob.shapes], dtype=np.int32)
        keep["center"] = np.array([s.center for s in prob.shapes], dtype=np.float64).reshape(-1)
        keep["radius"] = np.array([s.radius for s in prob.shapes], dtype=np.float64)
        keep["A"] = np.array([s.A if s.A is not None else np.zeros((m, m)) for s in prob.shapes],
                             dtype=np.float64).reshape(-1)
        # polylines (kind 2) and meshes (kind 3) keep their vertices in separate arrays
        nv = [len(s.vertices) if s.vertices is not None else 0 for s in prob.shapes]
        keep["nv"] = np.asarray(nv, dtype=np.int32)
        pl = [n if s.kind == 2 else 0 for n, s in zip(nv, prob.shapes)]
        ms = [n if s.kind == 3 else 0 for n, s in zip(nv, prob.shapes)]
        keep["voff"] = np.concatenate([[0], np.cumsum(pl)[:-1]]).astype(np.int64)
        verts = [s.vertices for s in prob.shapes if s.vertices is not None and s.kind == 2]
        keep["verts"] = np.ascontiguousarray(np.concatenate(verts, 0) if verts else np.zeros((1, 2)), dtype=np.float64).reshape(-1)
        keep["mvoff"] = np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(np.int64)
        mverts = [s.vertices for s in prob.shapes if s.vertices is not None and s.kind == 3]
        keep["mverts"] = np.ascontiguousarray(np.concatenate(mverts, 0) if mverts else np.zeros((1, 3)), dtype=np.float64).reshape(-1)
        nt = [len(s.triangles) if getattr(s, "triangles", None) is not None else 0 for s in prob.shapes]
        keep["nt"] = np.asarray(nt, dtype=np.int32)
        keep["toff"] = np.concatenate([[0], np.cumsum(nt)[:-1]]).astype(np.int64)
        tris = [s.triangles for s in prob.shapes if getattr(s, "triangles", None) is not None]
        keep["tris"] = np.ascontiguousarray(np.concatenate(tris, 0) if tris else np.zeros((1, 3)), dtype=np.int32).reshape(-1)
        keep["dkind"] = np.array([d.kind for d in prob.data], dtype=np.int32)
        keep["dcenter"] = np.array([np.asarray(d.center, dtype=np.float64).reshape(m) for d in prob.data]).reshape(-1)
        keep["nterms"] = np.array([d.n_terms for d in prob.data], dtype=np.int32)
        ncoef = [len(d.coef) for d in prob.data]
        keep["coff"] = np.concatenate([[0], np.cumsum(ncoef)[:-1]]).astype(np.int64)
        keep["coef"] = np.concatenate([np.asarray(d.coef, dtype=np.float64) for d in prob.data] + [np.zeros(1)])
        ex = np.zeros((sum(ncoef) + 1) * m, dtype=np.uint8)
        for d, off in zip(prob.data, keep["coff"]):
            if d.exps is not None:
                e = np.asarray(d.exps, dtype=np.uint8).reshape(-1)
                ex[off * m: off * m + len(e)] = e
        keep["exps"] = ex
        self._keep = keep
        s = _In(m, N, _p(keep["parent"], C.c_int), _p(keep["sigma"], C.c_double), _p(keep["kind"], C.c_int),
                _p(keep["center"], C.c_double), _p(keep["radius"], C.c_double), _p(keep["A"], C.c_double),
                _p(keep["nv"], C.c_int), _p(keep["voff"], C.c_int64), _p(keep["verts"], C.c_double),
                _p(keep["dkind"], C.c_int), _p(keep["dcenter"], C.c_double), _p(keep["nterms"], C.c_int),
                _p(keep["coff"], C.c_int64), _p(keep["coef"], C.c_double), _p(keep["exps"], C.c_ubyte),
                _p(keep["nt"], C.c_int), _p(keep["mvoff"], C.c_int64), _p(keep["mverts"], C.c_double),
                _p(keep["toff"], C.c_int64), _p(keep["tris"], C.c_int))
        h = C.c_void_p()
        rc = self.lib.or_problem_create(C.byref(s), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle problem_create failed: {rc}")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.or_problem_destroy(self.h)
            self.h = None

    def info(self):
        N = self.N
        out = {k: np.zeros(N) for k in ("alpha", "beta_scale", "area", "area_plus", "area_minus", "flux")}
        l1 = C.c_double()
        self.lib.or_problem_info(self.h, *[_p(out[k], C.c_double) for k in
                                        ("alpha", "beta_scale", "area", "area_plus", "area_minus", "flux")],
                              C.byref(l1))
        out["alpha_l1"] = l1.value
        return out

    def sample_surface(self, region, seed, n):
        y = np.zeros((n, self.dim))
        self.lib.or_sample_surface(self.h, region, seed, n, _p(y, C.c_double))
        return y

    def training_points(self, grid_n, margin=0.0, bc_n=0):
        """Surrogate training data (Sec. 5): interior grid points, boundary points, normals and
        b_1 / sigma_1 targets."""
        n_in, n_bc = C.c_int64(), C.c_int64()
        rc = self.lib.or_training_points(self.h, grid_n, margin, 0, None, 0, C.byref(n_in), None, None, None,
                                         C.byref(n_bc))
        if rc != 0:
            raise ValueError(f"oracle training points failed: {rc}")
        nb = (bc_n if self.dim == 2 else 2 * bc_n * bc_n) if bc_n else 0
        x = np.zeros((max(n_in.value, 1), self.dim)); yb = np.zeros((max(nb, 1), self.dim))
        nrm = np.zeros((max(nb, 1), self.dim)); fl = np.zeros(max(nb, 1))
        rc = self.lib.or_training_points(self.h, grid_n, margin, bc_n, _p(x, C.c_double), n_in.value, C.byref(n_in),
                                         _p(yb, C.c_double) if nb else None, _p(nrm, C.c_double), _p(fl, C.c_double),
                                         C.byref(n_bc))
        if rc != 0:
            raise ValueError(f"oracle training points failed: {rc}")
        return x[:n_in.value], yb[:nb], nrm[:nb], fl[:nb]


PLAIN, VR, NAIVE = 0, 1, 2   # estimators: Alg. 2, Alg. 3, the naive Markov-tree estimator (Sec. 4.2)


def _query(walks, M, seed=0, estimator=0, schedule_mode=0, batch_share=1, walk_offset=0, instance=0):
    return _Query(int(seed), int(walks), int(walk_offset), int(M), int(estimator), int(schedule_mode),
                  int(batch_share), int(instance))


def estimate(op: OracleProblem, x, walks, M, seed=0, estimator=0, schedule_mode=0, batch_share=1,
             walk_offset=0, instance=0, threads=None, groups=None):
    """Per-point mean, SE, gradient and gradient SE (Alg. 1, FP64).  `groups` optionally gives
    each point's random-stream group explicitly (default: point index // batch_share)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, op.dim)
    P = len(x)
    mean = np.zeros(P); se = np.zeros(P); g = np.zeros((P, op.dim)); gse = np.zeros((P, op.dim))
    cnt = _Counters()
    q = _query(walks, M, seed, estimator, schedule_mode, batch_share, walk_offset, instance)
    gr = None if groups is None else np.ascontiguousarray(groups, dtype=np.uint32)
    rc = op.lib.or_estimate_groups(op.h, _p(x, C.c_double), P, C.byref(q), _p(gr, C.c_uint32),
                                   threads or os.cpu_count() or 1, _p(mean, C.c_double), _p(se, C.c_double),
                                   _p(g, C.c_double), _p(gse, C.c_double), C.byref(cnt))
    if rc != 0:
        raise ValueError(f"oracle estimate failed: {rc}")
    counters = {f: getattr(cnt, f) for f, _ in _Counters._fields_}
    return mean, se, g, gse, counters


def trace(op: OracleProblem, x, n_samples, M, seed=0, estimator=0, schedule_mode=0, batch_share=1,
          walk_offset=0, instance=0, threads=None):
    """Per-walk values: F[p, j, k] (walker k of sample j at point p, times N), G[p, j, k, :],
    decision words T[p, j, k, i].  For the naive estimator, F[p, j, 0] is tree j's value
    (Eq. naive_woi_estimator) and T stays zero."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, op.dim)
    P = len(x); K = 2 if estimator == VR else 1
    F = np.zeros((P, n_samples, K)); G = np.zeros((P, n_samples, K, op.dim))
    T = np.zeros((P, n_samples, K, M + 1), dtype=np.uint32)
    walks = 2 * n_samples if estimator == VR else n_samples
    q = _query(walks, M, seed, estimator, schedule_mode, batch_share, walk_offset, instance)
    rc = op.lib.or_trace(op.h, _p(x, C.c_double), P, C.byref(q), n_samples, threads or os.cpu_count() or 1,
                        _p(F, C.c_double), _p(G, C.c_double), _p(T, C.c_uint32))
    if rc != 0:
        raise ValueError(f"oracle trace failed: {rc}")
    return F, G, T
