"""C ABI checks that need no GPU: the library loads, exports every symbol that
include/woi.h declares, and its host-side problem compiler validates inputs and
agrees with the oracle's independent computation of the problem constants."""
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def woi():
    from paper_2508_16767_amd import woi as mod
    return mod


def declared_functions():
    src = open(os.path.join(ROOT, "include", "woi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(woi_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = declared_functions()
    for n in ("woi_problem_create", "woi_problem_upload", "woi_problem_destroy", "woi_estimate", "woi_trace",
              "woi_estimate_batch", "woi_workspace_size"):
        assert n in names


def test_library_exports_every_declared_symbol(woi):
    out = subprocess.run(["nm", "-D", "--defined-only", woi.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (woi_[a-z_0-9]+)\b", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        getattr(woi._lib, n)
    assert set(woi.EXPORTS) <= set(declared_functions())


def _err(woi, prob, status, **kw):
    with pytest.raises(woi.WoiError) as e:
        woi.Problem(prob, **kw)
    assert e.value.status == status, str(e.value)


def test_validation_errors(woi):
    p, _ = W.concentric_disk_2d()
    bad = W.Problem(2, [-1, 1], p.sigma, p.shapes, p.data)
    _err(woi, bad, "WOI_E_GEOMETRY")                           # parent must precede child
    outside = W.Problem(2, [-1, 0], [1.0, 2.0], [W.sphere([0, 0], 1.0), W.sphere([0.9, 0], 0.3)], p.data)
    _err(woi, outside, "WOI_E_GEOMETRY")                       # child pokes out of its parent
    sib = W.Problem(2, [-1, 0, 0], [1.0, 2.0, 3.0],
                    [W.sphere([0, 0], 1.0), W.sphere([0.2, 0], 0.3), W.sphere([-0.2, 0], 0.3)], p.data + [W.zero_data(2)])
    _err(woi, sib, "WOI_E_GEOMETRY")                           # overlapping siblings
    inc = W.Problem(2, [-1], [1.0], [W.sphere([0, 0], 1.0)], [W.fourier([0, 0], 0.3, [1.0], [0.0])])
    _err(woi, inc, "WOI_E_INCOMPATIBLE")                       # nonzero net flux
    inc.compat_mode = 2
    woi.Problem(inc)                                           # accepted without the check
    cw = W.star_polyline([0, 0], 0.5, 0.1, 3, 64)
    cw.vertices = cw.vertices[::-1].copy()
    _err(woi, W.Problem(2, [-1, 0], [1.0, 2.0], [W.sphere([0, 0], 1.0), cw], p.data), "WOI_E_GEOMETRY")
    neg = W.Problem(2, [-1, 0], [1.0, -3.0], p.shapes, p.data)
    _err(woi, neg, "WOI_E_INVALID_ARG")


def test_mesh_validation(woi):
    """Triangle meshes: closed, outward, nested, 3D only; no variance reduction."""
    sh = W.icosphere([0, 0, 0], 1.0, 2)
    ff = W.field_flux([1.0, 0.0, 0.0])
    prob = woi.Problem(W.Problem(3, [-1], [1.0], [sh], [ff]))  # accepted (compatible linear data)
    flipped = W.mesh(sh.vertices, sh.triangles[:, ::-1])
    _err(woi, W.Problem(3, [-1], [1.0], [flipped], [ff]), "WOI_E_GEOMETRY")          # inward normals
    _err(woi, W.Problem(3, [-1], [1.0], [W.mesh(sh.vertices, sh.triangles[:-1])], [ff]), "WOI_E_GEOMETRY")  # open
    _err(woi, W.Problem(3, [-1, 0], [1.0, 2.0], [sh, W.icosphere([0.7, 0, 0], 0.5, 1)], [ff, ff]),
         "WOI_E_GEOMETRY")                                                            # leaves its parent
    bad = W.mesh(sh.vertices, np.where(sh.triangles == 0, len(sh.vertices), sh.triangles))
    _err(woi, W.Problem(3, [-1], [1.0], [bad], [ff]), "WOI_E_INVALID_ARG")          # index out of range
    with pytest.raises(woi.WoiError) as e:
        woi.workspace_size(prob, 16, woi.make_query(100, 4, estimator=woi.VR))
    assert e.value.status == "WOI_E_UNSUPPORTED"


def test_query_validation_without_gpu(woi):
    p5, _ = W.nested_spheres_6d()
    prob = woi.Problem(p5)
    with pytest.raises(woi.WoiError) as e:
        woi.workspace_size(prob, 16, woi.make_query(100, 4, estimator=woi.VR))
    assert e.value.status == "WOI_E_UNSUPPORTED"
    p1, _ = W.concentric_disk_2d()
    prob = woi.Problem(p1)
    for q in (woi.make_query(101, 4, estimator=woi.VR), woi.make_query(100, 99), woi.make_query(0, 4),
              woi.make_query(100, 4, batch_share=0), woi.make_query(100, 4, instance=1 << 24)):
        with pytest.raises(woi.WoiError):
            woi.workspace_size(prob, 16, q)
    assert woi.workspace_size(prob, 64, woi.make_query(10000, 4)) > 0
    # naive Markov trees: batch_share 1, instance 0 and (N + 1)^(M + 1) <= 2^31
    for q, st in ((woi.make_query(100, 4, estimator=woi.NAIVE, batch_share=2), "WOI_E_UNSUPPORTED"),
                  (woi.make_query(100, 4, estimator=woi.NAIVE, instance=1), "WOI_E_UNSUPPORTED"),
                  (woi.make_query(100, 19, estimator=woi.NAIVE), "WOI_E_INVALID_ARG"),
                  (woi.make_query(100, 24, estimator=woi.NAIVE), "WOI_E_INVALID_ARG")):
        with pytest.raises(woi.WoiError) as e:
            woi.workspace_size(prob, 16, q)
        assert e.value.status == st
    assert woi.workspace_size(prob, 64, woi.make_query(1000, 18, estimator=woi.NAIVE)) > 0   # 3^19 ids fit
    # work bound: N^(M + 1) <= 2^24 leaves per tree (N = 9: M = 6 fits, M = 8 has ids but 9^9 leaves)
    star = woi.Problem(W.star_tree_2d(n_points=8)[0])
    assert woi.workspace_size(star, 64, woi.make_query(10, 6, estimator=woi.NAIVE)) > 0
    with pytest.raises(woi.WoiError) as e:
        woi.workspace_size(star, 64, woi.make_query(10, 8, estimator=woi.NAIVE))
    assert e.value.status == "WOI_E_INVALID_ARG" and "leaves" in str(e.value)
    # 2D ellipses are refused at compile time (the oracle's plain 2D ellipse is a pin only)
    with pytest.raises(woi.WoiError) as e:
        woi.Problem(W.single_ellipsoid_linear(2, [0.9, 0.5])[0])
    assert e.value.status == "WOI_E_UNSUPPORTED" and "ellipse" in str(e.value)
    assert woi.workspace_size(prob, 64, woi.make_query(1000, 4, estimator=woi.NAIVE, precision=woi.FP32)) > 0


@pytest.mark.parametrize("make", [lambda: W.concentric_disk_2d()[0], lambda: W.star_tree_2d(n_points=8)[0], lambda: W.nested_spheres_6d()[0],
                                  lambda: W.zheng_ex3_3d(),
                                  lambda: W.single_ellipsoid_linear(3, [0.9, 0.6, 0.4])[0]])
def test_host_compile_matches_oracle(woi, oracle_mod, make):
    p = make()
    a = woi.Problem(p).info()
    b = oracle_mod.OracleProblem(p).info()
    for k in ("alpha", "beta_scale"):
        assert np.array_equal(a[k], b[k])
    assert a["alpha_l1"] == pytest.approx(b["alpha_l1"], rel=1e-15)
    assert np.allclose(a["area"], b["area"], rtol=1e-12)
    scale = np.abs(a["area"]).max()
    assert np.allclose(a["flux"], b["flux"], atol=1e-10 * scale)
    if p.dim <= 3:
        assert np.allclose(a["area_plus"], b["area_plus"], rtol=1e-6, atol=1e-12 * scale)
        assert np.allclose(a["area_minus"], b["area_minus"], rtol=1e-6, atol=1e-12 * scale)
    else:
        assert np.all(np.isnan(a["area_plus"]))


def test_stats_without_counters_or_events(woi):
    """woi_stats_read with neither counters nor events touches no device: zeros, seconds = -1."""
    st = woi.stats()
    assert all(st[k] == 0 for k in st if k != "seconds") and st["seconds"] == -1.0
    assert len(woi.COUNTER_NAMES) == woi.N_COUNTERS == 9


def test_batch_validation_without_gpu(woi):
    """woi_estimate_batch rejects malformed batches before touching a device."""
    import ctypes as C
    p1, _ = W.concentric_disk_2d()
    prob = woi.Problem(p1)
    p5 = woi.Problem(W.nested_spheres_6d()[0])

    def items(*queries, problems=None):
        arr = (woi._BatchItem * len(queries))()
        for i, q in enumerate(queries):
            it = arr[i]
            it.problem = (problems[i] if problems else prob).handle
            it.points, it.P, it.query = 16, 8, q              # never dereferenced on these paths
            it.mean, it.se = 16, 16
        return arr

    def status(arr, n=None):
        rc = woi._lib.woi_estimate_batch(arr, len(arr) if n is None else n, C.c_void_p(16), 1 << 20, None, None)
        return woi._lib.woi_status_string(rc).decode()

    q = woi.make_query(100, 4)
    assert status(items(q), n=0) == "WOI_E_INVALID_ARG"                                  # empty batch
    assert status(items(q, woi.make_query(100, 4, precision=woi.FP32))) == "WOI_E_INVALID_ARG"   # mixed precision
    assert status(items(q, woi.make_query(100, 4, estimator=woi.VR))) == "WOI_E_INVALID_ARG"     # mixed estimator
    assert status(items(woi.make_query(100, 4, batch_share=0))) == "WOI_E_INVALID_ARG"   # batch_share < 1
    assert status(items(woi.make_query(100, 4, block_size=128))) == "WOI_E_INVALID_ARG"  # launch shape
    assert status(items(q, woi.make_query(100, 4, block_size=256))) == "WOI_E_INVALID_ARG"
    assert status(items(woi.make_query(100, 99))) == "WOI_E_INVALID_ARG"                 # M above the maximum
    assert status(items(woi.make_query(1 << 33, 4))) == "WOI_E_INVALID_ARG"              # samples per point
    bad = items(q)
    bad[0].mean = None
    assert status(bad) == "WOI_E_INVALID_ARG"
    assert status(items(woi.make_query(100, 4, estimator=woi.VR), problems=[p5])) == "WOI_E_UNSUPPORTED"
    pm = woi.Problem(W.mesh_tree_3d(n_points=8, subdiv=1)[0])
    assert status(items(woi.make_query(100, 4), problems=[pm])) == "WOI_E_UNSUPPORTED"    # triangle meshes
    assert status(items(woi.make_query(100, 4, estimator=woi.NAIVE))) == "WOI_E_UNSUPPORTED"   # Markov trees


def test_schedule_lookup_in_integers():
    """The walkers decide the schedule on the 32-bit word w itself: with u(w) = (w + 1/2) 2^-32,
    floor(64 u) = w >> 26, floor(u N) = ((2w + 1) N) >> 33, and u < c exactly when
    w < ceil(c 2^32 - 1/2) (at least 0).  Checked here against the FP64 forms the oracle uses."""
    import math
    rng = np.random.default_rng(3)
    w = np.concatenate([rng.integers(0, 2 ** 32, 200000, dtype=np.uint64),
                        np.array([0, 1, 2 ** 26 - 1, 2 ** 26, 2 ** 31, 2 ** 32 - 1], dtype=np.uint64)])
    u = (w.astype(np.float64) + 0.5) * 2.0 ** -32
    assert np.array_equal(np.minimum((u * 64.0).astype(np.int64), 63), (w >> np.uint64(26)).astype(np.int64))
    for n in range(1, 33):
        h0 = (((w << np.uint64(1)) | np.uint64(1)) * np.uint64(n)) >> np.uint64(33)
        assert np.array_equal(np.floor(u * n).astype(np.int64), h0.astype(np.int64))
    for c in np.concatenate([rng.random(2000), [0.0, 1.0, 2.0 ** -33, 0.5, 1 - 2.0 ** -53]]):
        thr = max(math.ceil(math.ldexp(float(c), 32) - 0.5), 0)
        probe = [t for t in (thr - 2, thr - 1, thr, thr + 1) if 0 <= t < 2 ** 32]
        probe += [int(t) for t in rng.integers(0, 2 ** 32, 8)]
        for t in probe:
            assert ((t + 0.5) * 2.0 ** -32 < c) == (t < thr)
