"""GPU parity of the naive Markov-tree estimator (Sec. 4.2, Eq. naive_woi_estimator).

Per tree (FP64 on identical node-keyed Philox streams): the HIP kernel's tree values and
gradients agree with the oracle's depth-first tree to 1e-9 relative.  A tree holds up to a few
hundred sampled points and carries no decision words, so a rounding-level difference that
changes a discrete choice (a tangent line's hit count) shows up only as a differing tree; such
trees are counted against a small budget.  Per point: the estimate equals the mean of the trace
values; the tree size (walker-step counter) is sum_{i=0}^{M} N^{i+1}; the mean matches the exact
u_M of concentric circles.
"""
import numpy as np
import pytest

import closed_forms as CF
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_2508_16767_amd import woi  # noqa: E402


def _np(t):
    return t.detach().cpu().numpy()


def _tree_nodes(N, M):
    return sum(N ** (i + 1) for i in range(M + 1))


def tree_parity(prob, pts, n, M, seed=7, offset=0, budget=1e-3):
    """Per-tree values of both sides; returns (GPU problem, F_gpu) after the checks."""
    print(f"naive tree parity: {prob.name}, {len(pts)} points, {n} trees, M = {M}", flush=True)
    op = O.OracleProblem(prob)
    Fo, Go, _ = O.trace(op, pts, n, M, seed=seed, estimator=O.NAIVE, walk_offset=offset)
    gp = woi.Problem(prob)
    Fg, Gg, Tg = woi.trace(gp, pts, n, M, seed=seed, estimator=woi.NAIVE, walk_offset=offset)
    torch.cuda.synchronize()
    assert Tg is None
    Fg, Gg = _np(Fg), _np(Gg)
    assert Fg.shape == Fo.shape == (len(pts), n, 1)
    rms = np.sqrt(np.mean(Fo ** 2, axis=(1, 2), keepdims=True)) + 1e-300
    okF = np.abs(Fg - Fo) <= 1e-9 * np.maximum(np.abs(Fo), 1e-3 * rms)
    grms = np.sqrt(np.mean(Go ** 2, axis=(1, 2, 3), keepdims=True)) + 1e-300
    okG = np.all(np.abs(Gg - Go) <= 1e-9 * np.maximum(np.abs(Go), 1e-3 * grms), axis=-1)
    bad = ~(okF & okG)
    assert bad.sum() <= max(1, budget * bad.size), f"{bad.sum()} of {bad.size} trees differ"
    return gp, Fg


def test_naive_parity_concentric_disk():
    p, xs = W.concentric_disk_2d()
    tree_parity(p, xs[::5], 2000, 3, budget=0)
    tree_parity(p, xs[:4], 200, 0, budget=0)                  # roots only
    tree_parity(p, xs[:4], 100, 3, offset=300, budget=0)      # later trees


def test_naive_parity_star_tree_polylines():
    from test_oracle_pins import STAR_PTS, _star_tree
    p, _, _ = _star_tree()
    tree_parity(p, STAR_PTS, 1000, 2)


def test_naive_parity_spheres_3d_and_4d():
    p = W.zheng_ex3_3d()
    tree_parity(p, W.ball_points(np.random.default_rng(1), 6, 3, 0.95), 1000, 4)
    p4, x4 = W.point_charge_ellipsoids(4, n_points=6)
    tree_parity(p4, x4, 600, 2)


def test_naive_parity_meshes():
    from test_gpu_parity import MESH_PTS, _mesh_tree
    tree_parity(_mesh_tree(), MESH_PTS, 500, 2)


def test_naive_single_region_and_ragged_leaves():
    """N = 1: one leaf per tree (63 idle lanes); N = 5 (N^(M+1) = 125 leaves: two passes of
    the wave, the second ragged)."""
    from test_oracle_pins import NC_PTS, _nonconvex_root
    p, _, _ = _nonconvex_root()
    tree_parity(p, NC_PTS, 1000, 3)
    p5 = W.concentric(2, [1.0, 0.8, 0.6, 0.4, 0.2], [1.0, 3.0, 0.5, 2.0, 4.0],
                      [W.fourier([0, 0], 0, [1.0], [0.0])] * 5)
    tree_parity(p5, np.array([[0.1, 0.0], [0.0, 0.5], [-0.3, -0.55], [0.9, 0.1]]), 400, 2)


def test_naive_estimate_counters_and_exact_expectation():
    p, xs = W.concentric_disk_2d()
    gp = woi.Problem(p)
    pts = xs[::4]
    T, M = 3000, 3
    c = woi.new_counters()
    mean, se, g, gse = [_np(t) for t in woi.estimate(gp, pts, T, M, seed=5, estimator=woi.NAIVE, counters=c)]
    F, G, _ = woi.trace(gp, pts, T, M, seed=5, estimator=woi.NAIVE)
    F, G = _np(F)[..., 0], _np(G)[:, :, 0]
    assert np.allclose(mean, F.mean(1), rtol=1e-12, atol=1e-14 * np.abs(F).max())
    assert np.allclose(se, F.std(1, ddof=1) / np.sqrt(T), rtol=1e-9)
    assert np.allclose(g, G.mean(1), rtol=1e-12, atol=1e-14 * np.abs(G).max())
    c = _np(c)
    assert c[0] == len(pts) * T * _tree_nodes(2, M) and c[3] == 0
    mo, so, go, _, cnt = O.estimate(O.OracleProblem(p), pts, T, M, seed=5, estimator=O.NAIVE)
    assert cnt["walk_steps"] == c[0]
    assert np.allclose(mean, mo, rtol=1e-9, atol=1e-9 * so.max())
    # exact u_M (Theorem 2: the naive and scheduled estimators share their expectation)
    H, gH = CF.harmonic_2d(1, "cos")
    mean, se, g, gse = [_np(t) for t in woi.estimate(gp, xs, 100000, M, seed=9, estimator=woi.NAIVE)]
    ref = [CF.concentric_uM([1, .5], [10, 1], [1, 1], 1, 2, M, x, H, gH) for x in xs]
    z = (mean - np.array([r[0] for r in ref])) / se
    zg = (g - np.array([r[1] for r in ref])) / gse
    assert np.max(np.abs(z)) < 4.5 and np.max(np.abs(zg)) < 4.5
    assert 0.5 < np.mean(z ** 2) < 1.6


def test_naive_full_size_sampled():
    """The benchmark's naive configuration in full (star tree, 4096 points, N = 9, M = 2, 100
    trees per point, the launch it times); sampled points against the oracle on identical
    streams (explicit point groups).  A tree whose discrete choices flip at rounding level moves
    one point's mean by a fraction of its SE, so one such point is allowed."""
    p, xs = W.star_tree_2d()
    gp = woi.Problem(p)
    mean, se, g, gse = [_np(t) for t in woi.estimate(gp, xs, 100, 2, seed=31, estimator=woi.NAIVE)]
    assert np.all(np.isfinite(mean)) and np.all(np.isfinite(g)) and np.all(se > 0)
    idx = np.random.default_rng(3).choice(len(xs), 8, replace=False)
    mo, so, go, gso, cnt = O.estimate(O.OracleProblem(p), xs[idx], 100, 2, seed=31, estimator=O.NAIVE, groups=idx)
    assert cnt["walk_steps"] == len(idx) * 100 * _tree_nodes(9, 2)
    close = np.abs(mean[idx] - mo) <= 1e-9 * np.maximum(np.abs(mo), so)
    gclose = np.all(np.abs(g[idx] - go) <= 1e-9 * np.maximum(np.abs(go), gso), axis=1)
    assert (~(close & gclose)).sum() <= 1
    assert np.max(np.abs(mean[idx] - mo) / so) < 0.5


def test_naive_fp32_paired_with_fp64():
    """FP32 walks on the FP64 trees' streams: per-tree values differ only by rounding (a rare
    FP32 flip of a discrete choice aside), the means by a small fraction of the SE; the FP32
    mean matches the exact u_M."""
    p, xs = W.concentric_disk_2d()
    gp = woi.Problem(p)
    pts = xs[::4]
    F64, _, _ = woi.trace(gp, pts, 2000, 3, seed=6, estimator=woi.NAIVE)
    F32, _, _ = woi.trace(gp, pts, 2000, 3, seed=6, estimator=woi.NAIVE, precision=woi.FP32)
    F64, F32 = _np(F64)[..., 0], _np(F32)[..., 0]
    rms = np.sqrt(np.mean(F64 ** 2))
    close = np.abs(F32 - F64) <= 1e-3 * np.maximum(np.abs(F64), rms)
    assert close.mean() > 0.99
    se = F64.std(1, ddof=1) / np.sqrt(F64.shape[1])
    assert np.all(np.abs(F32.mean(1) - F64.mean(1)) < 0.05 * se)
    from test_oracle_pins import _star_tree, STAR_PTS
    ps, _, _ = _star_tree()
    gs = woi.Problem(ps)
    m64, s64, _, _ = [_np(a) for a in woi.estimate(gs, STAR_PTS, 4000, 2, seed=8, estimator=woi.NAIVE)]
    m32, _, _, _ = [_np(a) for a in woi.estimate(gs, STAR_PTS, 4000, 2, seed=8, estimator=woi.NAIVE, precision=woi.FP32)]
    assert np.all(np.abs(m32 - m64) < 0.1 * s64), (m32 - m64) / s64
    H, gH = CF.harmonic_2d(1, "cos")
    mean, se32, _, _ = [_np(t) for t in woi.estimate(gp, xs, 50000, 3, seed=9, estimator=woi.NAIVE, precision=woi.FP32)]
    ref = np.array([CF.concentric_uM([1, .5], [10, 1], [1, 1], 1, 2, 3, x, H, gH)[0] for x in xs])
    assert np.max(np.abs((mean - ref) / se32)) < 4.5


def _naive_cases():
    from test_oracle_pins import _star_tree, STAR_PTS
    ps, _, _ = _star_tree()
    pm, xm = W.mesh_tree_3d(n_points=6, subdiv=2)
    return [("sphere_3d", W.zheng_ex3_3d(), W.ball_points(np.random.default_rng(3), 6, 3, 0.9), 3, 600),
            ("mesh_3d", pm, xm, 2, 400),
            ("star_tree_M3", ps, STAR_PTS, 3, 200)]


@pytest.mark.parametrize("case", range(3))
def test_naive_fp32_paired_with_fp64_3d_mesh_star(case):
    """FP32 naive walks (FP32 node terms taken to FP64 before they are summed) against FP64 trees on
    identical node-keyed streams: a 3D sphere pair, triangle meshes, and the star tree at M = 3
    (about 340 signed terms per tree)."""
    name, p, pts, M, trees = _naive_cases()[case]
    gp = woi.Problem(p)
    F64, _, _ = woi.trace(gp, pts, trees, M, seed=12, estimator=woi.NAIVE)
    F32, _, _ = woi.trace(gp, pts, trees, M, seed=12, estimator=woi.NAIVE, precision=woi.FP32)
    F64, F32 = _np(F64)[..., 0], _np(F32)[..., 0]
    rms = np.sqrt(np.mean(F64 ** 2))
    close = np.abs(F32 - F64) <= 1e-3 * np.maximum(np.abs(F64), rms)
    assert close.mean() > 0.98, name
    se = F64.std(1, ddof=1) / np.sqrt(F64.shape[1])
    assert np.all(np.abs(F32.mean(1) - F64.mean(1)) < 0.25 * se), (name, (F32.mean(1) - F64.mean(1)) / se)


def test_naive_rejections():
    p, xs = W.concentric_disk_2d()
    gp = woi.Problem(p)
    for kw in ({"batch_share": 2}, {"instance": 3}):
        with pytest.raises(woi.WoiError, match="UNSUPPORTED"):
            woi.estimate(gp, xs, 100, 2, estimator=woi.NAIVE, **kw)
    with pytest.raises(woi.WoiError, match="INVALID_ARG"):    # (N + 1)^(M + 1) = 3^20 > 2^31
        woi.estimate(gp, xs, 100, 19, estimator=woi.NAIVE)
