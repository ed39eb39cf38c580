"""Pins of the FP64 CPU oracle against values the paper and the mathematics fix.

No GPU.  Every statistical check uses fixed seeds, so results are deterministic;
thresholds are on z = (MC mean - exact) / SE with the exact value from
tests/closed_forms.py (mode-matrix series, Example 3 closed forms, depolarisation
factors, Nystrom) -- none of which shares code with the oracle.
"""
import os

import numpy as np
import pytest

import closed_forms as CF
import workloads as W

ZMAX = 4.5


def _z(mean, ref, se):
    return (np.asarray(mean) - np.asarray(ref)) / np.asarray(se)


# ----------------------------------------------------------------------------- RNG
def test_philox_known_answers(oracle_mod):
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    n = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        out = oracle_mod.philox(v[:4], v[4:6])
        assert list(out) == v[6:], line
        n += 1
    assert n == 3


def test_philox_uniform_words_chi2(oracle_mod):
    # 2^14 blocks of consecutive counters: each output word's top 6 bits uniform over 64 bins
    words = []
    for c in range(4096):
        words.extend(oracle_mod.philox([c, 7, 1, 0], [123, 456]))
    w = np.array(words, dtype=np.uint64)
    counts = np.bincount((w >> 26).astype(np.int64), minlength=64)
    e = len(w) / 64
    chi2 = ((counts - e) ** 2 / e).sum()
    assert chi2 < 120  # 63 dof, p ~ 2e-5 at 120


# ----------------------------------------------------------------------------- closed forms
def test_mode_series_limit_reproduces_example3():
    """The M -> infinity mode-matrix series equals the paper's printed Example 3 solutions."""
    path = os.path.join(os.path.dirname(__file__), "golden", "example3_closed_forms.txt")
    H3, g3 = CF.harmonic_2d(3, "sin")
    Hx, gx = CF.harmonic_x1(3)
    n = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        v = [float(t) for t in line.split()]
        dim, x = int(v[0]), np.array(v[1:])
        if dim == 2:
            u, _ = CF.concentric_uM([1.0, 0.4], [1.0, 1 / 3], [20.0, 0.0], 3, 2, None, x, H3, g3)
            ref = CF.bower_2d_exact(x)
        else:
            u, _ = CF.concentric_uM([1.0, 0.4], [1.0, 0.5], [5.0, 0.0], 1, 3, None, x, Hx, gx)
            ref = CF.zheng_3d_exact(x)
        assert abs(u - ref) < 1e-12 * max(1.0, abs(ref))
        n += 1
    assert n == 6


def test_closed_form_gradient_matches_finite_difference():
    H, gH = CF.harmonic_2d(1, "cos")
    for x in (np.array([0.3, -0.2]), np.array([0.8, 0.1])):
        _, g = CF.concentric_uM([1, .5], [10, 1], [1, 1], 1, 2, 4, x, H, gH)
        h = 1e-6
        fd = [(CF.concentric_uM([1, .5], [10, 1], [1, 1], 1, 2, 4, x + h * e, H, gH)[0] -
               CF.concentric_uM([1, .5], [10, 1], [1, 1], 1, 2, 4, x - h * e, H, gH)[0]) / (2 * h)
              for e in np.eye(2)]
        assert np.allclose(g, fd, atol=1e-8)


# ----------------------------------------------------------------------------- problem constants
def test_alpha_beta_and_areas(oracle_mod):
    p, _ = W.concentric_disk_2d()
    info = oracle_mod.OracleProblem(p).info()
    # Eq. unit_coeff_charge_density_sys: alpha_1 = 2, alpha_2 = 2(1-10)/11; s_1 = 2/10, s_2 = -2/11
    assert np.allclose(info["alpha"], [2.0, -18 / 11])
    assert np.allclose(info["beta_scale"], [0.2, -2 / 11])
    assert np.allclose(info["area"], [2 * np.pi, np.pi])
    assert info["alpha_l1"] == pytest.approx(2 + 18 / 11)


def test_ellipsoid_area_matches_legendre(oracle_mod):
    p, _, _ = W.single_ellipsoid_linear(3, [0.9, 0.6, 0.4])
    area = oracle_mod.OracleProblem(p).info()["area"][0]
    assert area == pytest.approx(CF.ellipsoid3_area(0.9, 0.6, 0.4), rel=1e-12)
    # m-D sphere written as an ellipsoid: |S^{m-1}| R^{m-1}
    for m in (4, 6):
        p = W.Problem(m, [-1], [1.0], [W.ellipsoid(np.zeros(m), np.eye(m) / 0.7 ** 2)],
                      [W.zero_data(m)], 2)
        area = oracle_mod.OracleProblem(p).info()["area"][0]
        assert area == pytest.approx(CF.unit_sphere_area(m) * 0.7 ** (m - 1), rel=1e-10)


def test_vr_half_measures(oracle_mod):
    # x1/|x| on a sphere and cos(th) on a circle split the surface into exact halves;
    # zero data puts everything in {beta >= 0}
    p = W.zheng_ex3_3d()
    info = oracle_mod.OracleProblem(p).info()
    assert info["area_plus"][0] == pytest.approx(info["area"][0] / 2, rel=1e-9)
    assert info["area_minus"][0] == pytest.approx(info["area"][0] / 2, rel=1e-9)
    assert info["area_plus"][1] == pytest.approx(info["area"][1], rel=1e-12) and info["area_minus"][1] == 0.0
    p, _ = W.concentric_disk_2d()
    info = oracle_mod.OracleProblem(p).info()
    assert np.allclose(info["area_plus"], info["area"] / 2, rtol=1e-12)


def test_vr_half_measures_ellipsoid_odd_data(oracle_mod):
    """Variance reduction on an ellipsoid (Sec. 4.4): flux data n . g of a uniform field are odd
    under y -> 2c - y, which maps the ellipsoid onto itself with the same surface element, so
    {beta >= 0} and {beta < 0} are exact halves; their sum is Legendre's area.  The halves come
    from the oracle's ring quadrature (ellipsoid Jacobian, sign breakpoints), not from its area
    rule."""
    for axes, direction in (([0.9, 0.6, 0.4], 0), ([0.5, 0.8, 0.3], 2)):
        p, _, _ = W.single_ellipsoid_linear(3, axes, direction=direction)
        info = oracle_mod.OracleProblem(p).info()
        area = CF.ellipsoid3_area(*axes)
        assert info["area_plus"][0] == pytest.approx(area / 2, rel=1e-8)
        assert info["area_minus"][0] == pytest.approx(area / 2, rel=1e-8)


def test_vr_half_measures_ellipsoid_uneven_split(oracle_mod):
    """An uneven split: b = 0.35 + e . v in the direction e = (y - c)/|y - c| about a centre off
    the ellipsoid's own.  The fraction of the surface with b >= 0, counted on the oracle's uniform
    surface samples (pinned separately by the slab-area test), times Legendre's area, must match
    the quadrature's |dOmega^+| within Monte Carlo error, and |dOmega^+| + |dOmega^-| = area."""
    axes = [0.9, 0.6, 0.4]
    p0, A, Q = W.single_ellipsoid_linear(3, axes, direction=0)
    v = np.array([0.3, -0.8, 0.5])
    c = np.array([0.1, 0.05, -0.02])
    terms = {(0, 0, 0): 0.35, (1, 0, 0): v[0], (0, 1, 0): v[1], (0, 0, 1): v[2]}
    p = W.Problem(3, [-1], [1.0], p0.shapes, [W.dirpoly(c, terms)], 2, "ellipsoid-uneven")
    op = oracle_mod.OracleProblem(p)
    info = op.info()
    area = CF.ellipsoid3_area(*axes)
    assert info["area_plus"][0] + info["area_minus"][0] == pytest.approx(area, rel=1e-8)
    y = op.sample_surface(0, 17, 400000)
    e = (y - c) / np.linalg.norm(y - c, axis=1, keepdims=True)
    frac = np.mean(0.35 + e @ v >= 0)
    assert 0.55 < frac < 0.9                                  # genuinely uneven
    sd = np.sqrt(frac * (1 - frac) / len(y))
    assert abs(info["area_plus"][0] / area - frac) < 5 * sd


def test_ellipsoid_depolarization_gradient_vr(oracle_mod):
    """The variance-reduced estimator (Alg. 3) on a 3D ellipsoid has the same exact gradient as
    the plain one: first points on {beta >= 0} / {beta < 0} by sign rejection, weighted by the
    half-measures.  (In 2D the halves are arclength intervals of circles and polylines: VR on an
    ellipse is refused.)"""
    dim, axes = 3, [0.9, 0.6, 0.4]
    p2, _, _ = W.single_ellipsoid_linear(2, [0.9, 0.5], direction=0)
    with pytest.raises(ValueError):
        oracle_mod.estimate(oracle_mod.OracleProblem(p2), np.zeros((1, 2)), 100, 1, estimator=1)
    p, A, Q = W.single_ellipsoid_linear(dim, axes, direction=0)
    op = oracle_mod.OracleProblem(p)
    pts = np.random.default_rng(0).standard_normal((3, dim)) * 0.1
    for M in (1, 3):
        _, _, g, gse, _ = oracle_mod.estimate(op, pts, 100000, M, seed=19, estimator=1)
        gref = CF.ellipsoid_grad_uM(axes, Q, 0, M)
        assert np.max(np.abs(_z(g, gref[None, :], gse))) < ZMAX


def test_uniform_surface_samples(oracle_mod):
    """Uniform sampling on an ellipsoid: area fraction of a slab {|n1| < 0.5} matches quadrature,
    and on a polyline the arclength histogram is flat."""
    p, A, Q = W.single_ellipsoid_linear(3, [0.9, 0.6, 0.4])
    op = oracle_mod.OracleProblem(p)
    y = op.sample_surface(0, 11, 200000)
    assert np.allclose(np.einsum("ij,jk,ik->i", y, A, y), 1.0, atol=1e-12)
    # fraction of the surface with x1 > 0 is 1/2 by symmetry; with the projection on the longest
    # principal axis in (-0.3, 0.3) compare with a fine quadrature in principal coordinates
    z = y @ Q
    frac = np.mean(np.abs(z[:, 0]) < 0.3)
    a = np.array([0.9, 0.6, 0.4])
    th = np.linspace(0, np.pi, 1201)[:-1] + np.pi / 2400; ph = np.linspace(0, 2 * np.pi, 2401)[:-1] + np.pi / 2400
    T, P = np.meshgrid(th, ph, indexing="ij")
    u = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1)
    J = np.sqrt(((u / a) ** 2).sum(-1)) * np.prod(a) * np.sin(T)
    x1 = a[0] * u[..., 0]
    ref = (J * (np.abs(x1) < 0.3)).sum() / J.sum()
    assert abs(frac - ref) < 5 * np.sqrt(ref * (1 - ref) / len(z))
    p2 = W.Problem(2, [-1], [1.0], [W.star_polyline([0, 0], 0.6, 0.2, 5, 256)], [W.zero_data(2)], 2)
    op2 = oracle_mod.OracleProblem(p2)
    y2 = op2.sample_surface(0, 3, 100000)
    # arclength coordinate of each sample (vertex j sits at angle 2 pi j / n about the centre)
    v = p2.shapes[0].vertices; n = len(v)
    seg = np.linalg.norm(np.roll(v, -1, 0) - v, axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    j = np.floor(np.mod(np.arctan2(y2[:, 1], y2[:, 0]), 2 * np.pi) / (2 * np.pi / n)).astype(int) % n
    s = cum[j] + np.linalg.norm(y2 - v[j], axis=1)
    cnt, _ = np.histogram(s / cum[-1], np.linspace(0, 1, 21))
    exp = len(s) / 20.0
    assert (((cnt - exp) ** 2) / exp).sum() < 60  # 19 dof


# ----------------------------------------------------------------------------- estimator pins
CFG1 = ([1.0, 0.5], [10.0, 1.0], [1.0, 1.0])


@pytest.mark.parametrize("M", [0, 1, 2, 4])
@pytest.mark.parametrize("estimator", [0, 1])
def test_concentric_disk_exact_expectation(oracle_mod, M, estimator):
    p, xs = W.concentric_disk_2d()
    op = oracle_mod.OracleProblem(p)
    pts = xs[::5]
    mean, se, g, gse, cnt = oracle_mod.estimate(op, pts, 200000, M, seed=10 + M, estimator=estimator)
    H, gH = CF.harmonic_2d(1, "cos")
    ref = [CF.concentric_uM(*CFG1, 1, 2, M, x, H, gH) for x in pts]
    z = _z(mean, [r[0] for r in ref], se)
    zg = _z(g, np.array([r[1] for r in ref]), gse)
    assert np.max(np.abs(z)) < ZMAX and np.max(np.abs(zg)) < ZMAX
    assert 0.3 < np.mean(np.concatenate([z, zg.ravel()]) ** 2) < 2.0
    assert cnt["cap_hits"] == 0


@pytest.mark.parametrize("estimator", [0, 1])
def test_sphere_3d_exact_expectation(oracle_mod, estimator):
    p = W.zheng_ex3_3d()
    op = oracle_mod.OracleProblem(p)
    pts = np.array([[0.2, 0.1, -0.1], [0.5, -0.3, 0.2], [-0.1, 0.7, 0.1], [0.05, -0.2, 0.33], [0, 0, 0.9]])
    Hx, gx = CF.harmonic_x1(3)
    for M in (1, 3):
        mean, se, g, gse, _ = oracle_mod.estimate(op, pts, 100000, M, seed=3, estimator=estimator)
        ref = [CF.concentric_uM([1, .4], [1, .5], [5, 0], 1, 3, M, x, Hx, gx) for x in pts]
        assert np.max(np.abs(_z(mean, [r[0] for r in ref], se))) < ZMAX
        assert np.max(np.abs(_z(g, np.array([r[1] for r in ref]), gse))) < ZMAX


def test_six_ball_global_balance_exact_expectation(oracle_mod):
    p, xs = W.nested_spheres_6d()
    op = oracle_mod.OracleProblem(p)
    info = op.info()
    # global balance: flux through the boundary equals the sum of interface jumps (R12 reading)
    assert abs(info["flux"][0] - info["flux"][1:].sum()) < 1e-9 * abs(info["flux"][0])
    c1 = 0.7 ** 5 - 0.5 * 0.35 ** 5
    H0, g0 = CF.harmonic_const(6); H1, g1 = CF.harmonic_x1(6)
    # points away from the interfaces (the 6D gradient estimator is heavy-tailed near them)
    dirs = np.random.default_rng(1).standard_normal((6, 6))
    pts = dirs / np.linalg.norm(dirs, axis=1, keepdims=True) * np.array([0.1, 0.2, 0.5, 0.55, 0.82, 0.88])[:, None]
    for M in (0, 2, 4):
        mean, se, g, gse, _ = oracle_mod.estimate(op, pts, 100000, M, seed=5)
        ref = []
        for x in pts:
            a = CF.concentric_uM([1, .7, .35], [1, 5, .2], [c1, 1, -.5], 0, 6, M, x, H0, g0)
            b = CF.concentric_uM([1, .7, .35], [1, 5, .2], [1, .5, -.3], 1, 6, M, x, H1, g1)
            ref.append((a[0] + b[0], a[1] + b[1]))
        assert np.max(np.abs(_z(mean, [r[0] for r in ref], se))) < ZMAX
        assert np.max(np.abs(_z(g, np.array([r[1] for r in ref]), gse))) < ZMAX


def test_single_region_is_walk_on_boundary(oracle_mod):
    """N = 1 reduces WoI to the WoB estimator of Sec. 2 (alpha = 2, q = 1 on a sphere):
    its expectation is the exact truncated series of the interior Neumann problem."""
    p = W.concentric(3, [0.8], [2.0], [W.dirpoly([0, 0, 0], {(0, 1, 0): 1.5})])
    op = oracle_mod.OracleProblem(p)
    pts = np.array([[0.1, 0.2, 0.3], [-0.4, 0.1, 0.0], [0.0, -0.6, 0.2]])
    H = lambda x: x[1]; gH = lambda x: np.array([0.0, 1.0, 0.0])
    for M in (0, 3, 6):
        mean, se, g, gse, _ = oracle_mod.estimate(op, pts, 100000, M, seed=2)
        ref = [CF.concentric_uM([0.8], [2.0], [1.5], 1, 3, M, x, H, gH) for x in pts]
        assert np.max(np.abs(_z(mean, [r[0] for r in ref], se))) < ZMAX
        assert np.max(np.abs(_z(g, np.array([r[1] for r in ref]), gse))) < ZMAX


@pytest.mark.parametrize("dim,axes", [(2, [0.9, 0.5]), (3, [0.9, 0.6, 0.4]), (4, [0.8, 0.6, 0.5, 0.4])])
def test_ellipsoid_depolarization_gradient(oracle_mod, dim, axes):
    p, A, Q = W.single_ellipsoid_linear(dim, axes, direction=0)
    op = oracle_mod.OracleProblem(p)
    pts = np.random.default_rng(0).standard_normal((3, dim)) * 0.1
    for M in (1, 3):
        _, _, g, gse, _ = oracle_mod.estimate(op, pts, 100000, M, seed=9)
        gref = CF.ellipsoid_grad_uM(axes, Q, 0, M)
        assert np.max(np.abs(_z(g, gref[None, :], gse))) < ZMAX


def _star_tree(nv=512):
    star = W.star_polyline([0.05, -0.02], 0.5, 0.2, 5, nv, phase=0.3)
    shapes = [W.sphere([0, 0], 1.0), star, W.sphere([0.05, 0.0], 0.12), W.sphere([0.72, 0.35], 0.08)]
    parent = [-1, 0, 1, 0]
    sigma = [1.0, 2.5, 0.8, 4.0]
    coefs = [(0.0, [0.7, -0.3], [0.2, 0.5]), (0.0, [0.3, 0.0, 0.4], [-0.2, 0.1, 0.0]),
             (0.0, [0.5], [0.5]), (0.0, [-0.4, 0.2], [0.3, 0.0])]
    data = [W.fourier(s.center, *cf) for s, cf in zip(shapes, coefs)]
    curves = [CF.Curve([0, 0], 1.0, n=256), CF.Curve([0.05, -0.02], 0.5, 0.2, 5, 0.3, n=1024),
              CF.Curve([0.05, 0.0], 0.12, n=256), CF.Curve([0.72, 0.35], 0.08, n=256)]
    bf = [CF.fourier_b(s.center, *cf) for s, cf in zip(shapes, coefs)]
    return W.Problem(2, parent, sigma, shapes, data, 2, "star-tree"), curves, bf


STAR_PTS = np.array([[0.0, 0.3], [-0.5, -0.6], [0.3, 0.1], [0.62, 0.2], [-0.2, -0.25], [0.8, -0.3]])


def test_star_tree_matches_nystrom(oracle_mod):
    """Non-convex polyline interface (line/ray hit counts q > 1), nested and sibling regions."""
    p, curves, bf = _star_tree()
    op = oracle_mod.OracleProblem(p)
    for M in (1, 3):
        u, gu = CF.nystrom_uM(curves, p.parent, p.sigma, bf, M, STAR_PTS)
        mean, se, g, gse, cnt = oracle_mod.estimate(op, STAR_PTS, 200000, M, seed=4)
        assert np.max(np.abs(_z(mean, u, se))) < ZMAX
        assert np.max(np.abs(_z(g, gu, gse))) < ZMAX


def _nonconvex_root():
    coefs = (0.0, [0.0, 0.4, -0.3, 0.2], [0.0, 0.3, 0.1, 0.0])
    p = W.Problem(2, [-1], [1.0], [W.star_polyline([0.0, 0.0], 0.8, 0.45, 4, 1024, phase=0.2)],
                  [W.fourier([0, 0], *coefs)], 2, "nonconvex-root")
    return p, [CF.Curve([0, 0], 0.8, 0.45, 4, 0.2, n=2048)], [CF.fourier_b([0, 0], *coefs)]


NC_PTS = np.array([[0.0, 0.1], [0.3, 0.3], [-0.3, -0.2], [0.5, 0.0], [0.1, -0.4]])


def test_nonconvex_boundary_matches_nystrom(oracle_mod):
    """Strongly non-convex outer boundary (N = 1): every step is a line with q >= 1 hits."""
    p, curves, bf = _nonconvex_root()
    op = oracle_mod.OracleProblem(p)
    for M in (1, 2):
        u, gu = CF.nystrom_uM(curves, p.parent, p.sigma, bf, M, NC_PTS)
        mean, se, g, gse, _ = oracle_mod.estimate(op, NC_PTS, 100000, M, seed=4)
        assert np.max(np.abs(_z(mean, u, se))) < ZMAX
        assert np.max(np.abs(_z(g, gu, gse))) < ZMAX


def test_vr_same_mean_as_plain_on_star_tree(oracle_mod):
    p, curves, bf = _star_tree()
    op = oracle_mod.OracleProblem(p)
    u, _ = CF.nystrom_uM(curves, p.parent, p.sigma, bf, 2, STAR_PTS)
    mean, se, _, _, _ = oracle_mod.estimate(op, STAR_PTS, 400000, 2, seed=8, estimator=1)
    assert np.max(np.abs(_z(mean, u, se))) < ZMAX


# ----------------------------------------------------------------------------- naive Markov trees
# The naive estimator (Sec. 4.2, Eq. naive_woi_estimator) sums every interface tuple over an
# N-ary Markov tree instead of scheduling one (Theorem 2): same expectation as WoI, so the same
# exact u_M; its cost per tree is the tree size sum_{i=0}^{M} N^{i+1} interface points (the
# paper counts the root x as well).
def _tree_nodes(N, M):
    return sum(N ** (i + 1) for i in range(M + 1))


@pytest.mark.parametrize("M", [0, 1, 3])
def test_naive_concentric_disk_exact_expectation(oracle_mod, M):
    p, xs = W.concentric_disk_2d()
    op = oracle_mod.OracleProblem(p)
    pts = xs[::5]
    T = 40000
    mean, se, g, gse, cnt = oracle_mod.estimate(op, pts, T, M, seed=20 + M, estimator=oracle_mod.NAIVE)
    H, gH = CF.harmonic_2d(1, "cos")
    ref = [CF.concentric_uM(*CFG1, 1, 2, M, x, H, gH) for x in pts]
    z = _z(mean, [r[0] for r in ref], se)
    zg = _z(g, np.array([r[1] for r in ref]), gse)
    assert np.max(np.abs(z)) < ZMAX and np.max(np.abs(zg)) < ZMAX
    assert 0.3 < np.mean(np.concatenate([z, zg.ravel()]) ** 2) < 2.0
    assert cnt["cap_hits"] == 0
    assert cnt["walk_steps"] == len(pts) * T * _tree_nodes(2, M)


def test_naive_sphere_3d_exact_expectation(oracle_mod):
    p = W.zheng_ex3_3d()
    op = oracle_mod.OracleProblem(p)
    pts = np.array([[0.2, 0.1, -0.1], [0.5, -0.3, 0.2], [-0.1, 0.7, 0.1], [0.05, -0.2, 0.33], [0, 0, 0.9]])
    Hx, gx = CF.harmonic_x1(3)
    mean, se, g, gse, _ = oracle_mod.estimate(op, pts, 40000, 2, seed=21, estimator=oracle_mod.NAIVE)
    ref = [CF.concentric_uM([1, .4], [1, .5], [5, 0], 1, 3, 2, x, Hx, gx) for x in pts]
    assert np.max(np.abs(_z(mean, [r[0] for r in ref], se))) < ZMAX
    assert np.max(np.abs(_z(g, np.array([r[1] for r in ref]), gse))) < ZMAX


def test_naive_star_tree_matches_nystrom(oracle_mod):
    """Polyline lines/rays with q > 1 hits, sibling and nested regions (N = 4)."""
    p, curves, bf = _star_tree()
    op = oracle_mod.OracleProblem(p)
    u, gu = CF.nystrom_uM(curves, p.parent, p.sigma, bf, 2, STAR_PTS)
    mean, se, g, gse, cnt = oracle_mod.estimate(op, STAR_PTS, 20000, 2, seed=22, estimator=oracle_mod.NAIVE)
    assert np.max(np.abs(_z(mean, u, se))) < ZMAX
    assert np.max(np.abs(_z(g, gu, gse))) < ZMAX
    assert cnt["walk_steps"] == len(STAR_PTS) * 20000 * _tree_nodes(4, 2)


def test_naive_trace_matches_estimate_and_rejects_bad_queries(oracle_mod):
    p, xs = W.concentric_disk_2d()
    op = oracle_mod.OracleProblem(p)
    pts = xs[:3]
    F, G, T = oracle_mod.trace(op, pts, 2000, 2, seed=4, estimator=oracle_mod.NAIVE)
    mean, se, g, _, _ = oracle_mod.estimate(op, pts, 2000, 2, seed=4, estimator=oracle_mod.NAIVE)
    assert F.shape == (3, 2000, 1) and not T.any()
    assert np.allclose(F[:, :, 0].mean(1), mean, rtol=1e-12, atol=1e-15)
    assert np.allclose(G[:, :, 0].mean(1), g, rtol=1e-12, atol=1e-15)
    F2, _, _ = oracle_mod.trace(op, pts, 500, 2, seed=4, estimator=oracle_mod.NAIVE, walk_offset=1500)
    assert np.array_equal(F2, F[:, 1500:])
    for kw in ({"instance": 1}, {"batch_share": 2}):
        with pytest.raises(ValueError):
            oracle_mod.estimate(op, pts, 10, 2, estimator=oracle_mod.NAIVE, **kw)
    with pytest.raises(ValueError):   # node ids (N + 1)^(M + 1) = 3^20 exceed 2^31
        oracle_mod.estimate(op, pts, 10, 19, estimator=oracle_mod.NAIVE)


# ----------------------------------------------------------------------------- statistics
def test_standard_error_calibration_and_rate(oracle_mod):
    p, xs = W.concentric_disk_2d()
    op = oracle_mod.OracleProblem(p)
    H, gH = CF.harmonic_2d(1, "cos")
    ref = np.array([CF.concentric_uM(*CFG1, 1, 2, 4, x, H, gH)[0] for x in xs])
    mean, se, _, _, _ = oracle_mod.estimate(op, xs, 20000, 4, seed=77)
    z = _z(mean, ref, se)
    assert np.mean(np.abs(z) > 3) < 0.05
    assert 0.6 < np.mean(z ** 2) < 1.5
    ses = [oracle_mod.estimate(op, xs[:16], W_, 4, seed=5)[1].mean() for W_ in (2000, 8000, 32000)]
    slope = np.polyfit(np.log([2000, 8000, 32000]), np.log(ses), 1)[0]
    assert -0.55 < slope < -0.45


def test_trace_matches_estimate_and_resumes(oracle_mod):
    p, xs = W.concentric_disk_2d()
    op = oracle_mod.OracleProblem(p)
    pts = xs[:3]
    F, G, T = oracle_mod.trace(op, pts, 3000, 3, seed=4)
    mean, se, g, gse, _ = oracle_mod.estimate(op, pts, 3000, 3, seed=4)
    assert np.allclose(F[:, :, 0].mean(1), mean, rtol=1e-12, atol=1e-15)
    assert np.allclose(G[:, :, 0].mean(1), g, rtol=1e-12, atol=1e-15)
    assert np.allclose(F[:, :, 0].std(1, ddof=1) / np.sqrt(3000), se, rtol=1e-10)
    F2, _, T2 = oracle_mod.trace(op, pts, 1000, 3, seed=4, walk_offset=2000)
    assert np.array_equal(F2, F[:, 2000:]) and np.array_equal(T2, T[:, 2000:])


def test_shared_trajectories_batch(oracle_mod):
    """Points sharing a batch (B > 1) see identical schedules and trajectories; estimates stay exact."""
    p, xs = W.concentric_disk_2d()
    op = oracle_mod.OracleProblem(p)
    pts = xs[::4]
    F, G, T = oracle_mod.trace(op, pts, 200, 4, seed=4, batch_share=4)
    for b in range(0, len(pts), 4):
        assert all(np.array_equal(T[b] & 0xFF, T[b + j] & 0xFF) for j in range(1, 4))
    H, gH = CF.harmonic_2d(1, "cos")
    ref = np.array([CF.concentric_uM(*CFG1, 1, 2, 4, x, H, gH)[0] for x in pts])
    for sm in (0, 1):
        mean, se, _, _, _ = oracle_mod.estimate(op, pts, 100000, 4, seed=12, batch_share=4, schedule_mode=sm)
        assert np.max(np.abs(_z(mean, ref, se))) < ZMAX


# ----------------------------------------------------------------------------- planted mistakes
@pytest.mark.parametrize("plant", [1, 2, 3, 4, 5, 6, 7])
def test_pins_reject_planted_mistakes(oracle_mod, tmp_path, plant):
    """Each plausible mistake, planted in a copy of the oracle, fails one of the pins above."""
    libv = oracle_mod.load(oracle_mod.build_variant(plant, str(tmp_path)))
    if plant == 5:   # q matters only on non-convex interfaces
        p, curves, bf = _nonconvex_root()
        op = oracle_mod.OracleProblem(p, library=libv)
        u, gu = CF.nystrom_uM(curves, p.parent, p.sigma, bf, 1, NC_PTS)
        mean, se, g, gse, _ = oracle_mod.estimate(op, NC_PTS, 100000, 1, seed=4)
        z = np.concatenate([_z(mean, u, se), _z(g, gu, gse).ravel()])
    elif plant == 6:  # |alpha| in the naive tree weights (alpha_2 < 0 here)
        p, xs = W.concentric_disk_2d()
        op = oracle_mod.OracleProblem(p, library=libv)
        pts = xs[::6]
        H, gH = CF.harmonic_2d(1, "cos")
        ref = [CF.concentric_uM(*CFG1, 1, 2, 1, x, H, gH)[0] for x in pts]
        mean, se, _, _, _ = oracle_mod.estimate(op, pts, 100000, 1, seed=4, estimator=oracle_mod.NAIVE)
        z = _z(mean, ref, se)
    elif plant == 7:  # wrong ellipsoid Jacobian in the VR half-measures: the VR gradient is off
        axes = [0.9, 0.6, 0.4]
        p, A, Q = W.single_ellipsoid_linear(3, axes, direction=0)
        op = oracle_mod.OracleProblem(p, library=libv)
        pts = np.random.default_rng(0).standard_normal((3, 3)) * 0.1
        _, _, g, gse, _ = oracle_mod.estimate(op, pts, 100000, 1, seed=19, estimator=1)
        z = _z(g, CF.ellipsoid_grad_uM(axes, Q, 0, 1)[None, :], gse).ravel()
        assert op.info()["area_plus"][0] != pytest.approx(CF.ellipsoid3_area(*axes) / 2, rel=1e-3)
    elif plant == 4:  # normal at the wrong end of K* matters for the "other" transition
        p = W.concentric(2, [1.0, 0.5], [1.0, 3.0], [W.fourier([0, 0], 0, [0.5], [1.0]), W.fourier([0, 0], 0, [1.0], [0.0])])
        op = oracle_mod.OracleProblem(p, library=libv)
        pts = np.array([[0.1, 0.2], [0.6, -0.3], [-0.7, 0.1]])
        H, gH = CF.harmonic_2d(1, "cos"); Hs, gHs = CF.harmonic_2d(1, "sin")
        ref = [CF.concentric_uM([1, .5], [1, 3], [0.5, 1.0], 1, 2, 2, x, H, gH)[0] +
               CF.concentric_uM([1, .5], [1, 3], [1.0, 0.0], 1, 2, 2, x, Hs, gHs)[0] for x in pts]
        mean, se, _, _, _ = oracle_mod.estimate(op, pts, 800000, 2, seed=4)
        z = _z(mean, ref, se)
    else:
        p, xs = W.concentric_disk_2d()
        op = oracle_mod.OracleProblem(p, library=libv)
        pts = xs[::6]
        H, gH = CF.harmonic_2d(1, "cos")
        ref = [CF.concentric_uM(*CFG1, 1, 2, 1, x, H, gH)[0] for x in pts]
        mean, se, _, _, _ = oracle_mod.estimate(op, pts, 200000, 1, seed=4)
        z = _z(mean, ref, se)
    assert np.max(np.abs(z)) > 8, f"planted mistake {plant} not detected: max |z| = {np.max(np.abs(z)):.2f}"


# ----------------------------------------------------------------------------- point charge
def test_point_charge_data_is_the_flux_jump():
    """The point-charge workload's data are the flux jumps of u = |x|^(2-m) as the problem
    defines them: b_1 = sigma_1 d_n u on the outer boundary and, with the jump taken as exterior
    minus interior, b_i = (sigma_parent - sigma_i) d_n u on interface i (checked against a
    central difference of u along the normal)."""
    for m in (3, 4, 5, 6):
        p, _ = W.point_charge_ellipsoids(m)
        rng = np.random.default_rng(m)
        for i, (s, d) in enumerate(zip(p.shapes, p.data)):
            L = np.linalg.cholesky(np.linalg.inv(s.A))
            for _ in range(5):
                z = rng.normal(size=m)
                y = s.center + L @ (z / np.linalg.norm(z))            # on the ellipsoid
                n = s.A @ (y - s.center)
                n /= np.linalg.norm(n)
                h = 1e-6
                dnu = (W.point_charge_potential(y + h * n)[0] - W.point_charge_potential(y - h * n)[0]) / (2 * h)
                jump = p.sigma[0] if i == 0 else p.sigma[p.parent[i]] - p.sigma[i]
                b = d.coef[0] * np.dot(y - d.center, n) / np.linalg.norm(y - d.center) ** m
                assert abs(b - jump * dnu) <= 1e-6 * (1 + abs(b)), (m, i, b, jump * dnu)


def test_point_charge_ellipsoids_match_potential(oracle_mod):
    """Three nested ellipsoids around a point charge (3D, M = 5): the estimate equals
    u = 1/|x| up to the additive constant the Neumann problem leaves free (differences between
    points) and the gradient equals grad u, at points in each of the three regions."""
    p, pts = W.point_charge_ellipsoids(3)

    def inside(s, x):
        e = x - s.center
        return np.einsum("ij,jk,ik->i", e, s.A, e) < 1

    in2, in3 = inside(p.shapes[1], pts), inside(p.shapes[2], pts)
    x = np.concatenate([pts[~in2][:3], pts[in2 & ~in3][:3], pts[in3][:3]])
    u, gu = W.point_charge_potential(x)
    mean, se, g, gse, _ = oracle_mod.estimate(oracle_mod.OracleProblem(p), x, 1000000, 5, seed=2)
    d = (mean - mean[0]) - (u - u[0])
    assert np.max(np.abs(d[1:] / np.sqrt(se[1:] ** 2 + se[0] ** 2))) < ZMAX
    assert np.max(np.abs((g - gu) / gse)) < ZMAX


# ----------------------------------------------------------------------------- triangle meshes
def test_mesh_surface_samples(oracle_mod):
    """Uniform sampling on a triangle mesh: samples lie on their triangles' planes, and the
    fraction of samples per triangle matches its share of the area (chi-square)."""
    sh = W.icosphere([0.1, -0.2, 0.05], 0.8, 2, jitter=0.05, seed=3)
    p = W.Problem(3, [-1], [1.0], [sh], [W.zero_data(3)], 2, "mesh")
    op = oracle_mod.OracleProblem(p)
    n = 200000
    y = op.sample_surface(0, 5, n)
    V, T = sh.vertices, sh.triangles
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    nrm = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(nrm, axis=1)
    nrm /= (2 * area)[:, None]
    # the triangle of each sample: on its plane and inside its edges (barycentric test)
    d = np.abs(np.einsum("tk,ntk->nt", nrm, y[:, None, :] - a[None]))
    tri = np.argmin(d, axis=1)
    assert np.max(d[np.arange(n), tri]) < 1e-12
    counts = np.bincount(tri, minlength=len(T))
    expect = n * area / area.sum()
    chi2 = np.sum((counts - expect) ** 2 / expect)
    dof = len(T) - 1
    assert abs(chi2 - dof) < 5 * np.sqrt(2 * dof)


def test_mesh_sphere_matches_depolarization(oracle_mod):
    """A 1280-triangle icosphere with linear Neumann data: the gradient matches the exact u_M
    of the sphere (depolarization factor 1/3) up to the O(h^2) mesh error (0.5 % of the area)."""
    sh = W.icosphere([0, 0, 0], 1.0, 3)
    p = W.Problem(3, [-1], [1.0], [sh], [W.field_flux([1.0, 0.0, 0.0])], 0, "icosphere")
    op = oracle_mod.OracleProblem(p)
    pts = np.random.default_rng(0).standard_normal((3, 3)) * 0.1
    for M in (1, 3):
        _, _, g, gse, _ = oracle_mod.estimate(op, pts, 200000, M, seed=9)
        gref = CF.ellipsoid_grad_uM([1.0, 1.0, 1.0], np.eye(3), 0, M)
        assert np.max(np.abs(_z(g, gref[None, :], gse))) < ZMAX


def test_nested_meshes_match_concentric_spheres(oracle_mod):
    """Two nested icospheres (R = 1 and 0.5, 1280 triangles each) with l = 1 data: means and
    gradients match the exact u_M of concentric spheres (rays, lines and uniform transitions
    on meshes), with the O(h^2) mesh error far below the Monte Carlo error."""
    shapes = [W.icosphere([0, 0, 0], 1.0, 3), W.icosphere([0, 0, 0], 0.5, 3)]
    lam, sig = [1.0, -0.5], [1.0, 4.0]
    data = [W.dirpoly([0, 0, 0], {(1, 0, 0): lam[0]}), W.dirpoly([0, 0, 0], {(1, 0, 0): lam[1]})]
    p = W.Problem(3, [-1, 0], sig, shapes, data, 0, "nested-icospheres")
    op = oracle_mod.OracleProblem(p)
    x = np.array([[0.2, 0.1, -0.1], [0.7, -0.2, 0.1], [-0.3, 0.3, 0.35]])
    H, gH = CF.harmonic_x1(3)
    M = 3
    mean, se, g, gse, _ = oracle_mod.estimate(op, x, 200000, M, seed=4)
    for k, xk in enumerate(x):
        u, gu = CF.concentric_uM([1.0, 0.5], sig, lam, 1, 3, M, xk, H, gH)
        assert abs(mean[k] - u) < ZMAX * se[k]
        assert np.max(np.abs((g[k] - gu) / gse[k])) < ZMAX


# ----------------------------------------------------------------------------- surrogate training data
def test_training_grid_counts_lattice_points(oracle_mod):
    """Interior training points of the surrogate (Sec. 5): on the unit disk a grid of n = 2k + 1
    cells per axis has its centres at 2 (a, b) / (2k + 1), a, b in -k..k, so the nodes inside are
    the integer pairs with a^2 + b^2 <= k (k + 1) (counted here over the integers); with a margin,
    the nodes within it of the circles r = 1 and r = 0.5 are dropped."""
    p, _ = W.concentric_disk_2d()
    op = oracle_mod.OracleProblem(p)
    for k in (1, 2, 5, 13, 30):
        x, _, _, _ = op.training_points(2 * k + 1)
        a = np.arange(-k, k + 1)
        count = int(((a[:, None] ** 2 + a[None, :] ** 2) <= k * (k + 1)).sum())
        assert len(x) == count, (k, len(x), count)
        assert np.allclose(x * (2 * k + 1) / 2, np.round(x * (2 * k + 1) / 2), atol=1e-12)
    x, _, _, _ = op.training_points(61, margin=0.1)
    a = np.arange(-30, 31) * 2 / 61
    X, Y = np.meshgrid(a, a, indexing="ij")
    r = np.hypot(X, Y)
    keep = (r < 1) & (np.abs(r - 1) > 0.1) & (np.abs(r - 0.5) > 0.1)
    assert len(x) == int(keep.sum())
    assert np.allclose(x, np.stack([X[keep], Y[keep]], 1), atol=1e-14)   # row-major, last coordinate fastest


def test_training_grid_polyline_inside(oracle_mod):
    """A non-convex L-shaped polyline: its 8 x 8 cell centres (box [0, 2]^2) are inside unless both
    coordinates exceed 1: 48 nodes."""
    L = W.Shape(W.POLYLINE, np.array([0.6, 0.6]), 0.0, None,
                np.array([[0, 0], [2, 0], [2, 1], [1, 1], [1, 2], [0, 2]], dtype=np.float64))
    p = W.Problem(2, [-1], [1.0], [L], [W.zero_data(2)], 2, "L-shape")
    x, _, _, _ = oracle_mod.OracleProblem(p).training_points(8)
    assert len(x) == 48 and not np.any((x[:, 0] > 1) & (x[:, 1] > 1))


def test_training_boundary_samples(oracle_mod):
    """Boundary training points (Sec. 5, Eq. MLP_loss): uniform angles on dOmega with the outward
    normal and the normal-derivative target b_1 / sigma_1.  Circle: b = cos(theta), sigma_1 = 10;
    sphere: b = 5 x_1 / |x|; ellipsoid: on (y - c)^T A (y - c) = 1 with n = A y / |A y| and the
    uniform-field flux b = sigma n_1; star polyline: on the polyline, in the sampled direction from
    its vertex mean."""
    p, _ = W.concentric_disk_2d()
    _, y, n, f = oracle_mod.OracleProblem(p).training_points(5, bc_n=64)
    th = 2 * np.pi * np.arange(64) / 64
    assert np.allclose(y, np.stack([np.cos(th), np.sin(th)], 1), atol=1e-14) and np.allclose(n, y, atol=1e-14)
    assert np.allclose(f, np.cos(th) / 10.0, atol=1e-14)
    _, y, n, f = oracle_mod.OracleProblem(W.zheng_ex3_3d()).training_points(3, bc_n=6)
    assert len(y) == 72 and np.allclose(np.linalg.norm(y, axis=1), 1.0) and np.allclose(n, y)
    assert np.allclose(f, 5.0 * y[:, 0] / 1.0)
    pe, A, Q = W.single_ellipsoid_linear(3, [0.9, 0.6, 0.4], sigma=2.0)
    _, y, n, f = oracle_mod.OracleProblem(pe).training_points(3, bc_n=5)
    assert np.allclose(np.einsum("ij,jk,ik->i", y, A, y), 1.0, atol=1e-12)
    Ay = y @ A
    assert np.allclose(n, Ay / np.linalg.norm(Ay, axis=1, keepdims=True), atol=1e-12)
    assert np.allclose(f, n[:, 0], atol=1e-12)                         # b = sigma n . e_1, target b / sigma
    star = W.star_polyline([0.05, -0.02], 0.5, 0.2, 5, 512, phase=0.3)
    ps = W.Problem(2, [-1], [1.0], [star], [W.zero_data(2)], 2, "star")
    _, y, n, f = oracle_mod.OracleProblem(ps).training_points(3, bc_n=40)
    z = star.vertices.mean(0)
    th = 2 * np.pi * np.arange(40) / 40
    d = (y - z) / np.linalg.norm(y - z, axis=1, keepdims=True)
    assert np.allclose(d, np.stack([np.cos(th), np.sin(th)], 1), atol=1e-12)
    v, w = star.vertices, np.roll(star.vertices, -1, 0)
    e = w - v
    dist = [np.min(np.abs(e[:, 0] * (q - v)[:, 1] - e[:, 1] * (q - v)[:, 0]) / np.linalg.norm(e, axis=1)) for q in y]
    assert np.max(dist) < 1e-13 and np.all(f == 0.0)
