"""Seeded synthetic inputs for the Walk-on-Interfaces hot path.

This module is shared by the tests, the benchmark and the smoke check.  It only
builds problem descriptions (region tree, conductivities, interface geometry,
jump data) and evaluation points; it contains none of the estimator's arithmetic.
Geometry follows the paper's problem statement (Sec. 1, Eq. interface_problem):
region 0 is the root whose interface is the outer boundary, every other region
has a unique parent and its interface lies strictly inside the parent's.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SPHERE, ELLIPSOID, POLYLINE, MESH3D = 0, 1, 2, 3
SHAPE_MESH3D = MESH3D
DATA_ZERO, DATA_FOURIER2D, DATA_DIRPOLY, DATA_SOURCE_FLUX, DATA_FIELD_FLUX = 0, 1, 2, 3, 4


@dataclass
class Shape:
    kind: int
    center: np.ndarray
    radius: float = 0.0
    A: Optional[np.ndarray] = None          # ellipsoid: (y-c)^T A (y-c) = 1
    vertices: Optional[np.ndarray] = None   # polyline: (n, 2), counter-clockwise; mesh: (n, 3)
    triangles: Optional[np.ndarray] = None  # mesh: (t, 3) vertex indices, counter-clockwise from outside


@dataclass
class Data:
    kind: int
    center: np.ndarray
    coef: np.ndarray = field(default_factory=lambda: np.zeros(0))
    exps: Optional[np.ndarray] = None       # DIRPOLY: (n_terms, m) uint8

    @property
    def n_terms(self) -> int:
        if self.kind == DATA_FOURIER2D:
            return (len(self.coef) - 1) // 2
        if self.kind == DATA_DIRPOLY:
            return len(self.coef)
        return len(self.coef)


@dataclass
class Problem:
    dim: int
    parent: List[int]
    sigma: List[float]
    shapes: List[Shape]
    data: List[Data]
    compat_mode: int = 0                    # 0 per interface, 1 global balance, 2 none
    name: str = ""
    compat_tol: float = 1e-8                # relative tolerance of the compatibility check

    @property
    def n_regions(self) -> int:
        return len(self.parent)


# ----------------------------------------------------------------------------- shapes
def sphere(center, radius) -> Shape:
    return Shape(SPHERE, np.asarray(center, dtype=np.float64), float(radius))


def ellipsoid(center, A) -> Shape:
    return Shape(ELLIPSOID, np.asarray(center, dtype=np.float64), 0.0, np.asarray(A, dtype=np.float64))


def star_polyline(center, r0, amp, k, n, phase=0.0) -> Shape:
    """Closed CCW polyline through r(t) = r0 (1 + amp cos(k (t - phase))) at t_j = 2 pi j / n."""
    t = 2.0 * np.pi * np.arange(n) / n
    r = r0 * (1.0 + amp * np.cos(k * (t - phase)))
    c = np.asarray(center, dtype=np.float64)
    v = np.stack([c[0] + r * np.cos(t), c[1] + r * np.sin(t)], axis=1)
    return Shape(POLYLINE, c, 0.0, None, v)


# ----------------------------------------------------------------------------- data
def mesh(vertices, triangles) -> Shape:
    """Closed 3D triangle mesh, outward normal (b - a) x (c - a) for triangle (a, b, c)."""
    v = np.asarray(vertices, dtype=np.float64)
    return Shape(SHAPE_MESH3D, v.mean(0), vertices=v, triangles=np.asarray(triangles, dtype=np.int32))


def icosphere(center, radius, subdiv, jitter=0.0, seed=0) -> Shape:
    """Icosahedron subdivided `subdiv` times (20 * 4^subdiv triangles), vertices on the sphere,
    optionally moved radially by up to `jitter` (relative) to break the symmetry."""
    t = (1 + 5 ** 0.5) / 2
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    v = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6),
         (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        mid = {}

        def m(a, b):
            k = (min(a, b), max(a, b))
            if k not in mid:
                p = v[a] + v[b]
                v.append(p / np.linalg.norm(p))
                mid[k] = len(v) - 1
            return mid[k]
        f = [g for a, b, c in f for g in ((a, m(a, b), m(c, a)), (b, m(b, c), m(a, b)), (c, m(c, a), m(b, c)),
                                          (m(a, b), m(b, c), m(c, a)))]
    V = np.array(v)
    if jitter:
        V *= (1 + jitter * np.random.default_rng(seed).uniform(-1, 1, (len(V), 1)))
    return mesh(np.asarray(center, dtype=np.float64) + radius * V, np.array(f, dtype=np.int32))


def zero_data(m) -> Data:
    return Data(DATA_ZERO, np.zeros(m))


def fourier(center, a0, a, c) -> Data:
    """b = a0 + sum_k a_k cos(k th) + c_k sin(k th), th the polar angle about center."""
    coef = [a0]
    for ak, ck in zip(a, c):
        coef += [ak, ck]
    return Data(DATA_FOURIER2D, np.asarray(center, dtype=np.float64), np.asarray(coef, dtype=np.float64))


def dirpoly(center, terms) -> Data:
    """b = sum_t coef_t prod_d e_d^{exps_t,d}, e = (y - center)/|y - center|; terms: {exps: coef}."""
    items = [(tuple(int(x) for x in e), float(v)) for e, v in terms.items() if v != 0.0]
    m = len(center)
    if not items:
        items = [(tuple([0] * m), 0.0)]
    exps = np.array([e for e, _ in items], dtype=np.uint8).reshape(-1, m)
    coef = np.array([v for _, v in items], dtype=np.float64)
    return Data(DATA_DIRPOLY, np.asarray(center, dtype=np.float64), coef, exps)


def field_flux(g) -> Data:
    """b(y) = n(y) . g: the normal flux of the uniform field g (u_h linear)."""
    g = np.asarray(g, dtype=np.float64)
    return Data(DATA_FIELD_FLUX, np.zeros(len(g)), g.copy())


def source_flux(source, kappa) -> Data:
    """b(y) = kappa (y - s).n(y) / |y - s|^m: the normal flux of a point source at s."""
    return Data(DATA_SOURCE_FLUX, np.asarray(source, dtype=np.float64), np.array([float(kappa)]))


def real_sph_harm_polys(l: int):
    """Real spherical harmonics of degree l on S^2 as polynomials in (x, y, z)
    (unnormalised): Re/Im (x + i y)^k * d^k P_l / dz^k (z).  Returns a list of
    {exps: coef} dicts, 2l + 1 of them."""
    from numpy.polynomial import legendre as L
    P = np.zeros(l + 1); P[l] = 1.0
    Pz = L.leg2poly(P)                       # power-series coefficients of P_l(z)
    out = []
    for k in range(l + 1):
        dk = np.polynomial.polynomial.polyder(Pz, k) if k else Pz
        # (x + i y)^k = sum_j C(k,j) x^{k-j} (i y)^j
        re, im = {}, {}
        from math import comb
        for j in range(k + 1):
            c = comb(k, j)
            ij = [1, 0, -1, 0][j % 4], [0, 1, 0, -1][j % 4]
            for zp, dz in enumerate(dk):
                if dz == 0.0:
                    continue
                key = (k - j, j, zp)
                if ij[0]:
                    re[key] = re.get(key, 0.0) + ij[0] * c * dz
                if ij[1]:
                    im[key] = im.get(key, 0.0) + ij[1] * c * dz
        out.append(re)
        if k > 0:
            out.append(im)
    return out


# ----------------------------------------------------------------------------- points
def polar_grid_points(n_r=8, n_t=8):
    """n_r x n_t points at radii (a + 1/2)/n_r and angles 2 pi b / n_t."""
    pts = []
    for a in range(n_r):
        for b in range(n_t):
            r, t = (a + 0.5) / n_r, 2 * np.pi * b / n_t
            pts.append([r * np.cos(t), r * np.sin(t)])
    return np.array(pts)


def ball_points(rng, n, m, radius=1.0):
    g = rng.standard_normal((n, m))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return radius * g * rng.random((n, 1)) ** (1.0 / m)


# ----------------------------------------------------------------------------- problems
def concentric(dim, radii, sigma, data) -> Problem:
    """Concentric spheres about 0, region i inside region i-1."""
    n = len(radii)
    return Problem(dim, [-1] + list(range(n - 1)), list(sigma),
                   [sphere(np.zeros(dim), r) for r in radii], list(data))


def concentric_disk_2d(M=4):
    """Unit disk (sigma 10) with a concentric disk r = 0.5 (sigma 1); b = cos(th) on both."""
    m = 2
    data = [fourier([0, 0], 0.0, [1.0], [0.0]) for _ in range(2)]
    p = concentric(m, [1.0, 0.5], [10.0, 1.0], data)
    p.name = "disk-circle-cos"
    return p, polar_grid_points(8, 8)


def bower_ex3_2d(lam=20.0, alpha=0.4, sig=1.0 / 3.0, mode=3):
    """Concentric circles of radius 1 and alpha, sigma_2/sigma_1 = sig,
    d_r u = lam sin(mode th) on r = 1, homogeneous flux jump (Sec. 5, Example 3)."""
    a = np.zeros(mode); c = np.zeros(mode); c[mode - 1] = lam
    data = [fourier([0, 0], 0.0, a, c), zero_data(2)]
    p = concentric(2, [1.0, alpha], [1.0, sig], data)
    p.name = "bower-ex3-2d"
    return p


def zheng_ex3_3d(lam=5.0, alpha=0.4, sig=0.5):
    """Concentric spheres of radius 1 and alpha, d_r u = lam sin(phi)cos(th) = lam x/r on r = 1."""
    data = [dirpoly([0, 0, 0], {(1, 0, 0): lam}), zero_data(3)]
    p = concentric(3, [1.0, alpha], [1.0, sig], data)
    p.name = "zheng-ex3-3d"
    return p


def nested_spheres_6d():
    """Unit 6-ball, spheres 0.7 > 0.35, sigma (1, 5, 0.2), b_j = c_j + lam_j x1/|x| (global balance)."""
    m = 6
    c2, c3 = 1.0, -0.5
    c1 = c2 * 0.7 ** 5 + c3 * 0.35 ** 5
    cs, lams = [c1, c2, c3], [1.0, 0.5, -0.3]
    e1 = tuple([1] + [0] * (m - 1))
    data = [dirpoly(np.zeros(m), {tuple([0] * m): cj, e1: lj}) for cj, lj in zip(cs, lams)]
    p = concentric(m, [1.0, 0.7, 0.35], [1.0, 5.0, 0.2], data)
    p.compat_mode = 1
    p.name = "6ball-nested"
    pts = ball_points(np.random.default_rng(6), 1024, m)
    return p, pts


def _polyline_distance(v, p):
    a = v; b = np.roll(v, -1, axis=0)
    e = b - a
    t = np.clip(((p - a) * e).sum(1) / (e * e).sum(1), 0.0, 1.0)
    q = a + t[:, None] * e
    return np.min(np.linalg.norm(q - p, axis=1))


def _inside_star(center, r0, amp, k, p):
    d = np.asarray(p) - center
    t = np.arctan2(d[1], d[0])
    return np.hypot(d[0], d[1]) < r0 * (1 + amp * np.cos(k * t))


def _fourier_mean_removed(rng, shape, center, K=5):
    a = rng.standard_normal(K); c = rng.standard_normal(K)
    a0 = 0.0
    if shape.kind == POLYLINE:
        # arclength mean of the Fourier series over the closed polyline (4-point Gauss per segment)
        v = shape.vertices; w = np.roll(v, -1, axis=0)
        gx, gw = np.polynomial.legendre.leggauss(4)
        tot, acc = 0.0, 0.0
        for x, wt in zip(gx, gw):
            f = 0.5 * (x + 1)
            y = v + f * (w - v)
            th = np.arctan2(y[:, 1] - center[1], y[:, 0] - center[0])
            b = sum(a[j] * np.cos((j + 1) * th) + c[j] * np.sin((j + 1) * th) for j in range(K))
            seg = np.linalg.norm(w - v, axis=1)
            acc += 0.5 * wt * (seg * b).sum(); tot += 0.5 * wt * seg.sum()
        a0 = -acc / tot
    return fourier(center, a0, a, c)


def star_tree_2d(n_vertices=2048, n_points=4096, near_frac=0.25):
    """Unit disk with 3 nested stars r0(1 + 0.2 cos k t), (r0, k) = (0.7, 3) > (0.4, 5) > (0.2, 7),
    and 5 circular inclusions of radius U[0.03, 0.05] placed with clearance 0.01."""
    stars = [(0.70, 3), (0.40, 5), (0.20, 7)]
    amp = 0.2
    shapes = [sphere([0.0, 0.0], 1.0)]
    parent = [-1]
    for j, (r0, k) in enumerate(stars):
        shapes.append(star_polyline([0.0, 0.0], r0, amp, k, n_vertices))
        parent.append(j)
    rng = rng_place = np.random.default_rng(11)
    circles = []
    while len(circles) < 5:
        r = rng_place.uniform(0.03, 0.05)
        c = rng_place.uniform(-1, 1, 2)
        if np.hypot(*c) > 1.0 - r - 0.01:
            continue
        ok = all(_polyline_distance(s.vertices, c) > r + 0.01 for s in shapes[1:4])
        ok = ok and all(np.hypot(*(c - cc)) > r + rr + 0.01 for cc, rr in circles)
        if not ok:
            continue
        circles.append((c, r))
    for c, r in circles:
        par = 0
        for j, (r0, k) in enumerate(stars):
            if _inside_star(np.zeros(2), r0, amp, k, c):
                par = j + 1
        shapes.append(sphere(c, r))
        parent.append(par)
    N = len(shapes)
    sigma = list(10.0 ** np.random.default_rng(1).uniform(-1, 2, N))
    rng_d = np.random.default_rng(2)
    data = [_fourier_mean_removed(rng_d, s, s.center) for s in shapes]
    prob = Problem(2, parent, sigma, shapes, data, 0, "disk-3stars-5circles")
    pts = _star_tree_points(prob, np.random.default_rng(3), n_points, near_frac)
    return prob, pts


def _star_tree_points(prob, rng, n, near_frac):
    n_near = int(round(n * near_frac))
    far = []
    while len(far) < n - n_near:
        p = ball_points(rng, 1, 2)[0]
        if _min_interface_distance(prob, p) > 1e-3:
            far.append(p)
    near = []
    N = prob.n_regions
    while len(near) < n_near:
        h = rng.integers(0, N)
        s = prob.shapes[h]
        off = rng.uniform(1e-5, 1e-3) * (1 if rng.random() < 0.5 else -1)
        if s.kind == POLYLINE:
            j = rng.integers(0, len(s.vertices))
            a = s.vertices[j]; b = s.vertices[(j + 1) % len(s.vertices)]
            e = b - a
            nrm = np.array([e[1], -e[0]]) / np.linalg.norm(e)
            p = 0.5 * (a + b) + off * nrm
        else:
            t = rng.uniform(0, 2 * np.pi)
            u = np.array([np.cos(t), np.sin(t)])
            p = s.center + (s.radius + off) * u
        if np.hypot(*p) < 1.0:
            near.append(p)
    return np.concatenate([np.array(far), np.array(near)], axis=0)


def _min_interface_distance(prob, p):
    d = np.inf
    for s in prob.shapes:
        if s.kind == POLYLINE:
            d = min(d, _polyline_distance(s.vertices, p))
        elif s.kind == SPHERE:
            d = min(d, abs(np.linalg.norm(p - s.center) - s.radius))
    return d


def star_tree_instances_2d(n_inst=512, seed=4, n_vertices=512, scale_points=1.0, scale_walks=1.0):
    """Independent 2D instances with 1-16 circle/star interfaces in a random nesting tree.
    Returns a list of (problem, points, W)."""
    rng = np.random.default_rng(seed)
    out = []
    for it in range(n_inst):
        n_if = int(rng.integers(1, 17))
        shapes = [sphere([0.0, 0.0], 1.0)]
        parent = [-1]
        # bounding radius / inner radius of each region for placement
        bound = [(np.zeros(2), 1.0, 1.0)]
        children = {0: []}
        tries = 0
        while len(shapes) < n_if + 1 and tries < 5000:
            tries += 1
            par = int(rng.integers(0, len(shapes)))
            pc, pr_out, pr_in = bound[par]
            is_star = rng.random() < 0.5
            size = rng.uniform(0.15, 0.45) * pr_in
            r_out = size * (1.2 if is_star else 1.0)
            r_in = size * (0.8 * np.cos(np.pi / n_vertices) if is_star else 1.0)
            room = pr_in - r_out - 0.01
            if room <= 0 or r_out < 0.02:
                continue
            ang = rng.uniform(0, 2 * np.pi); rad = room * np.sqrt(rng.random())
            c = pc + rad * np.array([np.cos(ang), np.sin(ang)])
            ok = all(np.linalg.norm(c - bound[s][0]) > r_out + bound[s][1] + 0.01 for s in children[par])
            if not ok:
                continue
            if is_star:
                k = int(rng.integers(3, 8))
                shapes.append(star_polyline(c, size, 0.2, k, n_vertices, phase=rng.uniform(0, 2 * np.pi)))
            else:
                shapes.append(sphere(c, size))
            parent.append(par)
            idx = len(shapes) - 1
            bound.append((c, r_out, r_in))
            children[par].append(idx)
            children[idx] = []
        N = len(shapes)
        sigma = list(10.0 ** rng.uniform(-1, 3, N))
        data = [_fourier_mean_removed(rng, s, s.center) for s in shapes]
        P = max(1, int(round(2 ** rng.uniform(4, 10) * scale_points)))
        W = max(2, int(round(10 ** rng.uniform(3, 6) * scale_walks)))
        pts = ball_points(rng, P, 2, 0.999)
        out.append((Problem(2, parent, sigma, shapes, data, 0, f"inst{it}"), pts, W))
    return out


def _haar_rotation(rng, m):
    q, r = np.linalg.qr(rng.standard_normal((m, m)))
    return q * np.sign(np.diag(r))


def ellipsoid_tree_3d(n_points=16384):
    """Unit ball; concentric spheres 0.6 > 0.3; 10 ellipsoids (semi-axes U[0.03, 0.08],
    Haar rotation, clearance 0.01).  Data: real SH l = 1..4 (coefficient N(0,1)/(l+1)) on
    spheres, odd l in {1, 3} on ellipsoids (mean zero on centrally symmetric surfaces)."""
    m = 3
    rng = np.random.default_rng(50)
    shapes = [sphere(np.zeros(3), 1.0), sphere(np.zeros(3), 0.6), sphere(np.zeros(3), 0.3)]
    parent = [-1, 0, 1]
    placed = []
    while len(placed) < 10:
        ax = rng.uniform(0.03, 0.08, 3)
        rmax = ax.max()
        c = ball_points(rng, 1, 3, 1.0 - rmax - 0.01)[0]
        rc = np.linalg.norm(c)
        if any(abs(rc - R) < rmax + 0.01 for R in (0.6, 0.3)):
            continue
        if any(np.linalg.norm(c - cc) < rmax + rr + 0.01 for cc, rr, _ in placed):
            continue
        Q = _haar_rotation(rng, 3)
        A = Q @ np.diag(1.0 / ax ** 2) @ Q.T
        placed.append((c, rmax, A))
    for c, rmax, A in placed:
        rc = np.linalg.norm(c)
        par = 2 if rc < 0.3 else (1 if rc < 0.6 else 0)
        shapes.append(ellipsoid(c, A))
        parent.append(par)
    N = len(shapes)
    sigma = list(10.0 ** np.random.default_rng(51).uniform(np.log10(0.5), np.log10(50), N))
    rng_d = np.random.default_rng(52)
    data = []
    for i, s in enumerate(shapes):
        ls = (1, 2, 3, 4) if s.kind == SPHERE else (1, 3)
        terms = {}
        for l in ls:
            for poly in real_sph_harm_polys(l):
                cf = rng_d.standard_normal() / (l + 1)
                for e, v in poly.items():
                    terms[e] = terms.get(e, 0.0) + cf * v
        data.append(dirpoly(s.center, terms))
    prob = Problem(3, parent, sigma, shapes, data, 0, "ball-2spheres-10ellipsoids")
    pts = ball_points(np.random.default_rng(5), n_points, 3)
    return prob, pts


def single_ellipsoid_linear(dim, semi_axes, rotation_seed=7, direction=0, sigma=1.0):
    """One ellipsoid region with Neumann data b = sigma n . e_direction (u_h = x_direction)."""
    rng = np.random.default_rng(rotation_seed)
    Q = _haar_rotation(rng, dim)
    A = Q @ np.diag(1.0 / np.asarray(semi_axes, dtype=np.float64) ** 2) @ Q.T
    g = np.zeros(dim); g[direction] = sigma
    return Problem(dim, [-1], [sigma], [ellipsoid(np.zeros(dim), A)],
                   [field_flux(g)], 0, "single-ellipsoid"), A, Q


def point_charge_ellipsoids(dim, n_points=10000, seed=8, sigma=(1.1, 1.3, 0.9)):
    """Three nested ellipsoids (x - c)^T A (x - c) = 1 around the potential u = |x|^(2-m) of a
    unit point charge at the origin (outside every region), in m = dim >= 3 dimensions:
    centres (1.3, 0, ...), (1.4, 0, ...), (1.6, 0, ...); diag A = (1, 0.9, 1.2, ...),
    (1.5, 3.2, 2, ...) with A12 = -1, (8, 6, 4, ...) with A12 = -2; sigma = (1.1, 1.3, 0.9).
    Data from u itself: b_1 = sigma_1 d_n u on the outer boundary and b_i = (sigma_parent -
    sigma_i) d_n u on the interfaces, with d_n u = (2 - m) y.n / |y|^m (a point-source flux).
    Points uniform in the outer ellipsoid (rejection from its bounding box).  u solves the
    problem for any sigma (the data follow it).  As printed, the middle ellipsoid crosses the
    outer one (its surface reaches (x - c1)^T A1 (x - c1) = 1.137); its matrix is scaled by 1.2
    so that the tree is nested (surface within 0.964 of the outer form, the inner one within
    0.923 of the middle form, in every dimension)."""
    m = int(dim)
    assert m >= 3
    diag = [[1.0, 0.9] + [1.2] * (m - 2), [1.5, 3.2] + [2.0] * (m - 2), [8.0, 6.0] + [4.0] * (m - 2)]
    off = [0.0, -1.0, -2.0]
    cx = [1.3, 1.4, 1.6]
    sigma = [float(v) for v in sigma]
    shapes, data = [], []
    for i in range(3):
        A = np.diag(diag[i])
        A[0, 1] = A[1, 0] = off[i]
        if i == 1:
            A *= 1.2
        c = np.zeros(m); c[0] = cx[i]
        shapes.append(ellipsoid(c, A))
        kappa = (2 - m) * (sigma[0] if i == 0 else sigma[i - 1] - sigma[i])
        data.append(source_flux(np.zeros(m), kappa))
    # the data integrate to zero exactly; the compiler's surface quadrature resolves that to
    # about 2e-7 of the integral of |b| in 6D, so the check runs at 1e-5
    prob = Problem(m, [-1, 0, 1], sigma, shapes, data, 0, f"point-charge-ellipsoids-{m}d", 1e-5)
    rng = np.random.default_rng(seed + m)
    A1, c1 = shapes[0].A, shapes[0].center
    half = 1.0 / np.sqrt(np.linalg.eigvalsh(A1)[0])
    pts = []
    while sum(len(q) for q in pts) < n_points:
        x = c1 + rng.uniform(-half, half, (4 * n_points, m))
        e = x - c1
        pts.append(x[np.einsum("ij,jk,ik->i", e, A1, e) < 1.0])
    return prob, np.concatenate(pts)[:n_points]


def point_charge_potential(x):
    """u = |x|^(2-m) and its gradient, the exact solution of point_charge_ellipsoids."""
    x = np.asarray(x, dtype=np.float64)
    m = x.shape[-1]
    r = np.linalg.norm(x, axis=-1)
    return r ** (2 - m), ((2 - m) * r ** (-m))[..., None] * x


def mesh_tree_3d(n_points=4096, subdiv=3, seed=12):
    """Triangle-mesh interfaces: a jittered icosphere (R = 1, 20 4^subdiv triangles) around a
    jittered icosphere (R = 0.45, centre (0.1, -0.05, 0.02)) and a sphere sibling (R = 0.15 at
    (-0.55, 0.3, 0.1)); sigma (1, 4, 0.5); quadratic direction-polynomial data with N(0, 1)
    coefficients (no compatibility requirement); points uniform in the ball of radius 0.85."""
    shapes = [icosphere([0.0, 0.0, 0.0], 1.0, subdiv, jitter=0.03, seed=1),
              icosphere([0.1, -0.05, 0.02], 0.45, subdiv, jitter=0.05, seed=2),
              sphere([-0.55, 0.3, 0.1], 0.15)]
    rng = np.random.default_rng(seed)
    data = [dirpoly(sh.center, {(1, 0, 0): rng.normal(), (0, 1, 1): rng.normal(), (2, 0, 0): rng.normal(),
                                (0, 0, 1): rng.normal()}) for sh in shapes]
    prob = Problem(3, [-1, 0, 0], [1.0, 4.0, 0.5], shapes, data, 2, "mesh-tree-3d")
    return prob, ball_points(np.random.default_rng(seed + 1), n_points, 3, 0.85)


WORKLOAD_DESCRIPTIONS = {
    "concentric_disk_2d": "unit disk, concentric circle r=0.5, sigma 10/1, b = cos(theta); 64 points, W=1e4, M=4",
    "star_tree_2d": "unit disk, 3 nested stars (k=3,5,7) + 5 circles, sigma 10^U(-1,2), Fourier data; 4096 points, "
                    "W=1e5, M=4",
    "star_tree_instances_2d": "512 uneven instances, 1-16 interfaces, 16-1024 points, W 1e3-1e6, M=4",
    "ellipsoid_tree_3d": "unit ball, spheres 0.6/0.3, 10 ellipsoids, SH data; 16384 points, W=1e5 (VR), M=6",
    "nested_spheres_6d": "unit 6-ball, spheres 0.7/0.35, sigma (1,5,0.2), c + lam x1/|x| data; 1024 points, W=1e6, M=8",
    "point_charge_ellipsoids": "3 nested ellipsoids around the potential |x|^(2-m) of a point charge outside them, "
                               "m = 3..6; 1e4 points, M = m + 2",
    "mesh_tree_3d": "jittered icospheres (1280 triangles each) around a sphere sibling, direction-polynomial data; "
                    "4096 points, M = 4",
}
