"""Independent reference values that pin the oracle (no Monte Carlo, no shared code).

1. Concentric spheres in dimension m with data lambda_j Y_l on sphere j: every
   integral operator K*_{ij} of Sec. 3 acts on the degree-l harmonic Y_l as a scalar
   k_ij(l) (derived from the single-layer potential of Y_l on a sphere and the jump
   relation, Eq. interface_jump).  The truncated series of Eq. (approx_vector_form_gamma)
   then reduces to an N x N matrix power series, giving the exact expectation u_M of
   the estimator (Eq. finite_sum_approx_ux) for every M, and its gradient.
2. The paper's closed-form solutions of Example 3 (Sec. 5): concentric circles
   (Eq. C0_gradient_2D_analytical_soln) and spheres (Eq. C0_gradient_3D_analytical_soln,
   3 x 3 system) -- the M -> infinity limit of (1).
3. A single ellipsoid with Neumann data sigma n.e: the normal components along the
   principal axes are eigenfunctions of K* with eigenvalues 1/2 - L_k (L_k the
   depolarisation factors), so grad u_M is exact for every M.
4. 2D Nystrom discretisation of the integral operators on smooth closed curves
   (trapezoid rule, diagonal limit kappa/(4 pi)): a deterministic u_M for trees of
   circles and stars (non-convex interfaces, sibling regions).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


# ----------------------------------------------------------------------------- 1. concentric
def unit_sphere_area(m):
    return 2.0 * math.pi ** (m / 2) / math.gamma(m / 2)


def kstar_mode(l, m, Ri, Rj):
    """Scalar action of K*_{ij} (x on sphere i, density Y_l on sphere j) on Y_l."""
    if Ri == Rj:
        return 0.5 if l == 0 else (m - 2) / (2.0 * (2 * l + m - 2))
    if Rj < Ri:
        pre = 1.0 if (l == 0 and m == 2) else (l + m - 2) / (2 * l + m - 2)
        return pre * (Rj / Ri) ** (l + m - 1)
    if l == 0:
        return 0.0
    return -(l / (2 * l + m - 2)) * (Ri / Rj) ** (l - 1)


def alphas_scales(sigma, parent):
    N = len(sigma)
    a = np.zeros(N); s = np.zeros(N)
    a[0] = 2.0; s[0] = 2.0 / sigma[0]
    for i in range(1, N):
        sp, si = sigma[parent[i]], sigma[i]
        a[i] = 2 * (si - sp) / (sp + si); s[i] = -2.0 / (sp + si)
    return a, s


def series_weights(M):
    return [1.0 if i < M else 0.5 for i in range(M + 1)]


def concentric_density(radii, sigma, lam, l, m, M):
    """g^{(M)} = sum_i w_i Mmat^i beta_hat, for M = None the full series (I - Mmat)^{-1} beta_hat."""
    N = len(radii)
    a, s = alphas_scales(sigma, [-1] + list(range(N - 1)))
    K = np.array([[kstar_mode(l, m, radii[i], radii[j]) for j in range(N)] for i in range(N)])
    Mm = a[:, None] * K
    b = s * np.asarray(lam, dtype=np.float64)
    if M is None:
        return np.linalg.solve(np.eye(N) - Mm, b)
    g = np.zeros(N); v = b.copy()
    for i, w in enumerate(series_weights(M)):
        g += w * v
        v = Mm @ v
    return g


def single_layer_mode(l, m, R, x, H, gH):
    """Single-layer potential of Y_l on the sphere |y| = R at x and its gradient.
    H(x) = |x|^l Y_l(x/|x|) (harmonic polynomial), gH its gradient."""
    x = np.asarray(x, dtype=np.float64)
    r = np.linalg.norm(x)
    k = 2 * l + m - 2
    if l == 0 and m == 2:
        if r < R:
            return -R * math.log(R), np.zeros_like(x)
        return -R * math.log(r), -R * x / r ** 2
    if r < R:
        c = R ** (1 - l) / k
        return c * H(x), c * gH(x)
    c = R ** (l + m - 1) / k
    h = H(x)
    return c * h / r ** k, c * (gH(x) / r ** k - k * h * x / r ** (k + 2))


def concentric_uM(radii, sigma, lam, l, m, M, x, H, gH):
    """Exact expectation of the WoI estimator (and of its gradient) at x."""
    g = concentric_density(radii, sigma, lam, l, m, M)
    u = 0.0; gu = np.zeros(m)
    for j, R in enumerate(radii):
        v, dv = single_layer_mode(l, m, R, x, H, gH)
        u += g[j] * v; gu += g[j] * dv
    return u, gu


def harmonic_2d(l, kind):
    """cos(l th) or sin(l th) as the harmonic polynomial Re/Im (x + i y)^l."""
    def H(x):
        z = complex(x[0], x[1]) ** l
        return z.real if kind == "cos" else z.imag

    def gH(x):
        if l == 0:
            return np.zeros(2)
        d = l * complex(x[0], x[1]) ** (l - 1)
        # d/dx Re z^l = Re(l z^{l-1}), d/dy Re z^l = Re(i l z^{l-1}) = -Im(l z^{l-1})
        if kind == "cos":
            return np.array([d.real, -d.imag])
        return np.array([d.imag, d.real])
    return H, gH


def harmonic_x1(m):
    def H(x):
        return x[0]

    def gH(x):
        e = np.zeros(m); e[0] = 1.0
        return e
    return H, gH


def harmonic_const(m):
    return (lambda x: 1.0), (lambda x: np.zeros(m))


# ----------------------------------------------------------------------------- 2. Example 3
def bower_2d_exact(x, lam=20.0, alpha=0.4, sig=1.0 / 3.0, mode=3):
    """Eq. C0_gradient_2D_analytical_soln."""
    r = np.hypot(x[0], x[1]); th = math.atan2(x[1], x[0])
    A = (2.0 / mode) / (alpha ** (2 * mode) * (sig - 1) + sig + 1)
    B = A / 2 * (sig + 1); C = B - 1.0 / mode
    if r <= alpha:
        return lam * A * r ** mode * math.sin(mode * th)
    return lam * (B * r ** mode + C * r ** (-mode)) * math.sin(mode * th)


def zheng_3d_exact(x, lam=5.0, alpha=0.4, sig=0.5):
    """Eq. C0_gradient_3D_analytical_soln with its 3 x 3 system; Y_1^1 = sqrt(3/(4 pi)) x/r."""
    S = np.array([[0.0, 1.0, -2.0], [alpha, -alpha, -alpha ** -2], [sig, -1.0, 2 * alpha ** -3]])
    A, B, C = np.linalg.solve(S, np.array([math.sqrt(4 * math.pi / 3), 0.0, 0.0]))
    r = np.linalg.norm(x)
    Y = math.sqrt(3 / (4 * math.pi)) * x[0] / r
    if r <= alpha:
        return lam * A * r * Y
    return lam * (B * r + C / r ** 2) * Y


# ----------------------------------------------------------------------------- 3. ellipsoid
def depolarization(semi_axes):
    a = np.asarray(semi_axes, dtype=np.float64)
    pa = float(np.prod(a))
    out = []
    for k in range(len(a)):
        f = lambda s, k=k: 1.0 / ((s + a[k] ** 2) * np.prod(np.sqrt(s + a ** 2)))
        v, _ = integrate.quad(f, 0, np.inf, epsabs=1e-14, epsrel=1e-13, limit=500)
        out.append(pa / 2 * v)
    return np.array(out)


def ellipsoid_grad_uM(semi_axes, Q, direction, M):
    """grad u_M for one ellipsoid A = Q diag(a^-2) Q^T, data b = sigma n . e_direction."""
    L = depolarization(semi_axes)
    e = np.zeros(len(semi_axes)); e[direction] = 1.0
    grad = np.zeros(len(semi_axes))
    for k in range(len(semi_axes)):
        ck = Q[:, k] @ e
        G = sum(w * (1 - 2 * L[k]) ** i for i, w in enumerate(series_weights(M)))
        grad += 2 * ck * G * L[k] * Q[:, k]
    return grad


def ellipsoid3_area(a, b, c):
    """Surface area of a 3D ellipsoid (a >= b >= c) by Legendre's elliptic-integral formula."""
    from scipy.special import ellipeinc, ellipkinc
    a, b, c = sorted([a, b, c], reverse=True)
    phi = math.acos(c / a)
    k2 = a ** 2 * (b ** 2 - c ** 2) / (b ** 2 * (a ** 2 - c ** 2))
    E = ellipeinc(phi, k2); F = ellipkinc(phi, k2)
    return 2 * math.pi * c ** 2 + 2 * math.pi * a * b / math.sin(phi) * (E * math.sin(phi) ** 2 + F * math.cos(phi) ** 2)


# ----------------------------------------------------------------------------- 4. Nystrom 2D
class Curve:
    """Smooth closed curve z(t) = c + r(t)(cos t, sin t), r = r0 (1 + amp cos(k (t - phase)))."""

    def __init__(self, center, r0, amp=0.0, k=0, phase=0.0, n=512):
        t = 2 * np.pi * np.arange(n) / n
        r = r0 * (1 + amp * np.cos(k * (t - phase)))
        rp = -r0 * amp * k * np.sin(k * (t - phase))
        rpp = -r0 * amp * k * k * np.cos(k * (t - phase))
        ct, st = np.cos(t), np.sin(t)
        x = center[0] + r * ct; y = center[1] + r * st
        xp = rp * ct - r * st; yp = rp * st + r * ct
        xpp = rpp * ct - 2 * rp * st - r * ct; ypp = rpp * st + 2 * rp * ct - r * st
        sp = np.hypot(xp, yp)
        self.t = t
        self.pts = np.stack([x, y], 1)
        self.nrm = np.stack([yp / sp, -xp / sp], 1)
        self.w = sp * 2 * np.pi / n
        self.kappa = (xp * ypp - yp * xpp) / sp ** 3
        self.center = np.asarray(center, dtype=np.float64)


def nystrom_uM(curves, parent, sigma, bfuns, M, xs):
    """u_M and grad u_M at points xs via Nystrom on the curves; bfuns[i](pts) gives b_i."""
    a, s = alphas_scales(sigma, parent)
    pts = np.concatenate([c.pts for c in curves]); nrm = np.concatenate([c.nrm for c in curves])
    w = np.concatenate([c.w for c in curves]); kap = np.concatenate([c.kappa for c in curves])
    reg = np.concatenate([np.full(len(c.w), i) for i, c in enumerate(curves)])
    d = pts[:, None, :] - pts[None, :, :]
    r2 = (d ** 2).sum(-1)
    np.fill_diagonal(r2, 1.0)
    Kmat = (d * nrm[:, None, :]).sum(-1) / (2 * np.pi * r2) * w[None, :]
    np.fill_diagonal(Kmat, kap / (4 * np.pi) * w)
    Mm = a[reg][:, None] * Kmat
    beta = np.concatenate([s[i] * bfuns[i](c.pts) for i, c in enumerate(curves)])
    g = np.zeros_like(beta); v = beta.copy()
    for i, wt in enumerate(series_weights(M)):
        g += wt * v
        v = Mm @ v
    xs = np.asarray(xs, dtype=np.float64)
    dx = xs[:, None, :] - pts[None, :, :]
    rr2 = (dx ** 2).sum(-1)
    u = (-np.log(rr2) / (4 * np.pi) * (g * w)[None, :]).sum(1)
    gu = (-(dx / (2 * np.pi * rr2[..., None])) * (g * w)[None, :, None]).sum(1)
    return u, gu


def fourier_b(center, a0, a, c):
    def f(p):
        th = np.arctan2(p[:, 1] - center[1], p[:, 0] - center[0])
        out = np.full(len(p), a0, dtype=np.float64)
        for k, (ak, ck) in enumerate(zip(a, c), start=1):
            out += ak * np.cos(k * th) + ck * np.sin(k * th)
        return out
    return f
