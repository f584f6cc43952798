"""FP64 equilibrium shape of an axisymmetric droplet on the substrate (App. B,
eqs. YL, bc, volconstr; App. C, eqs. gcap, ell, angleh).

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: only tests/ and the
benchmark's measurement legs import it.  Plain numpy/scipy, written from
the appendix:

  unknowns   g(u) on a uniform grid of u = cos(phi) in [-1, 1] (the surface
             is r = R0 g(u) about an origin midway between the top and the
             bottom of the droplet), the gap delta between the bottom and
             the substrate, and k = dp R0 / sigma;
  equations  eq. YL at every grid point, with second-order central
             differences inside and second-order one-sided first
             derivatives at u = +-1 (where the second derivative drops out
             with its factor 1 - u^2); h = u g(u) + g(-1) + delta;
             eq. bc g(1) = g(-1); eq. volconstr (trapezoid rule).

Everything is in units of R0 (the radius of the sphere of the droplet's
volume); eps = xi / R0.
"""
from __future__ import annotations

import math

import numpy as np


def curvature(u, g, gd, gdd):
    """Divergence of the outward unit normal times R0 for r = R0 g(u), u =
    cos(phi) (App. B, the equation after eq. divn)."""
    s = (1.0 - u * u) * gd * gd + g * g
    return (u * g * gd - g * g - (1.0 - u * u) * g * gdd) / s ** 1.5 + (u * gd + 3.0 * g) / (g * np.sqrt(s))


def derivatives(g, du):
    """Second-order finite differences; one-sided first derivatives at the
    ends, where the second derivative is not needed."""
    gd = np.empty_like(g)
    gdd = np.zeros_like(g)
    gd[1:-1] = (g[2:] - g[:-2]) / (2.0 * du)
    gdd[1:-1] = (g[2:] - 2.0 * g[1:-1] + g[:-2]) / (du * du)
    gd[0] = (-3.0 * g[0] + 4.0 * g[1] - g[2]) / (2.0 * du)
    gd[-1] = (3.0 * g[-1] - 4.0 * g[-2] + g[-3]) / (2.0 * du)
    return gd, gdd


def wall_term(h, theta, eps, n=6, m=3):
    """Pi(h) R0 / sigma with A of eq. A_choice, h in units of R0 (eq. YL)."""
    return (m - 1) * (n - 1) / ((n - m) * eps) * (1.0 + math.cos(theta)) * (
        (eps / h) ** n - (eps / h) ** m)


def residual(x, u, theta, eps, n=6, m=3, wall=True):
    N = u.size
    g, delta, k = x[:N], x[N], x[N + 1]
    du = u[1] - u[0]
    gd, gdd = derivatives(g, du)
    r = curvature(u, g, gd, gdd) - k
    if wall:
        h = u * g + g[0] + delta
        r = r + wall_term(h, theta, eps, n, m)
    vol = du * (np.sum(g ** 3) - 0.5 * (g[0] ** 3 + g[-1] ** 3)) - 2.0
    return np.concatenate([r, [g[-1] - g[0], vol]])


def truncated_cap(u, theta):
    """Initial guess: the spherical cap of volume 4 pi / 3 meeting the wall at
    theta (eqs. contactr, voldrop, ell), seen from its mid-height: the
    sphere above the base plane, the plane below."""
    t = math.tan(theta / 2.0)
    rc = 2.0 / (t * (3.0 + t * t)) ** (1.0 / 3.0)  # eq. voldrop with R0 = 1
    Rc = rc / math.sin(theta)                        # eq. contactr
    ell = Rc * math.sin(theta / 2.0) ** 2            # eq. ell
    zc = ell - Rc                                    # sphere centre
    r_s = u * zc + np.sqrt(np.maximum(u * u * zc * zc - zc * zc + Rc * Rc, 0.0))
    with np.errstate(divide="ignore"):
        r_p = np.where(u < 0.0, ell / np.maximum(-u, 1e-300), np.inf)
    return np.minimum(r_s, r_p), Rc


def jacobian(x, u, theta, eps, n, m):
    """Jacobian of residual() by forward differences.  Grid value g_j enters
    the curvature rows j - 1 .. j + 1 only (and rows 0 or N - 1 through the
    one-sided end derivatives), so columns five apart share one perturbed
    evaluation; g_0 (through h), delta and k enter every row and get their
    own.  The rows of eqs. bc and volconstr are differentiated exactly."""
    N = u.size
    du = u[1] - u[0]
    r0 = residual(x, u, theta, eps, n, m)
    J = np.zeros((r0.size, x.size))

    def step(j):
        return 1e-7 * max(1.0, abs(x[j]))

    for j in (0, N, N + 1):
        xp = x.copy()
        xp[j] += step(j)
        J[:N, j] = (residual(xp, u, theta, eps, n, m)[:N] - r0[:N]) / step(j)
    for c in range(5):
        cols = np.arange(1 + c, N, 5)
        xp = x.copy()
        hs = np.array([step(j) for j in cols])
        xp[cols] += hs
        dr = residual(xp, u, theta, eps, n, m)[:N] - r0[:N]
        for j, hj in zip(cols, hs):
            rows = [i for i in (j - 1, j, j + 1) if 0 <= i < N]
            if j <= 2:
                rows.append(0)
            if j >= N - 3:
                rows.append(N - 1)
            for i in set(rows):
                J[i, j] = dr[i] / hj
    J[N, N - 1] = 1.0
    J[N, 0] = -1.0
    w = np.full(N, du)
    w[0] *= 0.5
    w[-1] *= 0.5
    J[N + 1, :N] = 3.0 * w * x[:N] ** 2
    return r0, J


def newton(x, u, theta, eps, n, m, tol=1e-10, iters=60):
    """Damped Newton: full steps while the residual norm falls, halved
    otherwise; the gap delta is kept positive."""
    N = u.size
    r, J = jacobian(x, u, theta, eps, n, m)
    nr = np.linalg.norm(r)
    for _ in range(iters):
        if nr < tol:
            break
        dx = np.linalg.solve(J, -r)
        lam = 1.0
        while lam > 1e-6:
            xn = x + lam * dx
            if xn[N] > 0.0 and np.all(xn[:N] > 0.0):
                rn = residual(xn, u, theta, eps, n, m)
                if np.all(np.isfinite(rn)) and np.linalg.norm(rn) < nr:
                    break
            lam *= 0.5
        else:
            break
        x = xn
        r, J = jacobian(x, u, theta, eps, n, m)
        nr = np.linalg.norm(r)
    return x, nr


def solve(theta, eps, N=801, n=6, m=3, guess=None):
    """Equilibrium profile for contact angle theta (radians) and eps = xi / R0.
    Returns dict(u, g, delta, k, ell) with ell = g(1) the half-height."""
    u = np.linspace(-1.0, 1.0, N)
    if guess is None:
        g0, Rc = truncated_cap(u, theta)
        x0 = np.concatenate([g0, [eps, 2.0 / Rc]])
    else:
        x0 = np.concatenate([np.interp(u, guess["u"], guess["g"]), [guess["delta"], guess["k"]]])
    x, nr = newton(x0, u, theta, eps, n, m)
    # the residual's rounding floor grows with 1/du^2 (second differences)
    if not np.isfinite(nr) or nr > 1e-9 * max(1.0, (N / 801.0) ** 2):
        raise RuntimeError(f"shape solver did not converge: |res| = {nr:.3e}")
    g = x[:N]
    return dict(u=u, g=g, delta=float(x[N]), k=float(x[N + 1]), ell=float(g[-1]))


def solve_continued(theta, eps, N=801, n=6, m=3, start_eps=0.3):
    """solve() reached by continuation from start_eps down to eps (each step
    starts from the previous solution)."""
    e, s = max(start_eps, eps), None
    while True:
        s = solve(theta, e, N, n, m, guess=s)
        if e <= eps:
            return s
        e = max(eps, e / 2.0)


def angle_from_half_height(ell):
    """eq. angleh with R0 = 1."""
    return 2.0 * math.atan(math.sqrt(3.0 * ell ** 3 / (1.0 - ell ** 3)))


def centroid_height(u, g):
    """Height of the centroid of the solid of revolution r <= g(u) above the
    origin: int z dV / int dV with dV = (2 pi / 3) g^3 du on each cone and
    z = (3/4) g u for the cone's centroid."""
    w = np.full_like(u, u[1] - u[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    V = np.sum(w * g ** 3)
    return float(np.sum(w * 0.75 * u * g ** 4) / V)


def radial_profile_about(u, g, z0, phis):
    """Distance from the axis point at height z0 (units of R0, relative to
    the origin of g) to the surface, along polar angles phis from the +z
    axis: solves |p| = G with p on the surface r = g(u) by sampling the
    surface densely and interpolating over its own polar angle about z0."""
    uu = np.linspace(-1.0, 1.0, 20001)
    gg = np.interp(uu, u, g)
    rho = gg * np.sqrt(np.maximum(1.0 - uu * uu, 0.0))
    z = gg * uu - z0
    ang = np.arctan2(rho, z)            # polar angle about the new centre
    dist = np.hypot(rho, z)
    order = np.argsort(ang)
    return np.interp(phis, ang[order], dist[order])


# --------------------------------------------------------------------------
# 2D counterpart (a droplet that is a long cylinder, the 2D model of this
# library): the outline r = R0 g(phi) in the plane, phi from the +z axis on
# [0, pi] by symmetry, origin midway between the top and the bottom.  The
# curvature of a polar curve replaces the divergence of eq. YL; the wall
# term is the same (the wedge argument of App. A is planar); the area of a
# circle of radius R0 replaces eq. volconstr.
# --------------------------------------------------------------------------

def curvature_2d(g, gd, gdd):
    """Curvature (times R0) of the polar curve r = g(phi)."""
    return (g * g + 2.0 * gd * gd - g * gdd) / (g * g + gd * gd) ** 1.5


def derivatives_2d(g, dphi):
    """Second-order central differences with the mirror symmetry of the
    outline about the axis at phi = 0 and phi = pi (g' = 0 there)."""
    ge = np.concatenate([[g[1]], g, [g[-2]]])
    gd = (ge[2:] - ge[:-2]) / (2.0 * dphi)
    gdd = (ge[2:] - 2.0 * g + ge[:-2]) / (dphi * dphi)
    return gd, gdd


def residual_2d(x, phi, theta, eps, n=6, m=3, wall=True):
    N = phi.size
    g, delta, k = x[:N], x[N], x[N + 1]
    dphi = phi[1] - phi[0]
    gd, gdd = derivatives_2d(g, dphi)
    r = curvature_2d(g, gd, gdd) - k
    if wall:
        h = g * np.cos(phi) + g[-1] + delta
        r = r + wall_term(h, theta, eps, n, m)
    area = dphi * (np.sum(g ** 2) - 0.5 * (g[0] ** 2 + g[-1] ** 2)) - math.pi
    return np.concatenate([r, [g[0] - g[-1], area]])


def solve_2d(theta, eps, N=801, n=6, m=3, guess=None):
    """2D equilibrium outline for contact angle theta and eps = xi / R0, from
    a truncated circular cap of the same area (or a previous solution).
    Returns dict(phi, g, delta, k, ell) with ell = g(0) the half-height."""
    phi = np.linspace(0.0, math.pi, N)
    if guess is None:
        # circular cap of area pi (R0 = 1): Rc^2 (theta - sin cos) = pi
        Rc = math.sqrt(math.pi / (theta - math.sin(theta) * math.cos(theta)))
        ell = Rc * math.sin(theta / 2.0) ** 2
        zc = ell - Rc
        u = np.cos(phi)
        r_s = u * zc + np.sqrt(np.maximum(u * u * zc * zc - zc * zc + Rc * Rc, 0.0))
        with np.errstate(divide="ignore"):
            r_p = np.where(u < 0.0, ell / np.maximum(-u, 1e-300), np.inf)
        x0 = np.concatenate([np.minimum(r_s, r_p), [eps, 1.0 / Rc]])
    else:
        x0 = np.concatenate([np.interp(phi, guess["phi"], guess["g"]), [guess["delta"], guess["k"]]])

    def res(x):
        return residual_2d(x, phi, theta, eps, n, m)

    dphi = phi[1] - phi[0]
    w = np.full(N, dphi)
    w[0] *= 0.5
    w[-1] *= 0.5

    def jac(x, r0):
        """Forward differences: g_j enters curvature rows j - 1 .. j + 1 only
        (the mirror ghosts keep rows 0 and N - 1 on g_1 and g_N-2), so columns
        five apart share an evaluation; g(pi) (through h), delta and k enter
        every row.  The rows of the end condition and the area are exact."""
        J = np.zeros((r0.size, x.size))
        for j in (N - 1, N, N + 1):
            hj = 1e-7 * max(1.0, abs(x[j]))
            xp = x.copy()
            xp[j] += hj
            J[:N, j] = (res(xp)[:N] - r0[:N]) / hj
        for c in range(5):
            cols = np.arange(c, N - 1, 5)
            hs = 1e-7 * np.maximum(1.0, np.abs(x[cols]))
            xp = x.copy()
            xp[cols] += hs
            dr = res(xp)[:N] - r0[:N]
            for j, hj in zip(cols, hs):
                for i in (j - 1, j, j + 1):
                    if 0 <= i < N:
                        J[i, j] = dr[i] / hj
        J[N, 0] = 1.0
        J[N, N - 1] = -1.0
        J[N + 1, :N] = 2.0 * w * x[:N]
        return J

    x = x0
    r = res(x)
    nr = np.linalg.norm(r)
    for _ in range(60):
        if nr < 1e-10:
            break
        J = jac(x, r)
        dx = np.linalg.solve(J, -r)
        lam = 1.0
        while lam > 1e-6:
            xn = x + lam * dx
            if xn[N] > 0.0 and np.all(xn[:N] > 0.0):
                rn = res(xn)
                if np.all(np.isfinite(rn)) and np.linalg.norm(rn) < nr:
                    break
            lam *= 0.5
        else:
            break
        x, r, nr = xn, rn, np.linalg.norm(rn)
    if not np.isfinite(nr) or nr > 1e-9 * max(1.0, (N / 801.0) ** 2):
        raise RuntimeError(f"2D shape solver did not converge: |res| = {nr:.3e}")
    g = x[:N]
    return dict(phi=phi, g=g, delta=float(x[N]), k=float(x[N + 1]), ell=float(g[0]))


def centroid_height_2d(phi, g):
    """Height of the centroid of the region r <= g(phi) above the origin:
    triangles of area g^2 dphi / 2 with centroids at (2/3) g cos(phi)."""
    w = np.full_like(phi, phi[1] - phi[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    return float(np.sum(w * g ** 3 * np.cos(phi)) * (2.0 / 3.0) / np.sum(w * g ** 2))


def radial_profile_about_2d(phi, g, z0, phis):
    """Distance from the axis point at height z0 to the outline along polar
    angles phis (from +z, in [0, pi])."""
    pp = np.linspace(0.0, math.pi, 20001)
    gg = np.interp(pp, phi, g)
    x = gg * np.sin(pp)
    z = gg * np.cos(pp) - z0
    ang = np.arctan2(x, z)
    dist = np.hypot(x, z)
    order = np.argsort(ang)
    return np.interp(phis, ang[order], dist[order])
