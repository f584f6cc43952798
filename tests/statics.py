"""Shape comparison of a simulated equilibrium droplet with the App. B
solution (eq. L2-error_equilibrium).  Test infrastructure shared by the GPU
statics test."""
import math

import numpy as np

from oracle import shape as sh


def volume_centroid(q, tris):
    """Volume and centroid of the closed mesh (tetrahedra on the origin)."""
    a, b, c = q[tris[:, 0]], q[tris[:, 1]], q[tris[:, 2]]
    v = np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0
    cen = ((a + b + c) / 4.0 * v[:, None]).sum(axis=0) / v.sum()
    return float(v.sum()), cen


def radial_profile(q, centre, nbins):
    """Mean distance of the nodes from centre per bin of polar angle (from
    +z) over [0, pi]."""
    d = q - centre[None, :]
    G = np.linalg.norm(d, axis=1)
    phi = np.arccos(np.clip(d[:, 2] / G, -1.0, 1.0))
    k = np.minimum((phi / math.pi * nbins).astype(int), nbins - 1)
    s = np.bincount(k, weights=G, minlength=nbins)
    n = np.bincount(k, minlength=nbins)
    return s / np.maximum(n, 1), n


def theory(theta, eps):
    """App. B solution, reached by continuation from theta = pi/2 at
    xi/R0 = 0.1 (where the truncated-cap guess converges): first in the angle
    (steps of pi/16), then in xi/R0 (steps of at most 0.02)."""
    s = sh.solve(math.pi / 2, 0.1)
    th = math.pi / 2
    while abs(th - theta) > 1e-12:
        th = th + max(-math.pi / 16, min(math.pi / 16, theta - th))
        s = sh.solve(th, 0.1, guess=s)
    e = 0.1
    while abs(e - eps) > 1e-12:
        e = e + max(-0.02, min(0.02, eps - e))
        s = sh.solve(theta, e, guess=s)
    return s


def l2_error(q, tris, theta, xi, nbins=90):
    """eq. L2-error_equilibrium: G_sim from the nodes about the droplet's
    centroid, G_theo about the centroid of the App. B solution of the same
    volume (R0 from the simulated volume), over phi in [0, pi]."""
    V, cen = volume_centroid(q, tris)
    R0 = (3.0 * V / (4.0 * math.pi)) ** (1.0 / 3.0)
    s = theory(theta, xi / R0)
    Gs, n = radial_profile(q, cen, nbins)
    phis = (np.arange(nbins) + 0.5) * math.pi / nbins
    Gt = R0 * sh.radial_profile_about(s["u"], s["g"], sh.centroid_height(s["u"], s["g"]), phis)
    sel = n > 0
    err = math.sqrt(np.sum((Gs[sel] - Gt[sel]) ** 2) / np.sum(Gt[sel] ** 2))
    return dict(E_L2=err, R0=R0, theta_bar_theory=sh.angle_from_half_height(s["ell"]),
                ell_theory=s["ell"] * R0, bins_filled=int(sel.sum()))


def theory_2d(theta, eps):
    """Planar outline, reached by the same continuation as theory(): from
    theta = pi/2 at xi/R0 = 0.1 first in the angle, then in xi/R0."""
    s = sh.solve_2d(math.pi / 2, 0.1)
    th = math.pi / 2
    while abs(th - theta) > 1e-12:
        th = th + max(-math.pi / 16, min(math.pi / 16, theta - th))
        s = sh.solve_2d(th, 0.1, guess=s)
    e = 0.1
    while abs(e - eps) > 1e-12:
        e = e + max(-0.02, min(0.02, eps - e))
        s = sh.solve_2d(theta, e, guess=s)
    return s


def l2_error_2d(q, theta, xi, nbins=90):
    """2D counterpart of eq. L2-error_equilibrium: node distances from the
    polygon's area centroid, binned by the polar angle from +y folded onto
    [0, pi], against the 2D App. B-type outline of the same area."""
    x, y = q[:, 0], q[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    cr = x * yn - xn * y
    A = 0.5 * cr.sum()
    cen = np.array([((x + xn) * cr).sum() / (6 * A), ((y + yn) * cr).sum() / (6 * A)])
    R0 = math.sqrt(A / math.pi)
    s = theory_2d(theta, xi / R0)
    d = q - cen[None, :]
    G = np.linalg.norm(d, axis=1)
    phi = np.arccos(np.clip(d[:, 1] / G, -1.0, 1.0))
    k = np.minimum((phi / math.pi * nbins).astype(int), nbins - 1)
    Gs = np.bincount(k, weights=G, minlength=nbins) / np.maximum(np.bincount(k, minlength=nbins), 1)
    n = np.bincount(k, minlength=nbins)
    phis = (np.arange(nbins) + 0.5) * math.pi / nbins
    Gt = R0 * sh.radial_profile_about_2d(s["phi"], s["g"], sh.centroid_height_2d(s["phi"], s["g"]), phis)
    sel = n > 0
    err = math.sqrt(np.sum((Gs[sel] - Gt[sel]) ** 2) / np.sum(Gt[sel] ** 2))
    return dict(E_L2=err, R0=R0, ell_theory=s["ell"] * R0, area=A)
