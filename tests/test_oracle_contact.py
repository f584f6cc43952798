"""Pins of the oracle's contact-radius protocols (Sec. Dynamics): (i) the
interface cut by the plane z = z_cut, mean distance of the cut to its centre;
(ii) the area of the flat lower part of the interface taken as a circle's.

A spherical cap cut at height z has the closed-form radius sqrt(R^2 - (z -
z_c)^2); the flat base of a cap mesh is a polygon whose area a convex hull
gives independently."""
import math

import numpy as np
import pytest
from scipy.spatial import ConvexHull

import oracle as o
import workloads as wl


@pytest.mark.parametrize("theta", [60.0, 90.0, 120.0])
def test_protocol_i_on_a_spherical_cap(theta):
    R, base = 20.0, 2.0
    V, T = wl.cap_mesh(R, theta, base, 24, (40.0, 40.0))
    zc = base - R * math.cos(math.radians(theta))  # centre height of the cap's sphere
    for z in (base + 0.7, base + 3.1, base + 6.0):
        want = math.sqrt(R * R - (z - zc) ** 2)
        got = o.contact_radius_3d(V, T, z)
        assert abs(got - want) < 5e-3 * want, (z, got, want)


def test_protocol_ii_is_the_base_disc_of_a_cap():
    """With a tolerance below the height of the rim triangles only the
    triangles lying on the flat base count: their union is the convex hull
    of the base vertices less a strip at most one edge wide along its rim."""
    R, base = 15.0, 2.0
    V, T = wl.cap_mesh(R, 90.0, base, 16, (30.0, 30.0))
    on_base = np.abs(V[:, 2] - base) < 1e-12
    hull = ConvexHull(V[on_base][:, :2])
    r_hull = math.sqrt(hull.volume / math.pi)  # 2D hull: volume is the area
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    edge = float(np.max(np.linalg.norm(V[e[:, 1]] - V[e[:, 0]], axis=1)))
    rim = V[~on_base][:, 2].min() - base  # lowest vertex off the base
    r1 = o.contact_radius_flat_3d(V, T, 1e-6 * R)
    assert r_hull - edge <= r1 <= r_hull
    assert o.contact_radius_flat_3d(V, T, 0.9 * rim) == r1
    # a tolerance above the rim height also takes the rim triangles
    assert o.contact_radius_flat_3d(V, T, 1.5 * rim) > r1


def test_protocol_ii_ignores_the_flat_top():
    """A full sphere's two polar caps are equally flat; only the lower one
    counts."""
    V, T = wl.sphere_mesh(10.0, 12, (20.0, 20.0, 15.0))
    tol = 0.05 * 10.0
    z = V[:, 2]
    lower = np.all(z[T] < 15.0, axis=1)
    flat = (z[T].max(axis=1) - z[T].min(axis=1)) < tol
    assert np.any(flat & ~lower) and np.any(flat & lower)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    want = math.sqrt(area[flat & lower].sum() / math.pi)
    assert abs(o.contact_radius_flat_3d(V, T, tol) - want) < 1e-12 * want


def test_protocols_2d_on_a_cap_polygon():
    R, base, th = 30.0, 2.0, 70.0
    q = wl.cap_polygon(R, th, base, 240, 80.0)
    rb = R * math.sin(math.radians(th))
    # (ii): the base edges are exactly flat and span the base nodes; the
    # edges that leave the base rise by more than the tolerance
    xb = q[np.abs(q[:, 1] - base) < 1e-9, 0]
    want = 0.5 * (xb.max() - xb.min())
    assert abs(o.contact_radius_flat_2d(q, 1e-9) - want) < 1e-12 * want
    assert rb - 2 * math.pi * R / 240 < want <= rb
    # (i): chord of the circle at height z
    zc = base - R * math.cos(math.radians(th))
    for z in (base + 0.5, base + 4.0):
        want = math.sqrt(R * R - (z - zc) ** 2)
        assert abs(o.contact_radius_2d(q, z) - want) < 2e-3 * want
