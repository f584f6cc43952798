"""Pins of the oracle's volume and angle-from-height diagnostics on exact caps.

App. C, eq. (angleh) with eq. (ell): the contact angle of a droplet is read
off its half-height l and the radius R0 of the sphere of equal volume.  For
a true spherical cap of circle radius Rc and angle theta, the volume is
pi Rc^3 (2 - 3 cos theta + cos^3 theta) / 3 and the height Rc (1 - cos
theta); the planar counterpart (a circular segment) has area
Rc^2 (theta - sin theta cos theta) and the same height.  These closed forms
are written here from elementary geometry, independently of the oracle.

The caps are meshed in the test itself: polygons and latitude-longitude
polyhedra whose vertices lie exactly on the circle or sphere, the apex and
the base included, so the height is exact and the enclosed area or volume
converges to the closed form at second order in the mesh spacing.  A wrong
equal-volume radius, a wrong cap-area formula or a transposed half-height
shifts the angle by degrees; the bounds below are hundredths of a degree.
"""
import math

import numpy as np
import pytest

import oracle as o

ANGLES = [20.0, 45.0, 90.0, 135.0, 160.0]


def segment_polygon(Rc, theta, n_arc, n_base):
    """CCW polygon of a circular cap of angle theta sitting on y = 0: n_arc
    points on the arc from the right contact point over the apex to the left
    one, then n_base - 1 points back along the flat base."""
    yc = -Rc * math.cos(theta)          # circle centre height
    a = np.linspace(-theta, theta, n_arc + 1)  # angle from the upward vertical (apex included)
    arc = np.stack([Rc * np.sin(-a), yc + Rc * np.cos(a)], axis=1)
    # arc[0] is the right contact point (x = Rc sin theta), arc[-1] the left
    xb = Rc * math.sin(theta)
    base = np.stack([np.linspace(-xb, xb, n_base + 1)[1:-1], np.zeros(n_base - 1)], axis=1)
    q = np.concatenate([arc, base])
    q[np.abs(q[:, 1]) < 1e-15, 1] = 0.0
    return q


def cap_polyhedron(Rc, theta, n_ring, n_az):
    """Closed latitude-longitude polyhedron of a spherical cap of angle theta
    on z = 0: an apex, n_ring rings at polar angles k theta / n_ring (the last
    one the contact circle, at z = 0), a centre vertex of the flat base.
    Triangles are counter-clockwise seen from outside."""
    zc = -Rc * math.cos(theta)
    verts = [(0.0, 0.0, zc + Rc)]
    az = 2.0 * math.pi * np.arange(n_az) / n_az
    for k in range(1, n_ring + 1):
        p = theta * k / n_ring
        z = 0.0 if k == n_ring else zc + Rc * math.cos(p)
        for a in az:
            verts.append((Rc * math.sin(p) * math.cos(a), Rc * math.sin(p) * math.sin(a), z))
    verts.append((0.0, 0.0, 0.0))
    q = np.array(verts)
    ring = lambda k, j: 1 + (k - 1) * n_az + (j % n_az)
    tris = []
    for j in range(n_az):
        tris.append((0, ring(1, j), ring(1, j + 1)))
    for k in range(1, n_ring):
        for j in range(n_az):
            a, b = ring(k, j), ring(k, j + 1)
            c, d = ring(k + 1, j), ring(k + 1, j + 1)
            tris.append((a, c, d))
            tris.append((a, d, b))
    centre = len(verts) - 1
    for j in range(n_az):
        tris.append((centre, ring(n_ring, j + 1), ring(n_ring, j)))
    return q, np.array(tris, dtype=np.int32)


def cap_volume(Rc, theta):
    c = math.cos(theta)
    return math.pi * Rc ** 3 * (2.0 - 3.0 * c + c ** 3) / 3.0


def segment_area(Rc, theta):
    return Rc * Rc * (theta - math.sin(theta) * math.cos(theta))


def test_closed_forms_against_quadrature():
    """The two closed forms themselves, against direct quadrature of the
    cap (horizontal slices), so that a typo in them cannot pin the oracle
    to a wrong value."""
    from scipy.integrate import quad
    for th in np.radians(ANGLES):
        Rc = 1.7
        zc = -Rc * math.cos(th)
        H = Rc * (1.0 - math.cos(th))
        v, _ = quad(lambda z: math.pi * (Rc * Rc - (z - zc) ** 2), 0.0, H, epsabs=1e-13)
        a, _ = quad(lambda z: 2.0 * math.sqrt(max(Rc * Rc - (z - zc) ** 2, 0.0)), 0.0, H,
                    epsabs=1e-13, limit=200)
        assert abs(v - cap_volume(Rc, th)) < 1e-9 * cap_volume(Rc, th)
        assert abs(a - segment_area(Rc, th)) < 1e-7 * segment_area(Rc, th)


@pytest.mark.parametrize("theta_deg", ANGLES)
def test_2d_area_and_angle_on_exact_segments(theta_deg):
    th = math.radians(theta_deg)
    Rc = 40.0
    errs = []
    for n_arc in (2048, 4096, 8192):
        q = segment_polygon(Rc, th, n_arc, n_arc // 4)
        area = o.volume_2d(q)
        assert area > 0.0  # counter-clockwise
        ell = 0.5 * float(q[:, 1].max() - q[:, 1].min())
        assert abs(2.0 * ell - Rc * (1.0 - math.cos(th))) < 1e-9 * Rc
        errs.append(abs(area - segment_area(Rc, th)) / segment_area(Rc, th))
        t = o.angle_from_height_2d(ell, area)
        # the inscribed polygon's area falls short by O((theta / n_arc)^2):
        # at 4096 arc points below 1e-6 relative, a hundredth of a degree
        # is far above what that moves the angle
        if n_arc >= 4096:
            assert abs(math.degrees(t) - theta_deg) < 0.01, (theta_deg, math.degrees(t))
            assert errs[-1] < 1e-6
    # inscribed polygon: second-order convergence of the area
    assert 3.5 < errs[0] / errs[1] < 4.5
    assert 3.5 < errs[1] / errs[2] < 4.5


@pytest.mark.parametrize("theta_deg", ANGLES)
def test_3d_volume_and_angle_on_exact_caps(theta_deg):
    th = math.radians(theta_deg)
    Rc = 12.0
    errs, angles = [], []
    for n_ring, n_az in ((48, 192), (96, 384)):
        q, tris = cap_polyhedron(Rc, th, n_ring, n_az)
        vol = o.volume_3d(q, tris)
        assert vol > 0.0  # outward orientation
        H = float(q[:, 2].max() - q[:, 2].min())
        assert abs(H - Rc * (1.0 - math.cos(th))) < 1e-9 * Rc
        errs.append(abs(vol - cap_volume(Rc, th)) / cap_volume(Rc, th))
        angles.append(math.degrees(o.angle_from_height_3d(0.5 * H, vol)))
    # the inscribed polyhedron's volume deficit: 1e-4 to 2.5e-4 relative at
    # 96 rings, second order in the mesh spacing; the angle it moves grows
    # towards 180 deg (0.03 deg at 160 deg), and the second-order
    # extrapolation of the two meshes removes it
    assert errs[1] < 3e-4
    assert 3.5 < errs[0] / errs[1] < 4.5
    assert abs(angles[1] - theta_deg) < 0.04, (theta_deg, angles)
    assert abs((4.0 * angles[1] - angles[0]) / 3.0 - theta_deg) < 2e-3, (theta_deg, angles)


@pytest.mark.parametrize("theta_deg", ANGLES)
def test_angle_from_height_inverts_the_closed_forms_exactly(theta_deg):
    """With the exact area / volume and half-height of a cap, both functions
    return theta to rounding (eq. angleh is an identity for a true cap)."""
    th = math.radians(theta_deg)
    for Rc in (3.0, 40.0, 250.0):
        ell = 0.5 * Rc * (1.0 - math.cos(th))
        assert abs(o.angle_from_height_3d(ell, cap_volume(Rc, th)) - th) < 1e-10
        assert abs(o.angle_from_height_2d(ell, segment_area(Rc, th)) - th) < 1e-10


def test_area_and_volume_of_the_oracle_on_hemisphere_and_half_disk():
    """Special cases: the 90 degree cap is a half disk / hemisphere."""
    q = segment_polygon(10.0, math.pi / 2, 8192, 2048)
    assert abs(o.volume_2d(q) - 0.5 * math.pi * 100.0) < 1e-5 * 50.0 * math.pi
    q, tris = cap_polyhedron(10.0, math.pi / 2, 96, 384)
    assert abs(o.volume_3d(q, tris) - 2.0 * math.pi * 1000.0 / 3.0) < 2e-4 * 2000.0 * math.pi / 3.0
    # surface: curved part 2 pi R^2 plus base pi R^2
    assert abs(o.area_3d(q, tris) - 3.0 * math.pi * 100.0) < 2e-4 * 300.0 * math.pi
