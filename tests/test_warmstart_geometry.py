"""Host-side geometry of the learned warm start: radial profiles, the
equal-area cap reference, outline reconstruction, coarse velocity grid and
the initial populations (checked against the FP64 oracle's equilibrium)."""
import math

import numpy as np

import oracle as o
import workloads as wl
from paper_2503_20605_amd import warmstart as ws


def test_radial_profile_of_circle_is_constant():
    q = wl.circle_polygon(10.0, 2000, (30.0, 40.0))
    r = ws.radial_profile(q, np.array([30.0, 40.0]))
    assert np.allclose(r, 10.0, atol=2e-4)


def test_cap_reference_and_reconstruction_round_trip():
    for th in (25.0, 60.0, 90.0, 140.0):
        theta = math.radians(th)
        area = 2000.0
        cap, rc = ws.cap_outline(theta, area, 2.0, 100.0)
        assert abs(ws.polygon_area(cap) - area) < 1e-3 * area
        ref, rcap, rc2 = ws.reference(theta, area, 2.0, 200)
        assert abs(rc - rc2) < 1e-12
        q = ws.outline_from_profile(ref, rcap, 300, 1.0)
        # 256 rays resolve the sharp contact corners of flat caps only to ~1 % in area
        assert abs(ws.polygon_area(q) - area) < 1e-2 * area
        assert np.all(q[:, 1] >= 1.0)
        # CCW and star-shaped about the reference
        assert ws.polygon_area(q) > 0
        r2 = ws.radial_profile(q, ref)
        assert np.max(np.abs(r2 - rcap)) < 0.05 * rc


def test_shape_error_zero_for_same_and_positive_for_different():
    theta = math.radians(70.0)
    ref, rcap, rc = ws.reference(theta, 1500.0, 2.0, 160)
    q = ws.outline_from_profile(ref, rcap, 200, 1.0)
    assert ws.shape_error(q, q, ref) == 0.0
    q2 = ws.outline_from_profile(ref, rcap * 1.01, 200, 1.0)
    assert 0.005 < ws.shape_error(q2, q, ref) < 0.02


def test_velocity_grid_round_trip():
    rng = np.random.default_rng(0)
    Uc = rng.standard_normal((2,) + ws.GRID)
    U = ws.fine_velocity(Uc, 64, 160)
    assert U.shape == (2, 64, 160)
    assert np.allclose(ws.coarse_velocity(U), Uc)


def test_inside_mask_of_circle():
    q = wl.circle_polygon(8.0, 400, (16.0, 12.0))
    m = ws.inside_mask(q, 24, 32)
    yy, xx = np.mgrid[0:24, 0:32] + 0.5
    want = (xx - 16) ** 2 + (yy - 12) ** 2 < 8.0 ** 2
    assert np.sum(m != want) <= 4          # cells whose centre sits on the boundary
