"""The shape comparison of the statics test, checked on a mesh built from
the App. B solution itself (its error must vanish up to the mesh's
discretisation) and on the initial sphere (it must not)."""
import math
import sys
import os

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import statics  # noqa: E402
import workloads as wl  # noqa: E402
from oracle import shape as sh  # noqa: E402


def test_error_vanishes_on_the_theoretical_shape():
    theta, R0, xi = 3 * math.pi / 4, 20.0, 2.0
    s = sh.solve(theta, xi / R0)
    zc = sh.centroid_height(s["u"], s["g"])
    U, T = wl.icosphere(30)
    phi = np.arccos(np.clip(U[:, 2], -1.0, 1.0))
    G = R0 * sh.radial_profile_about(s["u"], s["g"], zc, phi)
    q = np.array([40.0, 40.0, 30.0]) + G[:, None] * U
    r = statics.l2_error(q, T, theta, xi)
    assert r["E_L2"] < 2e-3, r
    assert abs(r["R0"] - R0) < 0.05


def test_error_of_the_initial_sphere_is_large():
    W = wl.droplet_3d_statics(90.0)
    r = statics.l2_error(W.nodes, W.tris, math.pi / 2, W.params.xi)
    assert r["E_L2"] > 0.1


def test_error_vanishes_on_the_theoretical_outline_2d():
    theta, R0, xi = 3 * math.pi / 4, 20.0, 2.0
    s = sh.solve_2d(theta, xi / R0)
    z0 = sh.centroid_height_2d(s["phi"], s["g"])
    a = np.linspace(0.0, 2.0 * math.pi, 2000, endpoint=False)
    phi = np.arccos(np.cos(a))              # polar angle from +y folded onto [0, pi]
    G = R0 * sh.radial_profile_about_2d(s["phi"], s["g"], z0, phi)
    # counter-clockwise from the top
    q = np.array([64.0, 30.0]) + G[:, None] * np.stack([-np.sin(a), np.cos(a)], axis=1)
    r = statics.l2_error_2d(q, theta, xi)
    assert r["E_L2"] < 2e-3, r
    assert abs(r["R0"] - R0) < 0.05


def test_error_of_the_initial_circle_is_large_2d():
    W = wl.droplet_2d_statics(45.0, 0.1)
    r = statics.l2_error_2d(W.nodes, math.radians(45.0), W.params.xi)
    assert r["E_L2"] > 0.1, r


def test_outline_continuation_reaches_the_direct_solution_2d():
    # where the truncated-cap guess converges on its own, the continued
    # solution is the same outline
    for theta, eps in ((math.pi / 4, 0.2), (3 * math.pi / 4, 0.3)):
        a = sh.solve_2d(theta, eps)
        b = statics.theory_2d(theta, eps)
        assert np.max(np.abs(a["g"] - b["g"])) < 1e-9
