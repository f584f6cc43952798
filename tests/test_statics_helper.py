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
