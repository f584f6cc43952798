"""GPU contact-radius protocols (Sec. Dynamics) against the oracle's
formulas evaluated on the same node positions read back from the device
(double precision on both sides; only the order of the sums differs)."""
import numpy as np
import pytest

import oracle as o
import workloads as wl
from helpers import gpu_run

pytestmark = pytest.mark.gpu


def test_contact_radius_2d():
    W = wl.droplet_2d_small()
    print("[contact] 2d", flush=True)
    g = gpu_run(W.params, W.nodes, 200)
    s, q = g["solver"], g["q"]
    for zc, tol in [(o.h_star(W.params.xi), 0.02 * 20.0), (3.5, 0.1 * 20.0), (1e6, 1e-9)]:
        ri, rii, n = s.contact_radius(0, zc, tol)
        want_i = o.contact_radius_2d(q, zc)
        if np.isnan(want_i):
            assert np.isnan(ri) and n < 2
        else:
            assert abs(ri - want_i) < 1e-12 * want_i
        assert abs(rii - o.contact_radius_flat_2d(q, tol)) <= 1e-12 * max(rii, 1.0)


def test_contact_radius_3d_benchmark_cap():
    W = wl.droplet_3d(small=False)
    print("[contact] 3d 256x256x128", flush=True)
    g = gpu_run(W.params, W.nodes, 4, tris=W.tris)
    s, q = g["solver"], g["q"]
    for zc, tol in [(o.h_star(W.params.xi), 0.05 * 40.0), (10.0, 0.1 * 40.0)]:
        ri, rii, n = s.contact_radius(0, zc, tol)
        assert n > 100
        assert abs(ri - o.contact_radius_3d(q, W.tris, zc)) < 1e-12 * ri
        assert abs(rii - o.contact_radius_flat_3d(q, W.tris, tol)) < 1e-12 * rii
