"""GPU parity of the elastic interface (strain energy w(a, b) = sigma e^a +
mu_s (b + 1 - e^a) in eq. force_bb, reference = the mesh at the time the
modulus is set) against the FP64 oracle, through the C ABI; tolerances of
the one-fluid 3D parity tests."""
import numpy as np
import pytest

import oracle as o
import workloads as wl
from helpers import compare_fields, gpu_run, gpu_solver

pytestmark = pytest.mark.gpu


def test_elastic_cap_across_periodic_edge():
    p = wl.Params(dim=3, nx=30, ny=28, nz=16, bc=(wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_WALL),
                  tau=0.7, sigma=0.006, theta_eq_deg=50.0, xi=2.0, shear=0.03)
    V, T = wl.cap_mesh(8.0, 90.0, 2.0, 5, (1.5, 27.3))
    print("[elastic] cap 30x28x16, 8 steps", flush=True)
    g = gpu_run(p, V, 8, tris=T, graph_steps=2)
    r = o.run(p, V, 8, tris=T)
    drho, du, dq = compare_fields(g, r, 3, "elastic-cap")
    assert drho <= 1e-5 and du <= 1e-5 and dq <= 1e-6
    assert np.max(np.abs(g["phi"] - r["phi"])) <= 1e-5 * np.max(np.abs(r["phi"]))


def test_elastic_benchmark_cap_two_steps():
    """256x256x128 cap of 20252 vertices, shear modulus 0.01, two steps."""
    W = wl.droplet_3d(small=False)
    p = wl.Params(**{**W.params.to_dict(), "shear": 0.01})
    print("[elastic] 256x256x128 2 steps", flush=True)
    g = gpu_run(p, W.nodes, 2, tris=W.tris)
    r = o.run(p, W.nodes, 2, tris=W.tris)
    drho, du, dq = compare_fields(g, r, 3, "elastic-full")
    assert drho <= 1e-5 and du <= 1e-5 and dq <= 1e-6


def test_shear_modulus_slows_spreading():
    """A sphere of the statics set-up flattens less with an elastic
    interface: after 3000 steps it stands taller with shear modulus 0.05
    than without."""
    W = wl.droplet_3d_statics(60.0)
    heights = []
    for mu in (0.0, 0.05):
        s = gpu_solver([wl.Params(**{**W.params.to_dict(), "shear": mu})], [W.nodes], [W.tris])
        s.step(3000)
        heights.append(s.diagnostics(0)["height"])
        s.close()
    print(f"[elastic] height liquid {heights[0]:.3f}, elastic {heights[1]:.3f} (initial 40)", flush=True)
    assert heights[0] < 39.0 and heights[1] > heights[0] + 0.5


def test_shear_modulus_errors():
    W = wl.droplet_2d_small()
    s = gpu_solver([W.params], [W.nodes])
    with pytest.raises(Exception, match="IBLB_EINVAL"):
        s.set_membrane_shear(0, 0.1)
    W3 = wl.droplet_3d(small=True)
    s3 = gpu_solver([W3.params], [W3.nodes], [W3.tris])
    with pytest.raises(Exception, match="IBLB_EINVAL"):
        s3.set_membrane_shear(0, -1.0)
    s3.set_membrane_shear(0, 0.0)
