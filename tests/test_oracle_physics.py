"""Whole-method pins of the oracle: the coupled IB-LB loop on a free droplet
(Laplace law, eq. laplace-pi with Pi = 0 and p = c_s^2 rho) and conservation
laws that the discrete method keeps exactly."""
import math

import numpy as np
import pytest

import oracle as o
import workloads as wl


def _free_droplet_2d(steps, R=14.0, L=64, N=96, sigma=0.01):
    p = wl.Params(dim=2, nx=L, ny=L, bc=(0, 0, 0), tau=1.0, sigma=sigma, wetting=False)
    q = wl.circle_polygon(R, N, (L / 2, L / 2))
    return p, q, o.run(p, q, steps)


def test_laplace_pressure_2d_free_droplet():
    p, q0, r = _free_droplet_2d(3000)
    L = p.nx
    y, x = np.mgrid[0:L, 0:L] + 0.5
    d = np.hypot(x - L / 2, y - L / 2)
    Reff = math.sqrt(o.volume_2d(r["q"]) / math.pi)
    rho = r["rho"][0]
    dp = (rho[d < Reff - 3].mean() - rho[d > Reff + 3].mean()) / 3.0
    want = p.sigma / Reff
    assert abs(dp / want - 1) < 0.05, (dp, want)
    # the droplet stays circular and centred, the fluid nearly at rest
    rr = np.linalg.norm(r["q"] - L / 2, axis=1)
    assert rr.std() / rr.mean() < 2e-3
    assert np.abs(r["U"]).max() < 1e-4


def test_momentum_and_mass_conserved_free_droplet():
    """Sum of surface-tension forces is zero and the box is periodic, so
    the total post-collision momentum stays zero and the mass stays at the
    cell count."""
    p, q0, r = _free_droplet_2d(300, R=10.0, L=40, N=64)
    c, _ = o.lattice(2)
    mom = np.einsum('ia,izyx->a', c, r["f"])
    assert np.max(np.abs(mom)) < 1e-12
    assert abs(r["f"].sum() - 40 * 40) < 1e-10
    assert np.allclose(r["phi"].sum(axis=0), 0, atol=1e-15)
    assert np.allclose(r["F"][:2].reshape(2, -1).sum(axis=1), 0, atol=1e-14)


def test_droplet_on_wall_conserves_mass_and_force_bookkeeping():
    W = wl.droplet_2d_small()
    r = o.run(W.params, W.nodes, 200)
    assert r["status"] == 0
    p = W.params
    assert abs(r["f"].sum() - p.nx * p.ny) < 1e-10
    tot = r["F"][:2].reshape(2, -1).sum(axis=1) + r["dropped"][:2]
    assert np.allclose(tot, r["phi"].sum(axis=0), atol=1e-14)


def test_node_reaching_wall_reports_unstable():
    W = wl.droplet_2d_small()
    q = W.nodes.copy()
    q[5, 1] = 0.0
    r = o.run(W.params, q, 3)
    assert r["status"] == -4


def test_laplace_pressure_3d_free_droplet():
    """3D free droplet: rho_in - rho_out = 3 * 2 sigma / R."""
    L, R, sigma = 32, 8.0, 0.01
    p = wl.Params(dim=3, nx=L, ny=L, nz=L, bc=(0, 0, 0), tau=1.0, sigma=sigma, wetting=False)
    V, T = wl.sphere_mesh(R, 8, (L / 2, L / 2, L / 2))
    r = o.run(p, V, 600, tris=T)
    z, y, x = np.mgrid[0:L, 0:L, 0:L] + 0.5
    d = np.sqrt((x - L / 2) ** 2 + (y - L / 2) ** 2 + (z - L / 2) ** 2)
    Reff = (3 * o.volume_3d(r["q"], T) / (4 * math.pi)) ** (1 / 3)
    rho = r["rho"]
    dp = (rho[d < Reff - 2.5].mean() - rho[d > Reff + 2.5].mean()) / 3.0
    want = 2 * sigma / Reff
    assert abs(dp / want - 1) < 0.08, (dp, want)
