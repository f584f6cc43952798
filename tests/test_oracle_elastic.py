"""Pins of the oracle's elastic interface (a strain energy w(a, b) other
than eq. energy_drop in eq. force_bb, as the paper's outlook proposes):
w(a, b) = sigma e^a + mu_s (b + 1 - e^a) with the invariants of eq.
strain_inv measured from a stress-free reference mesh.

The forces are pinned against central differences of the energy computed
straight from eq. strain_inv (D from a pseudo-inverse of the reference
edges, a and b from tr(D D^T) and tr((D D^T)^2)), and by the closed forms
of rigid motions and uniform dilations (no shear energy) and of a uniaxial
stretch (energy mu_s A0 (l - 1)^2 / 2)."""
import math

import numpy as np
import pytest

import oracle as o
import workloads as wl


def energy(q, qref, tris, sigma, mu_s):
    """sum over triangles of A0 w(a, b), eq. strain_inv taken literally."""
    W = 0.0
    for t in tris:
        R = qref[t]
        P = q[t]
        Er = np.stack([R[1] - R[0], R[2] - R[0]], axis=1)   # 3 x 2
        Ec = np.stack([P[1] - P[0], P[2] - P[0]], axis=1)
        D = Ec @ np.linalg.pinv(Er)                         # 3 x 3, maps the reference plane
        G = D @ D.T
        a = 0.5 * math.log(0.5 * np.trace(G) ** 2 - 0.5 * np.trace(G @ G))
        b = 0.5 * np.trace(G) - 1.0
        A0 = 0.5 * np.linalg.norm(np.cross(Er[:, 0], Er[:, 1]))
        W += A0 * (sigma * math.exp(a) + mu_s * (b + 1.0 - math.exp(a)))
    return W


def perturbed_sphere(seed=1):
    V, T = wl.sphere_mesh(3.0, 2, (5.0, 5.0, 5.0))
    rng = np.random.default_rng(seed)
    return V, V + 0.15 * rng.standard_normal(V.shape), T


@pytest.mark.parametrize("sigma,mu_s", [(0.0, 0.02), (0.01, 0.03)])
def test_forces_are_minus_the_energy_gradient(sigma, mu_s):
    Vr, V, T = perturbed_sphere()
    phi, _ = o.forces_3d(V, T, sigma, 0.0, 1.0, wetting=False, mu_s=mu_s, qref=Vr)
    h = 1e-6
    for j in (0, 7, 20, 33):
        for k in range(3):
            qp, qm = V.copy(), V.copy()
            qp[j, k] += h
            qm[j, k] -= h
            g = (energy(qp, Vr, T, sigma, mu_s) - energy(qm, Vr, T, sigma, mu_s)) / (2 * h)
            assert abs(phi[j, k] + g) < 1e-7 * max(1.0, abs(g)), (j, k, phi[j, k], -g)


def test_no_shear_force_after_rigid_motion_or_uniform_dilation():
    Vr, _, T = perturbed_sphere()
    c, s = math.cos(0.7), math.sin(0.7)
    Rz = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])
    for V in (Vr @ (Rz @ Rx).T + np.array([3.0, -1.0, 2.0]), 1.3 * Vr - 0.5):
        liquid, _ = o.forces_3d(V, T, 0.01, 0.0, 1.0, wetting=False)
        elastic, _ = o.forces_3d(V, T, 0.01, 0.0, 1.0, wetting=False, mu_s=0.05, qref=Vr)
        assert np.max(np.abs(elastic - liquid)) < 1e-12


def test_zero_modulus_is_the_liquid_droplet():
    Vr, V, T = perturbed_sphere()
    a, _ = o.forces_3d(V, T, 0.01, 0.02, 1.0, wetting=True)
    b, _ = o.forces_3d(V, T, 0.01, 0.02, 1.0, wetting=True, mu_s=0.0, qref=Vr)
    assert np.array_equal(a, b)


def test_uniaxial_stretch_energy():
    """A flat triangulated square stretched by l along x: each triangle has
    principal stretches (l, 1), so the shear energy is mu_s A0 (l - 1)^2 / 2
    in total; the force on the mesh sums to zero."""
    n = 5
    xs, ys = np.meshgrid(np.arange(n + 1, dtype=float), np.arange(n + 1, dtype=float))
    Vr = np.stack([xs.ravel(), ys.ravel(), np.zeros(xs.size)], axis=1)
    T = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = i * (n + 1) + j, i * (n + 1) + j + 1, (i + 1) * (n + 1) + j, (i + 1) * (n + 1) + j + 1
            T += [[a, b, d], [a, d, c]]
    T = np.array(T, dtype=np.int32)
    lam, mu_s = 1.25, 0.04
    V = Vr * np.array([lam, 1.0, 1.0])
    assert abs(energy(V, Vr, T, 0.0, mu_s) - mu_s * n * n * (lam - 1) ** 2 / 2) < 1e-12
    phi, _ = o.forces_3d(V, T, 0.0, 0.0, 1.0, wetting=False, mu_s=mu_s, qref=Vr)
    assert np.max(np.abs(phi.sum(axis=0))) < 1e-12
    # the stretched sheet pulls back along x at its right edge
    right = np.abs(V[:, 0] - lam * n) < 1e-12
    assert np.all(phi[right, 0] < 0)
