"""Pins of the oracle's interface forces.

Surface tension (Sec. "Modelling surface tension forces"): the nodal force
is minus the derivative of the strain energy w = sigma e^a, with a the
first strain invariant of the projected deformation gradient D.  The oracle
evaluates it in closed form as -sigma d|Gamma|/dq; here it is pinned by
finite differences of the energy computed literally from the paper's
invariant a = 1/2 log{ 1/2 [tr(D D^T)]^2 - 1/2 tr[(D D^T)^2] }, by
translation invariance, by Euler's relation for a homogeneous function and
by the closed form for a regular polygon.

Wetting (Sec. "Modelling wetting properties"): Pi(h) of eq. (disjoin-p),
the strength A of eq. (A_choice) checked through the wedge integral of
Appendix A, the minimum at h* = xi (n/m)^(1/(n-m)) (Sec. Dynamics), and
the nodal-area weighting chi_j / 3 (chi_j / 2 in 2D)."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as o
import workloads as wl


def _wobbly_polygon(n, seed):
    rng = np.random.default_rng(seed)
    a = np.sort(rng.uniform(0, 2 * np.pi, n))
    r = 5 + rng.uniform(-1, 1, n)
    return np.stack([20 + r * np.cos(a), 12 + r * np.sin(a)], axis=1)


def _perimeter(q):
    return float(np.sum(np.linalg.norm(np.roll(q, -1, axis=0) - q, axis=1)))


def test_membrane_2d_translation_and_homogeneity():
    sigma = 0.013
    for seed in range(4):
        q = _wobbly_polygon(17, seed)
        phi, _ = o.forces_2d(q, sigma, 0.0, 1.0, wetting=False)
        assert np.allclose(phi.sum(axis=0), 0, atol=1e-15)
        # perimeter is homogeneous of degree 1: sum q.grad = |Gamma|
        assert abs(np.sum(q * phi) + sigma * _perimeter(q)) < 1e-12


def test_membrane_2d_finite_difference():
    sigma = 0.02
    q = _wobbly_polygon(9, 7)
    phi, _ = o.forces_2d(q, sigma, 0.0, 1.0, wetting=False)
    h = 1e-6
    for j in range(len(q)):
        for a in range(2):
            qp, qm = q.copy(), q.copy()
            qp[j, a] += h
            qm[j, a] -= h
            g = sigma * (_perimeter(qp) - _perimeter(qm)) / (2 * h)
            assert abs(phi[j, a] + g) < 1e-8


@pytest.mark.parametrize("N", [3, 8, 64, 128])
def test_membrane_regular_polygon(N):
    sigma, R = 0.01, 7.0
    q = wl.circle_polygon(R, N, (10.0, 10.0))
    phi, nrm = o.forces_2d(q, sigma, 0.0, 1.0, wetting=False)
    radial = (q - np.array([10.0, 10.0])) / R
    assert np.allclose(np.linalg.norm(phi, axis=1), 2 * sigma * math.sin(math.pi / N), atol=1e-14)
    assert np.allclose(phi / np.linalg.norm(phi, axis=1)[:, None], -radial, atol=1e-12)
    assert np.allclose(nrm, radial, atol=1e-12)        # outward node normal


def _paper_energy(q_ref, q_cur, tris, sigma):
    """sum over triangles of reference area * sigma * e^a, with a computed
    from D D^T through the trace formula of the strain invariants."""
    W = 0.0
    for t in tris:
        E0 = np.stack([q_ref[t[1]] - q_ref[t[0]], q_ref[t[2]] - q_ref[t[0]]], axis=1)  # 3x2
        E1 = np.stack([q_cur[t[1]] - q_cur[t[0]], q_cur[t[2]] - q_cur[t[0]]], axis=1)
        D = E1 @ np.linalg.pinv(E0)          # maps reference tangents to current ones
        M = D @ D.T
        a = 0.5 * math.log(0.5 * np.trace(M) ** 2 - 0.5 * np.trace(M @ M))
        A0 = 0.5 * np.linalg.norm(np.cross(E0[:, 0], E0[:, 1]))
        W += A0 * sigma * math.exp(a)
    return W


def test_membrane_3d_is_minus_gradient_of_paper_energy():
    """R1: with w = sigma e^a the discrete energy's gradient is the oracle's
    surface-tension force, whatever the reference state."""
    V, T = wl.sphere_mesh(3.0, 2, (5.0, 5.0, 5.0))
    rng = np.random.default_rng(8)
    q_ref = V + 0.2 * rng.standard_normal(V.shape)
    q = V + 0.3 * rng.standard_normal(V.shape)
    sigma = 0.02
    phi, _ = o.forces_3d(q, T, sigma, 0.0, 1.0, wetting=False)
    h = 1e-6
    for j in rng.choice(len(q), 6, replace=False):
        for a in range(3):
            qp, qm = q.copy(), q.copy()
            qp[j, a] += h
            qm[j, a] -= h
            g = (_paper_energy(q_ref, qp, T, sigma) - _paper_energy(q_ref, qm, T, sigma)) / (2 * h)
            assert abs(phi[j, a] + g) < 1e-7


def test_membrane_2d_is_minus_gradient_of_line_tension():
    """2D analogue of the same energy: the invariant of a 1D stretch is the
    length ratio, so the energy is sigma times the perimeter."""
    q = _wobbly_polygon(6, 9)
    q_ref = _wobbly_polygon(6, 10)
    sigma = 0.03

    def energy(qc):
        W = 0.0
        for j in range(len(qc)):
            e0 = q_ref[(j + 1) % len(qc)] - q_ref[j]
            e1 = qc[(j + 1) % len(qc)] - qc[j]
            stretch = np.linalg.norm(e1) / np.linalg.norm(e0)
            W += np.linalg.norm(e0) * sigma * stretch
        return W

    phi, _ = o.forces_2d(q, sigma, 0.0, 1.0, wetting=False)
    h = 1e-6
    for j in range(len(q)):
        for a in range(2):
            qp, qm = q.copy(), q.copy()
            qp[j, a] += h
            qm[j, a] -= h
            assert abs(phi[j, a] + (energy(qp) - energy(qm)) / (2 * h)) < 1e-8


def test_membrane_3d_translation_and_homogeneity():
    V, T = wl.sphere_mesh(4.0, 4, (0.0, 0.0, 0.0))
    rng = np.random.default_rng(2)
    q = V + 0.1 * rng.standard_normal(V.shape)
    sigma = 0.01
    phi, _ = o.forces_3d(q, T, sigma, 0.0, 1.0, wetting=False)
    assert np.allclose(phi.sum(axis=0), 0, atol=1e-14)
    area = o.area_3d(q, T)
    assert abs(np.sum(q * phi) + 2 * sigma * area) < 1e-11


def test_sphere_pressure_balance():
    """On a fine sphere the summed surface-tension force per unit area is
    2 sigma / R, inward (Laplace, eq. laplace-pi with Pi = 0)."""
    R, sigma = 10.0, 0.01
    V, T = wl.sphere_mesh(R, 12, (0.0, 0.0, 0.0))
    phi, nrm = o.forces_3d(V, T, sigma, 0.0, 1.0, wetting=False)
    radial = V / R
    assert np.all(np.einsum('ij,ij->i', nrm, radial) > 0.999)
    p = -np.sum(np.einsum('ij,ij->i', phi, radial)) / o.area_3d(V, T)
    assert abs(p / (2 * sigma / R) - 1) < 5e-3


def test_pi_zero_minimum_and_wedge_integral():
    sigma, xi = 0.01, 2.0
    for th_deg in (20, 60, 90, 135, 160):
        th = math.radians(th_deg)
        A = o.wetting_strength(sigma, th, xi)
        assert abs(o.Pi(xi, A, xi)[0]) < 1e-18
        hs = o.h_star(xi)
        assert abs(hs - 2 ** (1 / 3) * xi) < 1e-14
        d = (o.Pi(hs + 1e-5, A, xi)[0] - o.Pi(hs - 1e-5, A, xi)[0]) / 2e-5
        assert abs(d) < 1e-9 * A
        assert o.Pi(hs, A, xi)[0] < o.Pi(hs * 1.01, A, xi)[0]
        assert o.Pi(hs, A, xi)[0] < o.Pi(hs * 0.99, A, xi)[0]
        # Appendix A: sigma * int_0^{pi - theta} sin(psi) dpsi = -int_xi^inf Pi dh
        val, _ = integrate.quad(lambda h: o.Pi(h, A, xi)[0], xi, np.inf, limit=200)
        assert abs(-val - sigma * (1 + math.cos(th))) < 1e-10
        # repulsive below xi, attractive above
        assert o.Pi(0.9 * xi, A, xi)[0] > 0 and o.Pi(1.5 * xi, A, xi)[0] < 0


def test_wetting_strength_6_3_closed_form():
    # (n, m) = (6, 3): A = 10 sigma (1 + cos theta) / (3 xi); 60 degrees,
    # sigma = 0.01, xi = 2 gives A = 0.025
    assert abs(o.wetting_strength(0.01, math.radians(60), 2.0) - 0.025) < 1e-16


def test_wetting_force_2d_nodal_length_weighting():
    """phi_Pi_j = -(chi_j / 2) Pi(h_j) n_j with chi_j the two adjacent edge
    lengths: the nodal lengths chi_j / 2 add up to the perimeter."""
    q = wl.cap_polygon(8.0, 70.0, 2.0, 40, 20.0)
    q[:, 1] += 0.3
    sigma, xi = 0.01, 2.0
    A = o.wetting_strength(sigma, math.radians(50), xi)
    phi_on, nrm = o.forces_2d(q, sigma, A, xi, wetting=True)
    phi_off, _ = o.forces_2d(q, sigma, A, xi, wetting=False)
    w = phi_on - phi_off
    P = o.Pi(q[:, 1], A, xi)
    share = -np.einsum('ij,ij->i', w, nrm) / P
    assert np.allclose(w, -(share * P)[:, None] * nrm, atol=1e-15)
    assert abs(share.sum() - _perimeter(q)) < 1e-12
    el = np.linalg.norm(np.roll(q, -1, axis=0) - q, axis=1)
    assert np.allclose(share, 0.5 * (el + np.roll(el, 1)), atol=1e-14)


def test_wetting_force_3d_nodal_area_weighting():
    V, T = wl.cap_mesh(5.0, 100.0, 2.2, 4, (8.0, 8.0))
    sigma, xi = 0.01, 2.0
    A = o.wetting_strength(sigma, math.radians(60), xi)
    phi_on, nrm = o.forces_3d(V, T, sigma, A, xi, wetting=True)
    phi_off, _ = o.forces_3d(V, T, sigma, A, xi, wetting=False)
    w = phi_on - phi_off
    P = o.Pi(V[:, 2], A, xi)
    share = -np.einsum('ij,ij->i', w, nrm) / P
    assert np.allclose(w, -(share * P)[:, None] * nrm, atol=1e-15)
    assert abs(share.sum() - o.area_3d(V, T)) < 1e-10
    assert np.allclose(np.linalg.norm(nrm, axis=1), 1.0)
