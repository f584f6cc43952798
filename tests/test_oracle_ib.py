"""Pins of the oracle's immersed-boundary coupling: the Peskin 4-point
kernel (Sec. IB-LB, Psi(x)), eq. (force_spread) and eq. (vel_interpolation).

The kernel is pinned by the moment conditions it was built to satisfy
(partition of unity, split even/odd sums, zero first moment, constant sum
of squares 3/8), not by re-typing its formula; spreading and interpolation
by force conservation, adjointness and exact interpolation of linear
fields."""
import numpy as np
import pytest

import oracle as o


def test_psi_support_symmetry_continuity():
    x = np.linspace(-3, 3, 1201)
    p = o.psi(x)
    assert np.all(p[np.abs(x) >= 2] == 0)
    assert np.all(p[np.abs(x) < 2] > 0)
    assert np.array_equal(p, o.psi(-x))
    for x0 in (1.0, 2.0):
        lo, hi = o.psi([x0 - 1e-9, x0 + 1e-9])
        assert abs(lo - hi) < 1e-8
    assert abs(o.psi(0.0)[0] - 0.5) < 1e-15


@pytest.mark.parametrize("r", list(np.linspace(0, 1, 17)[:-1]) + [0.123456, 0.987654])
def test_psi_moment_conditions(r):
    d = r - np.arange(-2, 3)          # distances to the five nearest integers
    p = o.psi(d)
    assert abs(p.sum() - 1) < 1e-15                     # partition of unity
    even = p[np.arange(-2, 3) % 2 == 0].sum()
    assert abs(even - 0.5) < 1e-15                      # even/odd split
    assert abs((d * p).sum()) < 1e-15                   # zero first moment
    assert abs((p * p).sum() - 3 / 8) < 1e-15           # sum of squares


def _nodes(n, lo, hi, dim, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, dim))


@pytest.mark.parametrize("dim", [2, 3])
def test_spread_conserves_force_and_drops_wall_taps(dim):
    nx, ny, nz = (20, 16, 1) if dim == 2 else (10, 9, 8)
    n = np.array([nx, ny, nz])
    bc = (0, 1, 0) if dim == 2 else (0, 0, 1)
    rng = np.random.default_rng(3)
    q = rng.uniform(0, 1, size=(30, dim)) * n[:dim]
    q[:5, dim - 1] = rng.uniform(0.05, 1.5, 5)        # close to the low wall
    q[5:8, dim - 1] = n[dim - 1] - rng.uniform(0.05, 1.5, 3)
    q[8:11, 0] = rng.uniform(0, 1, 3)                  # wrap across x = 0
    phi = rng.standard_normal((30, dim))
    F, dropped = o.spread(dim, nx, ny, nz, bc, q, phi)
    tot = F[:dim].reshape(dim, -1).sum(axis=1) + dropped[:dim]
    assert np.allclose(tot, phi.sum(axis=0), atol=1e-13)
    assert np.any(np.abs(dropped) > 1e-3)
    # a node far from the walls loses nothing
    qc = (n[:dim] / 2.0)[None, :]
    F1, d1 = o.spread(dim, nx, ny, nz, bc, qc, np.ones((1, dim)))
    assert np.allclose(d1, 0) and np.allclose(F1[:dim].reshape(dim, -1).sum(axis=1), 1.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_spread_interp_adjoint(dim):
    """sum_x F(x).U(x) = sum_j phi_j . qdot_j when F is spread from phi and
    qdot interpolated from U with the same kernel (dx = 1)."""
    nx, ny, nz = (18, 14, 1) if dim == 2 else (9, 8, 10)
    n = np.array([nx, ny, nz])
    bc = (0, 1, 0) if dim == 2 else (0, 0, 1)
    rng = np.random.default_rng(4)
    q = rng.uniform(0, 1, size=(25, dim)) * n[:dim]
    phi = rng.standard_normal((25, dim))
    U = np.zeros((3, nz, ny, nx))
    U[:dim] = rng.standard_normal((dim, nz, ny, nx))
    F, _ = o.spread(dim, nx, ny, nz, bc, q, phi)
    qdot = o.interp(dim, nx, ny, nz, bc, U, q)
    lhs = float(np.sum(F[:dim] * U[:dim]))
    rhs = float(np.sum(phi * qdot))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("dim", [2, 3])
def test_interp_linear_field_exact(dim):
    nx, ny, nz = (24, 20, 1) if dim == 2 else (14, 12, 13)
    n = np.array([nx, ny, nz])
    bc = (0, 1, 0) if dim == 2 else (0, 0, 1)
    rng = np.random.default_rng(5)
    a = rng.standard_normal(3)
    B = rng.standard_normal((3, 3))
    grids = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                        indexing='ij')
    X = np.stack([grids[2], grids[1], grids[0]])
    U = np.zeros((3, nz, ny, nx))
    for c in range(dim):
        U[c] = a[c] + sum(B[c, k] * X[k] for k in range(dim))
    # nodes at least 2.5 away from every edge: no wall tap, no wrap
    q = 2.5 + rng.uniform(0, 1, size=(20, dim)) * (n[:dim] - 5.0)
    got = o.interp(dim, nx, ny, nz, bc, U, q)
    want = a[None, :dim] + q @ B[:dim, :dim].T
    assert np.allclose(got, want, atol=1e-12)


def test_interp_wall_taps_read_zero_and_periodic_taps_wrap():
    nx, ny = 12, 10
    U = np.zeros((3, 1, ny, nx))
    U[0] = 1.0
    # at the wall the fluid velocity is zero: a node at h = 0.5 sees only
    # the taps with centres at y = 0.5, 1.5 (weights psi(0) + psi(1) = 3/4
    # of the one-dimensional unit mass); the rest lie in the solid
    q = np.array([[6.5, 0.5]])
    got = o.interp(2, nx, ny, 1, (0, 1, 0), U, q)
    assert abs(got[0, 0] - float(o.psi(0.0)[0] + o.psi(1.0)[0])) < 1e-15
    # periodic in x: a uniform field interpolates to 1 even across x = 0
    q = np.array([[0.1, 5.0]])
    got = o.interp(2, nx, ny, 1, (0, 1, 0), U, q)
    assert abs(got[0, 0] - 1.0) < 1e-15
