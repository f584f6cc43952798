"""Pins of the oracle's lattice, equilibrium, Guo source and LB update
against what the paper's equations and the lattice symmetry fix.

Velocity set: Table I (D3Q19) and its 2D analogue D2Q9; c_s^2 = 1/3.
Equilibrium and Guo source: Sec. "Immersed-boundary lattice Boltzmann
(IB-LB) method", the equilibrium expansion and S_i(U, F); moments from
eqs. (hydro_var1)-(hydro_var2)."""
import itertools
import math

import numpy as np
import pytest

import oracle as o

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("dim", [2, 3])
def test_velocity_set_isotropy(dim):
    c, w = o.lattice(dim)
    Q = 9 if dim == 2 else 19
    assert c.shape == (Q, 3)
    # Table I weights by speed shell
    sp = (c ** 2).sum(axis=1)
    if dim == 3:
        assert np.allclose(w[sp == 0], 1 / 3) and np.allclose(w[sp == 1], 1 / 18)
        assert np.allclose(w[sp == 2], 1 / 36)
        assert (sp == 1).sum() == 6 and (sp == 2).sum() == 12
    else:
        assert np.allclose(w[sp == 0], 4 / 9) and np.allclose(w[sp == 1], 1 / 9)
        assert np.allclose(w[sp == 2], 1 / 36)
    assert len({tuple(v) for v in c}) == Q
    ax = range(dim)
    assert abs(w.sum() - 1.0) < 1e-15
    for a in ax:
        assert abs((w * c[:, a]).sum()) < 1e-15
    for a, b in itertools.product(ax, ax):
        assert abs((w * c[:, a] * c[:, b]).sum() - CS2 * (a == b)) < 1e-15
    for a, b, g in itertools.product(ax, ax, ax):
        assert abs((w * c[:, a] * c[:, b] * c[:, g]).sum()) < 1e-15
    for a, b, g, d in itertools.product(ax, ax, ax, ax):
        want = CS2 ** 2 * ((a == b) * (g == d) + (a == g) * (b == d) + (a == d) * (b == g))
        assert abs((w * c[:, a] * c[:, b] * c[:, g] * c[:, d]).sum() - want) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_opposite_pairs_are_adjacent(dim):
    c, _ = o.lattice(dim)
    assert (c[0] == 0).all()
    for i in range(1, len(c)):
        j = i + 1 if i % 2 == 1 else i - 1
        assert (c[j] == -c[i]).all()


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_moments(dim):
    c, _ = o.lattice(dim)
    rng = np.random.default_rng(0)
    for _ in range(5):
        rho = 1 + 0.1 * rng.standard_normal()
        U = np.zeros(3)
        U[:dim] = 0.05 * rng.standard_normal(dim)
        feq = o.equilibrium(dim, rho, U[:dim])
        assert abs(feq.sum() - rho) < 1e-14
        assert np.allclose(c.T @ feq, rho * U, atol=1e-15)
        Pi = np.einsum('i,ia,ib->ab', feq, c, c)
        want = rho * CS2 * np.diag([1.0] * dim + [0.0] * (3 - dim)) + rho * np.outer(U, U)
        assert np.allclose(Pi, want, atol=1e-15)
    # at rest the equilibrium is rho * w
    _, w = o.lattice(dim)
    assert np.allclose(o.equilibrium(dim, 1.3, [0.0] * dim), 1.3 * w, atol=1e-16)


@pytest.mark.parametrize("dim", [2, 3])
def test_guo_source_moments(dim):
    c, _ = o.lattice(dim)
    rng = np.random.default_rng(1)
    for tau in (0.6, 1.0, 1.7):
        U = np.zeros(3)
        F = np.zeros(3)
        U[:dim] = 0.05 * rng.standard_normal(dim)
        F[:dim] = 1e-3 * rng.standard_normal(dim)
        S = o.guo_source(dim, tau, U[:dim], F[:dim])
        pre = 1 - 1 / (2 * tau)
        assert abs(S.sum()) < 1e-17
        assert np.allclose(c.T @ S, pre * F, atol=1e-17)
        M2 = np.einsum('i,ia,ib->ab', S, c, c)
        assert np.allclose(M2, pre * (np.outer(U, F) + np.outer(F, U)), atol=1e-17)
    # the prefactor vanishes at tau = 1/2
    S = o.guo_source(dim, 0.5, [0.01] * dim, [1e-3] * dim)
    assert np.allclose(S, 0.0, atol=1e-18)


def _random_state(dim, nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    Q = 9 if dim == 2 else 19
    _, w = o.lattice(dim)
    f = w[:, None, None, None] * (1 + 0.05 * rng.standard_normal((Q, nz, ny, nx)))
    F = np.zeros((3, nz, ny, nx))
    F[:dim] = 1e-3 * rng.standard_normal((dim, nz, ny, nx))
    return np.ascontiguousarray(f), F


@pytest.mark.parametrize("dim", [2, 3])
def test_step_adds_exactly_the_force_to_momentum(dim):
    """Post-collision momentum = pre-collision momentum + F dt in every
    cell (half-force U and Guo source together); on a fully periodic box the
    streaming only permutes, so the totals obey the same law."""
    nx, ny, nz = (6, 5, 1) if dim == 2 else (4, 3, 5)
    c, _ = o.lattice(dim)
    f, F = _random_state(dim, nx, ny, nz, 2)
    fo, rho, U = o.lb_step(dim, nx, ny, nz, (0, 0, 0), 0.8, f, F)
    mom_in = np.einsum('ia,izyx->a', c, f)
    mom_out = np.einsum('ia,izyx->a', c, fo)
    assert np.allclose(mom_out, mom_in + F.reshape(3, -1).sum(axis=1), atol=1e-13)
    assert abs(fo.sum() - f.sum()) < 1e-12
    # the reported U is the half-force velocity of the pulled populations
    fp, _, _ = o.lb_step(dim, nx, ny, nz, (0, 0, 0), math.inf, f, None)
    rho_p = fp.sum(axis=0)
    mom_p = np.einsum('ia,izyx->azyx', c, fp)
    assert np.allclose(rho, rho_p, atol=1e-14)
    assert np.allclose(U, (mom_p + 0.5 * F) / rho_p, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_conserved_with_walls(dim):
    nx, ny, nz = (7, 6, 1) if dim == 2 else (4, 5, 6)
    bc = (0, 1, 0) if dim == 2 else (0, 0, 1)
    f, F = _random_state(dim, nx, ny, nz, 3)
    m0 = f.sum()
    for _ in range(20):
        f, _, _ = o.lb_step(dim, nx, ny, nz, bc, 0.7, f, F)
    assert abs(f.sum() - m0) < 1e-11


@pytest.mark.parametrize("dim", [2, 3])
def test_rest_state_is_fixed_point(dim):
    nx, ny, nz = (5, 4, 1) if dim == 2 else (3, 4, 5)
    bc = (0, 1, 0) if dim == 2 else (0, 0, 1)
    f = o.rest_populations(dim, nx, ny, nz)
    fo, rho, U = o.lb_step(dim, nx, ny, nz, bc, 0.9, f, None)
    assert np.allclose(fo, f, atol=1e-16)
    assert np.allclose(rho, 1.0) and np.allclose(U, 0.0)
