"""Pins of the oracle's two-viscosity pieces (Sec. "Immersed-boundary lattice
Boltzmann (IB-LB) method", last paragraph; eq. def_lambda): the
inside/outside classification of cells against the closed interface and
the LB update with a relaxation time per cell.

The classification is pinned by shapes whose interior has a closed form
(circle and sphere up to their discretisation band, an axis-aligned
L-shaped polygon, a box), both orientations, and a droplet straddling a
periodic edge.  The relaxation-time field is pinned by locality (every cell
takes the collision of its own tau, force included) and by the steady
two-layer channel flow, whose profile is piecewise parabolic with
continuous velocity and shear stress."""
import math

import numpy as np
import pytest

import oracle as o
import workloads as wl


def centres(nx, ny, nz=1):
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                          indexing="ij")
    return x, y, z


def test_tau_inside_from_viscosity_ratio():
    # mu = rho cs^2 (tau - 1/2): lam = mu_in / mu_out
    for tau, lam in [(0.8, 10.0), (0.6, 0.25), (1.3, 1.0)]:
        t_in = o.tau_inside(tau, lam)
        assert abs((t_in - 0.5) / (tau - 0.5) - lam) < 1e-14


@pytest.mark.parametrize("ccw", [True, False])
def test_circle_polygon_inside(ccw):
    p = wl.Params(dim=2, nx=41, ny=33, bc=(wl.BC_WALL, wl.BC_WALL, wl.BC_PERIODIC))
    R, N, c = 10.3, 200, (20.2, 15.7)
    q = wl.circle_polygon(R, N, c)
    if not ccw:
        q = q[::-1].copy()
    m = o.inside_mask(p, q)[0]
    x, y, _ = centres(p.nx, p.ny)
    d = np.hypot(x - c[0], y - c[1])[0]
    r_in = R * math.cos(math.pi / N)  # distance of the edges' midpoints
    sure_in, sure_out = d < r_in - 1e-9, d > R + 1e-9
    assert np.all(m[sure_in] == 1) and np.all(m[sure_out] == 0)
    assert sure_in.sum() > 300 and (sure_in | sure_out).sum() > m.size - 80


def test_l_shaped_polygon_inside():
    """Non-convex polygon with vertices off the cell centres: the interior is
    the union of two rectangles."""
    p = wl.Params(dim=2, nx=20, ny=16, bc=(wl.BC_PERIODIC, wl.BC_WALL, wl.BC_PERIODIC))
    q = np.array([[2.25, 1.75], [14.75, 1.75], [14.75, 5.25], [7.25, 5.25], [7.25, 12.75],
                  [2.25, 12.75]])
    m = o.inside_mask(p, q)[0]
    x, y, _ = centres(p.nx, p.ny)
    x, y = x[0], y[0]
    want = (((x > 2.25) & (x < 14.75) & (y > 1.75) & (y < 5.25)) |
            ((x > 2.25) & (x < 7.25) & (y > 1.75) & (y < 12.75)))
    assert np.array_equal(m.astype(bool), want)
    assert np.array_equal(o.inside_mask(p, q[::-1].copy())[0], m)


def test_polygon_across_periodic_edge():
    """A circle centred beyond the right edge of a periodic x axis, nodes not
    wrapped: the cells enclosed are those within R of the centre in the
    periodic distance."""
    p = wl.Params(dim=2, nx=30, ny=24, bc=(wl.BC_PERIODIC, wl.BC_WALL, wl.BC_PERIODIC))
    R, N, c = 7.4, 160, (31.3, 11.6)
    q = wl.circle_polygon(R, N, c)
    m = o.inside_mask(p, q)[0]
    x, y, _ = centres(p.nx, p.ny)
    dx = np.abs(((x[0] - c[0]) + p.nx / 2) % p.nx - p.nx / 2)
    d = np.hypot(dx, y[0] - c[1])
    r_in = R * math.cos(math.pi / N)
    assert np.all(m[d < r_in - 1e-9] == 1) and np.all(m[d > R + 1e-9] == 0)
    assert m[:, :5].sum() > 20 and m[:, -5:].sum() > 20
    # the same droplet one period to the left classifies the same cells
    q2 = q - np.array([p.nx, 0.0])
    assert np.array_equal(o.inside_mask(p, q2)[0], m)


def box_mesh(lo, hi):
    """Closed triangulated box, counter-clockwise seen from outside."""
    V = np.array([[lo[0], lo[1], lo[2]], [hi[0], lo[1], lo[2]], [hi[0], hi[1], lo[2]],
                  [lo[0], hi[1], lo[2]], [lo[0], lo[1], hi[2]], [hi[0], lo[1], hi[2]],
                  [hi[0], hi[1], hi[2]], [lo[0], hi[1], hi[2]]])
    T = np.array([[0, 2, 1], [0, 3, 2], [4, 5, 6], [4, 6, 7], [0, 1, 5], [0, 5, 4],
                  [2, 3, 7], [2, 7, 6], [1, 2, 6], [1, 6, 5], [0, 4, 7], [0, 7, 3]],
                 dtype=np.int32)
    return V, T


@pytest.mark.parametrize("ccw", [True, False])
def test_box_mesh_inside(ccw):
    p = wl.Params(dim=3, nx=10, ny=9, nz=8, bc=(wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_WALL))
    lo, hi = (2.25, 3.25, 1.75), (7.75, 6.75, 5.25)
    V, T = box_mesh(lo, hi)
    # outward normals of the box faces
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(b - a, c - a)
    mid = 0.5 * (np.array(lo) + np.array(hi))
    assert np.all(np.einsum("ij,ij->i", n, (a + b + c) / 3 - mid) > 0)
    if not ccw:
        T = T[:, ::-1].copy()
    m = o.inside_mask(p, V, T)
    x, y, z = centres(p.nx, p.ny, p.nz)
    want = ((x > lo[0]) & (x < hi[0]) & (y > lo[1]) & (y < hi[1]) & (z > lo[2]) & (z < hi[2]))
    assert np.array_equal(m.astype(bool), want)


def test_sphere_mesh_inside_and_across_periodic_edge():
    p = wl.Params(dim=3, nx=18, ny=16, nz=16, bc=(wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_WALL))
    R, c = 5.6, (16.9, 8.2, 8.1)  # crosses the periodic x edge
    V, T = wl.sphere_mesh(R, 6, c)
    m = o.inside_mask(p, V, T)
    a, b, cc = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(b - a, cc - a)
    n /= np.linalg.norm(n, axis=1)[:, None]
    r_in = np.min(np.abs(np.einsum("ij,ij->i", n, a - np.array(c))))  # closest face plane
    x, y, z = centres(p.nx, p.ny, p.nz)
    dx = np.abs(((x - c[0]) + p.nx / 2) % p.nx - p.nx / 2)
    d = np.sqrt(dx ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    sure_in, sure_out = d < r_in - 1e-9, d > R + 1e-9
    assert np.all(m[sure_in] == 1) and np.all(m[sure_out] == 0)
    assert sure_in.sum() > 400
    # inside count against the enclosed volume
    vol = o.volume_3d(V, T)
    assert abs(m.sum() - vol) < 0.15 * vol


def test_cap_mesh_inside_count_matches_volume():
    p = wl.Params(dim=3, nx=32, ny=32, nz=20, bc=(wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_WALL))
    V, T = wl.cap_mesh(9.0, 90.0, 2.0, 10, (16.0, 16.0))
    m = o.inside_mask(p, V, T)
    vol = o.volume_3d(V, T)
    assert abs(m.sum() - vol) < 0.08 * vol
    # nothing below the flat base, which lies at z = 2
    assert m[:2].sum() == 0 and m[2].sum() > 100


@pytest.mark.parametrize("dim", [2, 3])
def test_lb_step_tau_field_is_local(dim):
    """The update with a relaxation-time field equals, cell by cell, the
    update with that cell's tau everywhere (collision is local; the Guo
    prefactor takes the same tau), force included."""
    nx, ny, nz = (11, 7, 1) if dim == 2 else (7, 6, 5)
    bc = (0, 1, 0) if dim == 2 else (0, 0, 1)
    Q = 9 if dim == 2 else 19
    rng = np.random.default_rng(5)
    _, w = o.lattice(dim)
    f = w[:, None] * (1.0 + 0.05 * rng.standard_normal((Q, nz * ny * nx)))
    F = np.zeros((3, nz, ny, nx))
    F[:dim] = 1e-3 * rng.standard_normal((dim, nz, ny, nx))
    mask = rng.random((nz, ny, nx)) < 0.4
    t_in, t_out = 3.1, 0.62
    tau_cell = np.where(mask, t_in, t_out)
    got, rho, U = o.lb_step(dim, nx, ny, nz, bc, t_out, f, F, tau_cell=tau_cell)
    a, rho_a, U_a = o.lb_step(dim, nx, ny, nz, bc, t_in, f, F)
    b, rho_b, U_b = o.lb_step(dim, nx, ny, nz, bc, t_out, f, F)
    want = np.where(mask[None], a, b)
    assert np.array_equal(got, want)
    assert np.array_equal(rho, rho_a) and np.array_equal(U, U_b)
    assert not np.array_equal(a, b)


def test_two_layer_channel_flow():
    """Steady channel flow between walls at y = 0 and y = H driven by a body
    force g, the lower layer (y < h) with viscosity nu1 and the upper with
    nu2: u is parabolic in each layer with u = 0 at the walls, u and
    nu u' continuous at y = h (rho = 1)."""
    H, h, g = 24, 12, 1e-6
    tau1, tau2 = 0.8, 2.3
    nu1, nu2 = (tau1 - 0.5) / 3, (tau2 - 0.5) / 3
    nx, ny = 2, H
    _, y, _ = centres(nx, ny)
    tau_cell = np.where(y < h, tau1, tau2)
    F = np.zeros((3, 1, ny, nx))
    F[0] = g
    f = o.rest_populations(2, nx, ny)
    for _ in range(12000):
        f, rho, U = o.lb_step(2, nx, ny, 1, (0, 1, 0), tau1, f, F, tau_cell=tau_cell)
    u = U[0, 0, :, 0]
    # u_k(y) = -g y^2 / (2 nu_k) + a_k y + b_k; b1 = 0, u2(H) = 0,
    # u1(h) = u2(h), nu1 u1'(h) = nu2 u2'(h)
    Amat = np.array([[h, -h, -1.0],
                     [0.0, H, 1.0],
                     [nu1, -nu2, 0.0]])
    rhs = np.array([g * h * h / (2 * nu1) - g * h * h / (2 * nu2),
                    g * H * H / (2 * nu2),
                    0.0])
    a1, a2, b2 = np.linalg.solve(Amat, rhs)
    yc = np.arange(ny) + 0.5
    exact = np.where(yc < h, -g * yc ** 2 / (2 * nu1) + a1 * yc,
                     -g * yc ** 2 / (2 * nu2) + a2 * yc + b2)
    err = np.max(np.abs(u - exact)) / np.max(exact)
    assert err < 0.02, err
    # a single-fluid channel of the lower viscosity would be much faster
    assert np.max(u) < 0.5 * g * H * H / (8 * nu1)


def test_run_classifies_at_the_start_of_each_step():
    """One coupled step with lam != 1 equals: forces and spreading at q(0),
    classification at q(0), LB with the tau field, interpolation at q(0)."""
    p = wl.Params(dim=2, nx=40, ny=24, tau=0.7, sigma=0.01, theta_eq_deg=70.0, xi=2.0, lam=8.0)
    q = wl.cap_polygon(8.0, 90.0, 2.0, 60, 20.0)
    r = o.run(p, q, 1)
    A = o.wetting_strength(p.sigma, math.radians(p.theta_eq_deg), p.xi)
    phi, _ = o.forces_2d(q, p.sigma, A, p.xi)
    F, _ = o.spread(2, p.nx, p.ny, 1, p.bc, q, phi)
    m = o.inside_mask(p, q)
    tc = np.where(m == 1, o.tau_inside(p.tau, p.lam), p.tau)
    f, rho, U = o.lb_step(2, p.nx, p.ny, 1, p.bc, p.tau, o.rest_populations(2, p.nx, p.ny), F,
                          tau_cell=tc)
    qdot = o.interp(2, p.nx, p.ny, 1, p.bc, U, q)
    assert np.array_equal(r["f"], f) and np.array_equal(r["q"], q + qdot)
    # and lam changes the result
    p1 = wl.Params(**{**p.to_dict(), "lam": 1.0})
    assert not np.array_equal(o.run(p1, q, 1)["f"], f)


def test_inside_cells_matches_the_full_mask():
    p = wl.Params(dim=3, nx=18, ny=16, nz=16, bc=(wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_WALL))
    V, T = wl.sphere_mesh(5.6, 4, (16.9, 8.2, 8.1))
    m = o.inside_mask(p, V, T).ravel()
    cells = np.arange(m.size)[3::5]
    assert np.array_equal(o.inside_cells(p, V, cells, T), m[cells])
