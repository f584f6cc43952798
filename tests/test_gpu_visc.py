"""GPU parity of the two-viscosity path (viscosity ratio lambda != 1; Sec.
"Immersed-boundary lattice Boltzmann (IB-LB) method", last paragraph; eq.
def_lambda) against the FP64 oracle, through the C ABI.

The classification is an integer decision taken in double precision on both
sides (the oracle by winding numbers, the library by crossing counts along
rows): masks must agree exactly, on whole boxes at small sizes and on
sampled cells (mostly next to the interface) at the benchmark sizes.
Coupled runs use the tolerances of the one-fluid parity tests."""
import numpy as np
import pytest

import oracle as o
import workloads as wl
from helpers import collect, compare_fields, gpu_run, gpu_solver

pytestmark = pytest.mark.gpu


def comb_polygon():
    """Closed CCW polygon: a bar along y = 2..4 carrying twelve teeth up to
    y = 20, so a row through the teeth crosses the outline 24 times."""
    pts = [(2.0, 2.0), (56.0, 2.0), (56.0, 4.0)]
    for k in range(11, -1, -1):
        pts += [(6.0 + 4 * k, 4.0), (6.0 + 4 * k, 20.0), (4.0 + 4 * k, 20.0), (4.0 + 4 * k, 4.0)]
    pts += [(2.0, 4.0)]
    return np.array(pts) + np.array([0.25, 0.125])


def near_interface_cells(p, q, tris, n_near, n_rand, seed):
    """Flat indices of cells within 1.5 lattice units of a node, plus random
    cells."""
    rng = np.random.default_rng(seed)
    dim = p.dim
    nz = p.nz if dim == 3 else 1
    n = np.array([p.nx, p.ny, nz])
    pick = rng.choice(q.shape[0], size=n_near)
    base = np.zeros((n_near, 3))
    base[:, :dim] = q[pick]
    off = rng.uniform(-1.5, 1.5, size=(n_near, 3))
    off[:, dim:] = 0.0
    c = np.floor(base + off).astype(np.int64)
    for a in range(3):
        c[:, a] = np.mod(c[:, a], n[a]) if (a < dim and p.bc[a] == wl.BC_PERIODIC) else \
            np.clip(c[:, a], 0, n[a] - 1)
    near = (c[:, 2] * p.ny + c[:, 1]) * p.nx + c[:, 0]
    rand = rng.integers(0, p.nx * p.ny * nz, size=n_rand)
    return np.unique(np.concatenate([near, rand]))


@pytest.mark.parametrize("shape", ["circle", "lshape", "straddle", "cw"])
def test_inside_mask_2d_shapes(shape):
    p = wl.Params(dim=2, nx=67, ny=45, bc=(wl.BC_PERIODIC, wl.BC_WALL, wl.BC_PERIODIC),
                  wetting=False)
    if shape == "circle":
        q = wl.circle_polygon(15.3, 300, (30.2, 21.7))
    elif shape == "lshape":
        q = np.array([[2.25, 1.75], [44.75, 1.75], [44.75, 9.25], [17.25, 9.25], [17.25, 40.75],
                      [2.25, 40.75]])
    elif shape == "straddle":
        q = wl.circle_polygon(12.4, 200, (64.3, 20.6))
    else:
        q = wl.circle_polygon(15.3, 300, (30.2, 21.7))[::-1].copy()
    print(f"[visc] inside mask 2d {shape}", flush=True)
    s = gpu_solver([p], [q])
    m = s.inside_mask(0).cpu().numpy()
    want = o.inside_mask(p, q)
    assert np.array_equal(m, want) and want.sum() > 200


def test_inside_mask_3d_box_exact():
    """Cap of radius 12 on a 64x64x32 box (periodic x, y), coarse mesh: whole
    box against the oracle."""
    p = wl.Params(dim=3, nx=64, ny=64, nz=32, bc=(wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_WALL),
                  tau=0.8, sigma=0.005, theta_eq_deg=90.0, xi=2.0)
    V, T = wl.cap_mesh(12.0, 90.0, p.xi, 8, (61.7, 32.4))  # across the periodic x edge
    print("[visc] inside mask 3d 64x64x32", flush=True)
    s = gpu_solver([p], [V], [T])
    m = s.inside_mask(0).cpu().numpy()
    want = o.inside_mask(p, V, T)
    assert np.array_equal(m, want) and want.sum() > 2000


def test_inside_mask_full_size_2d_sampled():
    """The 1024x512 benchmark droplet (1024 nodes): sampled cells, mostly
    within 1.5 of the interface, against the oracle."""
    W = wl.droplet_2d_large(run=1)
    print("[visc] inside mask 1024x512 sampled", flush=True)
    s = gpu_solver([W.params], [W.nodes])
    m = s.inside_mask(0).cpu().numpy().ravel()
    cells = near_interface_cells(W.params, W.nodes, None, 6000, 2000, seed=11)
    want = o.inside_cells(W.params, W.nodes, cells)
    assert np.array_equal(m[cells], want)
    # enclosed area against the count of inside cells
    assert abs(m.sum() - o.volume_2d(W.nodes)) < 0.01 * o.volume_2d(W.nodes)


def test_inside_mask_full_size_3d_sampled():
    """The 256x256x128 benchmark cap (R = 40, 40500 triangles): sampled cells
    against the oracle, and every cell farther than 1 from the cap's surface
    against the closed form of a spherical cap above the plane z = xi."""
    W = wl.droplet_3d(small=False)
    p, V, T = W.params, W.nodes, W.tris
    print("[visc] inside mask 256x256x128 sampled", flush=True)
    s = gpu_solver([p], [V], [T])
    m = s.inside_mask(0).cpu().numpy()
    cells = near_interface_cells(p, V, T, 3000, 1000, seed=12)
    want = o.inside_cells(p, V, cells, T)
    assert np.array_equal(m.ravel()[cells], want)
    # closed form: the mesh's vertices lie on a sphere of radius 40 about
    # (128, 128, xi) (90-degree cap) or on its base disc at z = xi
    z, y, x = np.meshgrid(np.arange(p.nz) + 0.5, np.arange(p.ny) + 0.5, np.arange(p.nx) + 0.5,
                          indexing="ij")
    c = np.array([128.0, 128.0, p.xi])
    d = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    sure_in = (d < 39.0) & (z > p.xi + 1.0)
    sure_out = (d > 41.0) | (z < p.xi - 1.0)
    assert np.all(m[sure_in] == 1) and np.all(m[sure_out] == 0)


def test_two_viscosities_droplet_300_steps():
    """128x64 droplet (R = 20, 128 nodes), lambda = 10: 300 coupled steps
    (graph replays and direct launches) against the oracle."""
    W = wl.droplet_2d_small()
    p = wl.Params(**{**W.params.to_dict(), "lam": 10.0})
    print("[visc] droplet_2d_small lambda=10 300 steps", flush=True)
    g = gpu_run(p, W.nodes, 300)
    r = o.run(p, W.nodes, 300)
    drho, du, dq = compare_fields(g, r, 2, "lambda10-300")
    assert drho <= 1e-5 and du <= 1e-5 and dq <= 1e-5
    # the ratio shows at this tolerance
    g1 = gpu_run(W.params, W.nodes, 300)
    assert np.max(np.abs(g1["U"] - g["U"])) > 100 * du * np.max(np.abs(r["U"]))


@pytest.mark.parametrize("variant", [0, 4, 8, 11, 12, 15])
def test_two_viscosities_lattice_variants(variant):
    """Every tile shape and load/store kind takes the classification (BX >= 64
    keeps each wavefront on one row; the flat form reads the row per lane)."""
    W = wl.droplet_2d_small()
    p = wl.Params(**{**W.params.to_dict(), "lam": 0.3})
    print(f"[visc] variant {variant}", flush=True)
    g = gpu_run(p, W.nodes, 20, shape=variant, graph_steps=4)
    r = o.run(p, W.nodes, 20)
    drho, du, dq = compare_fields(g, r, 2, f"lambda0.3-variant{variant}")
    assert drho <= 1e-5 and du <= 1e-5 and dq <= 1e-6


@pytest.mark.parametrize("variant", [0, 13])
def test_two_viscosities_3d_across_periodic_edge(variant):
    p = wl.Params(dim=3, nx=30, ny=28, nz=16, bc=(wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_WALL),
                  tau=0.7, sigma=0.006, theta_eq_deg=80.0, xi=2.0, lam=6.0)
    V, T = wl.cap_mesh(8.0, 90.0, 2.0, 5, (1.5, 27.3))
    print(f"[visc] 3d lambda=6 6 steps, variant {variant}", flush=True)
    g = gpu_run(p, V, 6, tris=T, graph_steps=2, shape=variant)
    r = o.run(p, V, 6, tris=T)
    drho, du, dq = compare_fields(g, r, 3, "3d-lambda6")
    assert drho <= 1e-5 and du <= 1e-5 and dq <= 1e-6
    ref = o.reference_point(V)
    m = g["solver"].inside_mask(0).cpu().numpy()
    assert np.array_equal(m, o.inside_mask(p, g["q"], T, ref=ref))


def test_two_viscosities_batch():
    """Eight droplets of the batch workload with ratios from 0.1 to 10 (and
    one at 1) in one handle: each against its own oracle run."""
    draws = wl.batch_draws(n=8, seed=21)
    lams = [0.1, 0.5, 1.0, 2.0, 4.0, 7.0, 10.0, 3.0]
    ps = [wl.Params(**{**w.params.to_dict(), "lam": lam}) for w, lam in zip(draws, lams)]
    qs = [w.nodes for w in draws]
    print("[visc] batch of 8, 40 steps", flush=True)
    s = gpu_solver(ps, qs)
    s.set_graph_steps(8)
    s.step(40)
    for d in range(len(ps)):
        g = collect(s, d, 2)
        r = o.run(ps[d], qs[d], 40)
        drho, du, dq = compare_fields(g, r, 2, f"batch-lambda{lams[d]}")
        assert drho <= 1e-5 and du <= 1e-5 and dq <= 1e-6


def test_ratio_one_restores_the_one_fluid_path():
    """5 steps at lambda = 10, then 7 at lambda = 1 on the same handle, against
    the oracle run the same way (spreading adds in fp32 atomics, so two GPU
    runs agree to rounding, not bit for bit)."""
    W = wl.droplet_2d_small()
    p10 = wl.Params(**{**W.params.to_dict(), "lam": 10.0})
    print("[visc] lambda 10 then 1", flush=True)
    a = gpu_solver([W.params], [W.nodes])
    a.set_viscosity_ratio(0, 10.0)
    a.step(5)
    a.set_viscosity_ratio(0, 1.0)
    a.step(7)
    r5 = o.run(p10, W.nodes, 5)
    r = o.run(W.params, r5["q"], 7, f0=r5["f"])
    drho, du, dq = compare_fields(collect(a, 0, 2), r, 2, "lambda10-then-1")
    assert drho <= 1e-5 and du <= 1e-5 and dq <= 1e-6


def test_too_many_crossings_on_a_row_is_reported():
    p = wl.Params(dim=2, nx=64, ny=32, tau=0.8, sigma=0.005, wetting=False)
    q = comb_polygon()
    assert o.inside_mask(p, q).sum() > 0
    s = gpu_solver([p], [q])
    with pytest.raises(Exception, match="IBLB_ELIMIT"):
        s.inside_mask(0)
    s.set_viscosity_ratio(0, 3.0)
    with pytest.raises(Exception, match="IBLB_ELIMIT"):
        s.step(2)


def test_droplet_wider_than_the_window_is_reported():
    """An ellipse wider than the periodic box along x: its nodes cannot all
    lie in the classification window, which the mask and the step report."""
    p = wl.Params(dim=2, nx=40, ny=32, tau=0.8, sigma=0.004, wetting=False)
    t = 2.0 * np.pi * np.arange(120) / 120
    q = np.stack([20.0 + 22.0 * np.cos(t), 16.0 + 6.0 * np.sin(t)], axis=1)
    s = gpu_solver([p], [q])
    with pytest.raises(Exception, match="IBLB_ELIMIT"):
        s.inside_mask(0)
    s.set_viscosity_ratio(0, 2.0)
    with pytest.raises(Exception, match="IBLB_ELIMIT"):
        s.step(1)

