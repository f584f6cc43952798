"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only draws and lays out inputs: lattice sizes, physical
parameters, initial interface meshes (a circular cap sitting on the wall, a
free circle or sphere) and tagged population arrays.  It holds none of the
method's arithmetic (no forces, no delta kernel, no collision, no wetting
strength), so both sides of every parity test consume identical inputs
without sharing any of the computation being checked.

Geometry conventions (lattice units, dx = dt = 1):
  * fluid cells are centred at (i + 1/2, j + 1/2[, k + 1/2]);
  * the substrate is the plane y = 0 in 2D and z = 0 in 3D, so the height of
    a node above it is simply its last coordinate;
  * a 2D interface is a closed polygon listed counter-clockwise, so the
    outward normal of edge q_j -> q_{j+1} is the edge rotated by -90 degrees;
  * a 3D interface is a closed triangle mesh, each triangle listed
    counter-clockwise when seen from outside.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

BC_PERIODIC = 0
BC_WALL = 1


@dataclass
class Params:
    """Physical and lattice parameters of one droplet simulation."""
    dim: int = 2
    nx: int = 128
    ny: int = 64
    nz: int = 1
    # boundary condition per axis; walls are half-way bounce-back planes at
    # coordinate 0 and at coordinate n of that axis
    bc: tuple = (BC_PERIODIC, BC_WALL, BC_PERIODIC)
    tau: float = 1.0
    sigma: float = 0.01
    theta_eq_deg: float = 60.0
    xi: float = 2.0
    n_exp: int = 6
    m_exp: int = 3
    # whether the wetting interaction acts (substrate at the low end of the
    # last axis); off for a free droplet in a periodic box
    wetting: bool = True
    # viscosity ratio mu_in / mu_out of the fluid inside the interface to the
    # fluid outside (tau is the outside relaxation time); 1: one fluid
    lam: float = 1.0
    # surface shear modulus of an elastic interface (3D; the stress-free
    # reference is the mesh as first set); 0: a liquid droplet
    shear: float = 0.0
    # rate beta of the tangential re-spacing of a 2D outline (nodes moved
    # along the chord of their neighbours by beta/2 times the difference of
    # their two edge lengths each step; an addition for long runs); 0: off
    respace: float = 0.0

    def to_dict(self):
        return asdict(self)


# ----------------------------------------------------------------------------
# 2D interfaces
# ----------------------------------------------------------------------------

def cap_polygon(R: float, theta_deg: float, base_h: float, n_nodes: int,
                xc: float) -> np.ndarray:
    """Closed CCW polygon of a circular cap of circle radius R whose flat base
    lies on the line y = base_h and meets the arc at angle theta (measured
    inside the liquid).  Nodes are spaced uniformly in arc length along the
    closed outline (arc, then base), node 0 at the right contact corner.
    Returns an (n_nodes, 2) float64 array."""
    th = math.radians(theta_deg)
    yc = base_h - R * math.cos(th)
    arc = 2.0 * th * R
    base = 2.0 * R * math.sin(th)
    perim = arc + base
    s = np.arange(n_nodes, dtype=np.float64) * (perim / n_nodes)
    pts = np.empty((n_nodes, 2), dtype=np.float64)
    a0 = 0.5 * math.pi - th
    on_arc = s < arc
    ang = a0 + s[on_arc] / R
    pts[on_arc, 0] = xc + R * np.cos(ang)
    pts[on_arc, 1] = yc + R * np.sin(ang)
    sb = s[~on_arc] - arc
    pts[~on_arc, 0] = xc - R * math.sin(th) + sb
    pts[~on_arc, 1] = base_h
    return pts


def circle_polygon(R: float, n_nodes: int, center) -> np.ndarray:
    """Regular CCW n-gon inscribed in a circle of radius R."""
    a = 2.0 * math.pi * np.arange(n_nodes, dtype=np.float64) / n_nodes
    return np.stack([center[0] + R * np.cos(a), center[1] + R * np.sin(a)], axis=1)


def equal_area_cap(area: float, theta_deg: float):
    """Circle radius, base half-width and height of the 2D circular cap of
    the given area and contact angle (used only to reject draws that would
    not fit their box)."""
    th = math.radians(theta_deg)
    rc = math.sqrt(area / (th - math.sin(th) * math.cos(th)))
    return rc, rc * math.sin(th), rc * (1.0 - math.cos(th))


# ----------------------------------------------------------------------------
# 3D interfaces
# ----------------------------------------------------------------------------

def icosphere(nu: int):
    """Class-I geodesic sphere of frequency nu: each icosahedron face split
    into nu^2 triangles, vertices pushed onto the unit sphere.
    Returns (verts (10 nu^2 + 2, 3) float64, tris (20 nu^2, 3) int32), each
    triangle counter-clockwise seen from outside."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    base = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                     [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                     [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    base /= np.linalg.norm(base, axis=1, keepdims=True)
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = []
    index = {}

    def vid(a, b, c, i, j):
        # lattice point i*(B-A)/nu + j*(C-A)/nu on face (a,b,c); shared
        # points on edges/corners get one id through a canonical key
        k = nu - i - j
        wts = {a: k, b: i, c: j}
        key = tuple(sorted((v, w) for v, w in wts.items() if w > 0))
        if key not in index:
            pt = sum(w * base[v] for v, w in key) / nu
            index[key] = len(verts)
            verts.append(pt / np.linalg.norm(pt))
        return index[key]

    tris = []
    for (a, b, c) in faces:
        for i in range(nu):
            for j in range(nu - i):
                v0 = vid(a, b, c, i, j)
                v1 = vid(a, b, c, i + 1, j)
                v2 = vid(a, b, c, i, j + 1)
                tris.append((v0, v1, v2))
                if i + j < nu - 1:
                    v3 = vid(a, b, c, i + 1, j + 1)
                    tris.append((v1, v3, v2))
    V = np.array(verts, dtype=np.float64)
    T = np.array(tris, dtype=np.int32)
    # orient every triangle counter-clockwise seen from outside
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    flip = np.einsum('ij,ij->i', np.cross(b - a, c - a), a + b + c) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return V, T


def cap_mesh(R: float, theta_deg: float, base_h: float, nu: int, center_xy):
    """Closed triangle mesh of a spherical cap (sphere radius R, contact
    angle theta, flat base disk on the plane z = base_h), obtained by
    projecting a frequency-nu icosphere radially from an interior point onto
    the cap surface (the cap is convex, so the projection is one-to-one).
    Returns (verts (V,3) float64, tris (T,3) int32)."""
    th = math.radians(theta_deg)
    U, T = icosphere(nu)
    zc = base_h - R * math.cos(th)
    H = R * (1.0 - math.cos(th))
    p0 = np.array([center_xy[0], center_xy[1], base_h + 0.4 * H])
    C = np.array([center_xy[0], center_xy[1], zc])
    # exit distance along each ray through the ball |x - C| <= R
    m = p0 - C
    bq = U @ m
    cq = m @ m - R * R
    t_sph = -bq + np.sqrt(bq * bq - cq)
    # exit distance through the half space z >= base_h
    with np.errstate(divide='ignore'):
        t_pln = np.where(U[:, 2] < 0, (base_h - p0[2]) / U[:, 2], np.inf)
    t = np.minimum(t_sph, t_pln)
    V = p0[None, :] + t[:, None] * U
    on_base = t_pln <= t_sph
    V[on_base, 2] = base_h
    return V, T


def sphere_mesh(R: float, nu: int, center):
    U, T = icosphere(nu)
    return np.asarray(center, dtype=np.float64)[None, :] + R * U, T


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    params: Params
    nodes: np.ndarray                 # (N, dim) float64
    tris: np.ndarray | None = None    # (T, 3) int32 in 3D, None in 2D
    steps: int = 0
    meta: dict = field(default_factory=dict)


def droplet_2d_small(steps: int = 2000) -> Workload:
    """128x64 D2Q9, tau = 1, walls at y = 0 and y = 64, periodic x; a
    half-disk cap of radius 20 (90 degrees) with 128 nodes, base at h = xi = 2,
    centred at x = 64; sigma = 0.01, theta_eq = 60 degrees."""
    p = Params(dim=2, nx=128, ny=64, tau=1.0, sigma=0.01, theta_eq_deg=60.0, xi=2.0)
    q = cap_polygon(20.0, 90.0, p.xi, 128, 64.0)
    return Workload("d2q9_128x64_R20_N128", p, q, steps=steps)


def droplet_2d_large(run: int = 0, steps: int = 50000) -> Workload:
    """1024x512 D2Q9 plain FP32 sweep point `run` in 0..9: tau in {0.6, 1.0}
    times theta_eq in {30, 60, 90, 120, 150} degrees; circle radius 120, 1024
    nodes, xi = 3, sigma = 0.005, initial cap angle theta_eq + U(-5, 5)
    degrees drawn from seed 1000 + run."""
    taus = (0.6, 1.0)
    thetas = (30.0, 60.0, 90.0, 120.0, 150.0)
    tau = taus[run // 5]
    th = thetas[run % 5]
    rng = np.random.default_rng(1000 + run)
    th0 = th + rng.uniform(-5.0, 5.0)
    p = Params(dim=2, nx=1024, ny=512, tau=tau, sigma=0.005, theta_eq_deg=th, xi=3.0)
    q = cap_polygon(120.0, th0, p.xi, 1024, 512.0)
    return Workload(f"d2q9_1024x512_R120_N1024_run{run}", p, q, steps=steps,
                    meta={"theta0_deg": th0})


def batch_draws(n: int = 256, seed: int = 3):
    """Independent droplets of uneven box size and wettability: Nx in
    {128,...,512} and Ny in {64,...,256} (multiples of 32), circle radius
    R ~ U[15, 100] with round(2 pi R / 0.8) nodes, theta_eq ~ U[20, 160] deg,
    tau ~ U[0.6, 1.5], sigma ~ U[0.002, 0.01], xi = 2, tangential node
    re-spacing at rate 0.05 (these droplets are run for up to 10^6 steps).
    A draw is rejected and redrawn when the 90-degree start or the
    equal-area theta_eq cap would not fit its box.  Returns a list of
    Workloads starting from the half disk."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        nx = int(rng.integers(4, 17)) * 32
        ny = int(rng.integers(2, 9)) * 32
        R = float(rng.uniform(15.0, 100.0))
        th = float(rng.uniform(20.0, 160.0))
        tau = float(rng.uniform(0.6, 1.5))
        sigma = float(rng.uniform(0.002, 0.01))
        xi = 2.0
        nn = int(round(2.0 * math.pi * R / 0.8))
        area = 0.5 * math.pi * R * R
        _, half_w, h = equal_area_cap(area, th)
        fits90 = 2 * R <= nx - 32 and R + xi <= ny - 8
        fits_eq = 2 * half_w <= nx - 32 and h + xi <= ny - 8
        if not (fits90 and fits_eq):
            continue
        p = Params(dim=2, nx=nx, ny=ny, tau=tau, sigma=sigma, theta_eq_deg=th, xi=xi, respace=0.05)
        q = cap_polygon(R, 90.0, xi, nn, nx / 2.0)
        out.append(Workload(f"batch{len(out)}", p, q, meta={"R": R}))
    return out


def droplet_3d(theta_eq_deg: float = 90.0, small: bool = False) -> Workload:
    """D3Q19 droplet on the wall z = 0, periodic x and y, wall also at the
    top.  Full size: 256x256x128, hemispherical cap R = 40 from a
    frequency-45 icosphere (40500 triangles, 20252 vertices), xi = 4,
    sigma = 0.005, tau = 0.8.  Small copy: 64x64x32, R = 12, frequency 20,
    xi = 2."""
    if small:
        p = Params(dim=3, nx=64, ny=64, nz=32, bc=(BC_PERIODIC, BC_PERIODIC, BC_WALL),
                   tau=0.8, sigma=0.005, theta_eq_deg=theta_eq_deg, xi=2.0)
        V, T = cap_mesh(12.0, 90.0, p.xi, 20, (32.0, 32.0))
        name = "d3q19_64x64x32_R12"
    else:
        p = Params(dim=3, nx=256, ny=256, nz=128, bc=(BC_PERIODIC, BC_PERIODIC, BC_WALL),
                   tau=0.8, sigma=0.005, theta_eq_deg=theta_eq_deg, xi=4.0)
        V, T = cap_mesh(40.0, 90.0, p.xi, 45, (128.0, 128.0))
        name = "d3q19_256x256x128_R40"
    return Workload(name, p, V, tris=T)


def droplet_3d_spreading(lam: float = 10.0, theta_eq_deg: float = 60.0) -> Workload:
    """Set-up of the paper's spreading runs (Sec. Dynamics): a 240x240x130
    D3Q19 box (periodic x and y, walls at z = 0 and z = 130), a sphere of
    radius R0 = 60 whose lowest point sits at h = 1.5 xi above the
    substrate, xi = 2, viscosity ratio lam.  The sphere is a frequency-64
    icosphere (81920 triangles, 40962 vertices, edges about 1 lattice unit);
    tau_out = 0.8, sigma = 0.005 (the paper does not list them)."""
    p = Params(dim=3, nx=240, ny=240, nz=130, bc=(BC_PERIODIC, BC_PERIODIC, BC_WALL),
               tau=0.8, sigma=0.005, theta_eq_deg=theta_eq_deg, xi=2.0, lam=lam)
    R0 = 60.0
    V, T = sphere_mesh(R0, 64, (120.0, 120.0, R0 + 1.5 * p.xi))
    return Workload(f"d3q19_240x240x130_R60_lam{lam:g}", p, V, tris=T)


def droplet_3d_statics(theta_eq_deg: float, xi_over_R0: float = 0.1, nu: int = 45) -> Workload:
    """Set-up of the paper's equilibrium runs (Sec. Statics): an 80x80x60
    D3Q19 box (periodic x and y, walls at z = 0 and 60), a sphere of radius
    R0 = 20 from a frequency-nu icosphere (nu = 45: 40500 triangles, the
    paper's N_t = 40 000) with its lowest point at h = 1.5 xi, xi = xi_over_R0
    R0, viscosity ratio 1; tau = 1 and sigma = 0.01 (the paper does not list
    them)."""
    R0 = 20.0
    p = Params(dim=3, nx=80, ny=80, nz=60, bc=(BC_PERIODIC, BC_PERIODIC, BC_WALL),
               tau=1.0, sigma=0.01, theta_eq_deg=theta_eq_deg, xi=xi_over_R0 * R0)
    V, T = sphere_mesh(R0, nu, (40.0, 40.0, R0 + 1.5 * p.xi))
    return Workload(f"d3q19_80x80x60_R20_theta{theta_eq_deg:g}_xi{xi_over_R0:g}", p, V, tris=T,
                    meta={"R0": R0})


def droplet_2d_statics(theta_eq_deg: float, xi_over_R0: float = 0.1,
                       n_nodes: int = 800) -> Workload:
    """2D counterpart of the equilibrium runs: a 128x80 D2Q9 box (periodic x,
    walls at y = 0 and 80), a circle of radius R0 = 20 with n_nodes nodes
    whose lowest point sits at h = 1.5 xi, xi = xi_over_R0 R0, tau = 1,
    sigma = 0.01.  A line tension does not hold the nodes in place along the
    outline, and spreading stretches the base most, so the outline gets
    several nodes per lattice unit: with 200 the largest gap grows past 3
    lattice units at 45 degrees and fluid leaks through it."""
    R0 = 20.0
    p = Params(dim=2, nx=128, ny=80, tau=1.0, sigma=0.01, theta_eq_deg=theta_eq_deg,
               xi=xi_over_R0 * R0)
    q = circle_polygon(R0, n_nodes, (64.0, R0 + 1.5 * p.xi))
    return Workload(f"d2q9_128x80_R20_n{n_nodes}_theta{theta_eq_deg:g}_xi{xi_over_R0:g}", p, q,
                    meta={"R0": R0})


def droplet_3d_tanner(theta_eq_deg: float = 22.5, R0: float = 60.0, xi: float = 3.0,
                      nu: int = 80) -> Workload:
    """Late-stage (viscous) spreading set-up after Sec. Dynamics: the droplet
    starts as a hemisphere of the volume of a sphere of radius R0 (so the
    inertial stage is skipped) on the substrate of a periodic box wide enough
    for its equilibrium cap at theta_eq (contact radius about 2.4 R0 at
    22.5 deg), xi = 3.  Frequency-nu icosphere projected onto the cap (nu = 80:
    128000 triangles, edges of about 1.4 lattice units at R0 = 60); tau = 0.8,
    sigma = 0.005 (the paper lists neither)."""
    Rc = R0 * 2.0 ** (1.0 / 3.0)                       # hemisphere of the sphere's volume
    th = math.radians(theta_eq_deg)
    # equilibrium cap of the same volume: V = (pi/3) R^3 (2 - 3 cos + cos^3)
    Req = (4.0 * R0 ** 3 / (2.0 - 3.0 * math.cos(th) + math.cos(th) ** 3)) ** (1.0 / 3.0)
    r_eq = Req * math.sin(th)
    n = int(math.ceil((2.0 * r_eq + 40.0) / 16.0)) * 16
    nz = int(math.ceil((Rc + xi + 20.0) / 16.0)) * 16
    p = Params(dim=3, nx=n, ny=n, nz=nz, bc=(BC_PERIODIC, BC_PERIODIC, BC_WALL),
               tau=0.8, sigma=0.005, theta_eq_deg=theta_eq_deg, xi=xi)
    V, T = cap_mesh(Rc, 90.0, xi, nu, (n / 2.0, n / 2.0))
    return Workload(f"d3q19_{n}x{n}x{nz}_R{R0:g}_theta{theta_eq_deg:g}_tanner", p, V, tris=T,
                    meta={"R0": R0, "r_eq": r_eq})


# ----------------------------------------------------------------------------
# Raw arrays for unit and parity tests
# ----------------------------------------------------------------------------

def tagged_deviation(q: int, cells: int, seed: int, kmax: int = 100) -> np.ndarray:
    """Population deviations k * 2^-10 with integer k in [-kmax, kmax]: exact
    in fp16, bf16, fp32 and fp64 once the weight is added back or removed."""
    rng = np.random.default_rng(seed)
    return rng.integers(-kmax, kmax + 1, size=(q, cells)).astype(np.float64) * 2.0 ** -10


def random_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(shape)
