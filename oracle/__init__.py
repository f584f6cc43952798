"""FP64 CPU oracle of the IB-LB wetting model.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product library never loads
it, and it shares no code with the HIP path: the arithmetic lives in
iblb_oracle.c (plain C, double precision, plain loops) and in the numpy
diagnostics below, each citing the passage of the paper it follows.

Array conventions (numpy side):
  populations  (Q, nz, ny, nx)    float64, x fastest
  F, U         (3, nz, ny, nx)    unused components zero
  rho          (nz, ny, nx)
  nodes q      (N, dim)           lattice units, cell (i,j,k) centred at +1/2
  tris         (T, 3) int32       counter-clockwise seen from outside
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

PERIODIC = 0
WALL = 1


def _load():
    global _lib
    if _lib is not None:
        return _lib
    src = os.path.join(_HERE, "iblb_oracle.c")
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(src):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB)
    D = ctypes.POINTER(ctypes.c_double)
    I = ctypes.POINTER(ctypes.c_int)
    c_int, c_double = ctypes.c_int, ctypes.c_double
    lib.orc_lattice.argtypes = [c_int, I, D]
    lib.orc_equilibrium.argtypes = [c_int, c_double, D, D]
    lib.orc_guo_source.argtypes = [c_int, c_double, D, D, D]
    lib.orc_lb_step.argtypes = [c_int, c_int, c_int, c_int, I, c_double, D, D, D, D, D, D]
    lib.orc_psi.argtypes = [c_double]
    lib.orc_psi.restype = c_double
    lib.orc_spread.argtypes = [c_int, c_int, c_int, c_int, I, c_int, D, D, D, D]
    lib.orc_interp.argtypes = [c_int, c_int, c_int, c_int, I, D, c_int, D, D]
    lib.orc_wetting_strength.argtypes = [c_double, c_double, c_double, c_int, c_int]
    lib.orc_wetting_strength.restype = c_double
    lib.orc_pi.argtypes = [c_double, c_double, c_double, c_int, c_int]
    lib.orc_pi.restype = c_double
    lib.orc_forces_2d.argtypes = [c_int, D, c_double, c_double, c_double, c_int, c_int,
                                  c_int, D, D]
    lib.orc_forces_3d.argtypes = [c_int, D, c_int, I, c_double, c_double, c_double,
                                  c_int, c_int, c_int, D, D]
    lib.orc_inside.argtypes = [c_int, c_int, c_int, c_int, I, c_int, D, c_int, I, D, I]
    lib.orc_respace_2d.argtypes = [c_int, D, c_double, D]
    lib.orc_threads.argtypes = [c_int]
    lib.orc_threads.restype = c_int
    lib.orc_inside_cells.argtypes = [c_int, c_int, c_int, c_int, I, c_int, D, c_int, I, D,
                                     ctypes.c_long, ctypes.POINTER(ctypes.c_long), I]
    lib.orc_forces_3d_elastic.argtypes = [c_int, D, D, c_int, I, c_double, c_double, c_double,
                                          c_double, c_int, c_int, c_int, D, D]
    lib.orc_run.argtypes = [c_int, c_int, c_int, c_int, I, c_double, c_double, D,
                            c_double, c_double, D, c_double, c_double, c_int, c_int, c_int,
                            c_double, c_int, D, c_int, I, c_int,
                            D, D, D, D, D, D, D, D]
    lib.orc_run.restype = c_int
    _lib = lib
    return lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _bc(bc):
    return np.ascontiguousarray(np.asarray(bc, dtype=np.int32))


# --------------------------------------------------------------------------
# lattice and collision pieces
# --------------------------------------------------------------------------

def threads(n: int = 0) -> int:
    """Threads of the lattice update (OpenMP over rows); n > 0 sets the
    count.  Returns the count in force."""
    return int(_load().orc_threads(int(n)))


def lattice(dim: int):
    """Velocity set of Table I (D3Q19) or its 2D analogue D2Q9."""
    Q = 9 if dim == 2 else 19
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    _load().orc_lattice(dim, _i(c), _d(w))
    return c, w


def equilibrium(dim, rho, U):
    Q = 9 if dim == 2 else 19
    out = np.zeros(Q)
    u = np.zeros(3)
    u[:len(U)] = U
    _load().orc_equilibrium(dim, float(rho), _d(u), _d(out))
    return out


def guo_source(dim, tau, U, F):
    Q = 9 if dim == 2 else 19
    out = np.zeros(Q)
    u = np.zeros(3)
    u[:len(U)] = U
    fv = np.zeros(3)
    fv[:len(F)] = F
    _load().orc_guo_source(dim, float(tau), _d(u), _d(fv), _d(out))
    return out


def rest_populations(dim, nx, ny, nz=1):
    """f_i = w_i everywhere: density one, fluid at rest."""
    _, w = lattice(dim)
    return np.ascontiguousarray(np.broadcast_to(w[:, None, None, None],
                                                (len(w), nz, ny, nx)).astype(np.float64))


def lb_step(dim, nx, ny, nz, bc, tau, f, F=None, tau_cell=None):
    """One pull-form LB step (eq. LBE).  tau_cell (nz, ny, nx), if given, is
    the relaxation time of every cell.  Returns (f_new, rho, U)."""
    lib = _load()
    Q = 9 if dim == 2 else 19
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(Q, nz, ny, nx)
    out = np.empty_like(f)
    rho = np.empty((nz, ny, nx))
    U = np.empty((3, nz, ny, nx))
    Fa = None if F is None else np.ascontiguousarray(F, dtype=np.float64).reshape(3, nz, ny, nx)
    tc = None if tau_cell is None else np.ascontiguousarray(tau_cell, dtype=np.float64).reshape(nz, ny, nx)
    lib.orc_lb_step(dim, nx, ny, nz, _i(_bc(bc)), float(tau), _d(tc), _d(f), _d(Fa), _d(out),
                    _d(rho), _d(U))
    return out, rho, U


# --------------------------------------------------------------------------
# delta kernel, spreading, interpolation
# --------------------------------------------------------------------------

def psi(x):
    lib = _load()
    xs = np.atleast_1d(np.asarray(x, dtype=np.float64))
    return np.array([lib.orc_psi(float(v)) for v in xs.ravel()]).reshape(xs.shape)


def spread(dim, nx, ny, nz, bc, q, phi):
    """eq. (force_spread).  q, phi: (N, dim).  Returns (F (3,nz,ny,nx), dropped (3,))."""
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).T)
    ph = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).T)
    F = np.zeros((3, nz, ny, nx))
    dropped = np.zeros(3)
    _load().orc_spread(dim, nx, ny, nz, _i(_bc(bc)), q.shape[1], _d(q), _d(ph), _d(F),
                       _d(dropped))
    return F, dropped


def interp(dim, nx, ny, nz, bc, U, q):
    """eq. (vel_interpolation).  U: (3,nz,ny,nx); q: (N, dim).  Returns (N, dim)."""
    qa = np.ascontiguousarray(np.asarray(q, dtype=np.float64).T)
    Ua = np.ascontiguousarray(U, dtype=np.float64).reshape(3, nz, ny, nx)
    out = np.zeros_like(qa)
    _load().orc_interp(dim, nx, ny, nz, _i(_bc(bc)), _d(Ua), qa.shape[1], _d(qa), _d(out))
    return out.T.copy()


# --------------------------------------------------------------------------
# interface forces
# --------------------------------------------------------------------------

def wetting_strength(sigma, theta_rad, xi, n=6, m=3):
    """eq. (A_choice)."""
    return _load().orc_wetting_strength(float(sigma), float(theta_rad), float(xi), n, m)


def Pi(h, A, xi, n=6, m=3):
    """eq. (disjoin-p)."""
    lib = _load()
    hs = np.atleast_1d(np.asarray(h, dtype=np.float64))
    return np.array([lib.orc_pi(float(v), A, xi, n, m) for v in hs.ravel()]).reshape(hs.shape)


def forces_2d(q, sigma, A, xi, n=6, m=3, wetting=True):
    """Nodal forces of a closed CCW polygon.  Returns (phi (N,2), normals (N,2))."""
    qa = np.ascontiguousarray(np.asarray(q, dtype=np.float64).T)
    N = qa.shape[1]
    phi = np.zeros_like(qa)
    nrm = np.zeros_like(qa)
    _load().orc_forces_2d(N, _d(qa), float(sigma), float(A), float(xi), n, m, int(wetting),
                          _d(phi), _d(nrm))
    return phi.T.copy(), nrm.T.copy()


def forces_3d(q, tris, sigma, A, xi, n=6, m=3, wetting=True, mu_s=0.0, qref=None):
    """Nodal forces of a closed triangle mesh.  With mu_s != 0 the interface
    is elastic, its shear part measured from the reference positions qref
    (N, 3).  Returns (phi (N,3), normals (N,3))."""
    qa = np.ascontiguousarray(np.asarray(q, dtype=np.float64).T)
    T = np.ascontiguousarray(tris, dtype=np.int32)
    N = qa.shape[1]
    phi = np.zeros_like(qa)
    nrm = np.zeros_like(qa)
    if mu_s == 0.0:
        _load().orc_forces_3d(N, _d(qa), T.shape[0], _i(T), float(sigma), float(A), float(xi),
                              n, m, int(wetting), _d(phi), _d(nrm))
    else:
        ra = np.ascontiguousarray(np.asarray(qref, dtype=np.float64).T)
        _load().orc_forces_3d_elastic(N, _d(qa), _d(ra), T.shape[0], _i(T), float(sigma),
                                      float(mu_s), float(A), float(xi), n, m, int(wetting),
                                      _d(phi), _d(nrm))
    return phi.T.copy(), nrm.T.copy()


# --------------------------------------------------------------------------
# two viscosities (Sec. IB-LB, last paragraph; eq. def_lambda)
# --------------------------------------------------------------------------

def tau_inside(tau_out, lam):
    """Relaxation time inside the droplet for viscosity ratio lam:
    mu = rho cs^2 (tau - 1/2) on both sides and lam = mu_in / mu_out (eq.
    def_lambda), so tau_in - 1/2 = lam (tau_out - 1/2)."""
    return 0.5 + lam * (tau_out - 0.5)


def reference_point(q0):
    """Centre of the classification window of a droplet: the mean of its
    node positions (N, dim) as first set, padded to three components."""
    r = np.zeros(3)
    q0 = np.asarray(q0, dtype=np.float64)
    r[:q0.shape[1]] = q0.mean(axis=0)
    return r


def inside_mask(params, q, tris=None, ref=None):
    """(nz, ny, nx) int array: 1 where the cell centre is enclosed by the
    interface (winding number, see orc_inside), 0 elsewhere.  ref: window
    centre (default: mean of q)."""
    p = params
    dim = p.dim
    nz = p.nz if dim == 3 else 1
    qa = np.ascontiguousarray(np.asarray(q, dtype=np.float64).T)
    T = (np.zeros((0, 3), dtype=np.int32) if tris is None
         else np.ascontiguousarray(tris, dtype=np.int32))
    r = reference_point(q) if ref is None else np.ascontiguousarray(ref, dtype=np.float64)
    out = np.zeros((nz, p.ny, p.nx), dtype=np.int32)
    _load().orc_inside(dim, p.nx, p.ny, nz, _i(_bc(p.bc)), qa.shape[1], _d(qa), T.shape[0],
                       _i(T), _d(r), _i(out))
    return out


def inside_cells(params, q, cells, tris=None, ref=None):
    """inside_mask at the listed flat cell indices ([z][y][x] order) only."""
    p = params
    dim = p.dim
    nz = p.nz if dim == 3 else 1
    qa = np.ascontiguousarray(np.asarray(q, dtype=np.float64).T)
    T = (np.zeros((0, 3), dtype=np.int32) if tris is None
         else np.ascontiguousarray(tris, dtype=np.int32))
    r = reference_point(q) if ref is None else np.ascontiguousarray(ref, dtype=np.float64)
    cl = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros(cl.shape[0], dtype=np.int32)
    _load().orc_inside_cells(dim, p.nx, p.ny, nz, _i(_bc(p.bc)), qa.shape[1], _d(qa), T.shape[0],
                             _i(T), _d(r), cl.shape[0],
                             cl.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _i(out))
    return out


# --------------------------------------------------------------------------
# time loop
# --------------------------------------------------------------------------

def respace_2d(q, beta):
    """Tangential re-spacing displacement of the closed 2D outline q (N, 2):
    node j moves by beta/2 (l_j+ - l_j-) along the unit chord of its two
    neighbours (l_j-, l_j+: lengths of its two edges).  An addition to the
    method for long runs, not part of the paper: a line tension has no
    tangential stiffness, so nodes carried by the fluid drift along the
    outline, and this keeps their spacing even."""
    lib = _load()
    q = np.asarray(q, dtype=np.float64)
    N = q.shape[0]
    qa = np.ascontiguousarray(q.T).copy()
    dq = np.zeros((2, N))
    lib.orc_respace_2d(N, _d(qa), float(beta), _d(dq))
    return dq.T.copy()


def run(params, q0, nsteps, tris=None, f0=None, F_fixed=None):
    """Run `nsteps` of the coupled method from post-collision populations f0
    (default: fluid at rest, density one) and nodes q0 (N, dim; N may be 0
    for the fluid alone, optionally driven by F_fixed (3,nz,ny,nx)).

    `params` is any object with attributes dim, nx, ny, nz, bc, tau, sigma,
    theta_eq_deg, xi, n_exp, m_exp, wetting, and optionally lam (viscosity
    ratio, default 1; the classification window is centred on the mean of
    q0), shear (surface shear modulus of an elastic interface, 3D,
    default 0; the reference mesh is q0) and respace (rate beta of the
    tangential re-spacing of a 2D outline, respace_2d; default 0).  Returns a dict with the final f, q, and the last step's rho, U, F,
    phi, qdot, dropped, status."""
    p = params
    lib = _load()
    dim = p.dim
    nz = p.nz if dim == 3 else 1
    Q = 9 if dim == 2 else 19
    f = (rest_populations(dim, p.nx, p.ny, nz) if f0 is None
         else np.ascontiguousarray(f0, dtype=np.float64).reshape(Q, nz, p.ny, p.nx).copy())
    q0 = np.zeros((0, dim)) if q0 is None else np.asarray(q0, dtype=np.float64)
    N = q0.shape[0]
    q = np.ascontiguousarray(q0.T).copy()
    T = (np.zeros((0, 3), dtype=np.int32) if tris is None
         else np.ascontiguousarray(tris, dtype=np.int32))
    rho = np.zeros((nz, p.ny, p.nx))
    U = np.zeros((3, nz, p.ny, p.nx))
    F = np.zeros((3, nz, p.ny, p.nx))
    Ff = None if F_fixed is None else np.ascontiguousarray(F_fixed, dtype=np.float64)
    phi = np.zeros((dim, max(N, 1)))
    qdot = np.zeros((dim, max(N, 1)))
    dropped = np.zeros(3)
    qa = q if N > 0 else np.zeros((dim, 1))
    lam = float(getattr(p, "lam", 1.0))
    tau_in = tau_inside(float(p.tau), lam) if lam != 1.0 else float(p.tau)
    ref = reference_point(q0) if N > 0 else np.zeros(3)
    mu_s = float(getattr(p, "shear", 0.0))
    qref = q.copy() if N > 0 else np.zeros((dim, 1))
    status = lib.orc_run(dim, p.nx, p.ny, nz, _i(_bc(p.bc)), float(p.tau), tau_in, _d(ref),
                         float(p.sigma), mu_s, _d(qref), math.radians(p.theta_eq_deg), float(p.xi),
                         int(p.n_exp), int(p.m_exp), int(bool(p.wetting)),
                         float(getattr(p, "respace", 0.0)),
                         N, _d(qa), T.shape[0], _i(T), int(nsteps),
                         _d(f), _d(rho), _d(U), _d(F), _d(Ff), _d(phi), _d(qdot), _d(dropped))
    return dict(f=f, q=qa.T[:N].copy(), rho=rho, U=U, F=F, phi=phi.T[:N].copy(),
                qdot=qdot.T[:N].copy(), dropped=dropped, status=status)


# --------------------------------------------------------------------------
# FP64 diagnostics (numpy, plain definitions)
# --------------------------------------------------------------------------

def h_star(xi, n=6, m=3):
    """Height of the minimum of Pi(h): xi (n/m)^(1/(n-m)) (Sec. Dynamics)."""
    return xi * (n / m) ** (1.0 / (n - m))


def volume_2d(q):
    """Area enclosed by the CCW polygon (shoelace formula)."""
    x, y = q[:, 0], q[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def volume_3d(q, tris):
    """Enclosed volume (divergence theorem over the outward-oriented mesh)."""
    a, b, c = q[tris[:, 0]], q[tris[:, 1]], q[tris[:, 2]]
    return float(np.sum(np.einsum('ij,ij->i', a, np.cross(b, c)))) / 6.0


def area_3d(q, tris):
    a, b, c = q[tris[:, 0]], q[tris[:, 1]], q[tris[:, 2]]
    return 0.5 * float(np.sum(np.linalg.norm(np.cross(b - a, c - a), axis=1)))


def perimeter_2d(q):
    return float(np.sum(np.linalg.norm(np.roll(q, -1, axis=0) - q, axis=1)))


def contact_radius_2d(q, zcut):
    """Protocol (i) in 2D: crossings of the outline with the line y = zcut;
    half the distance between the outermost crossings (nan if fewer than
    two)."""
    y = q[:, 1] - zcut
    yn = np.roll(y, -1)
    qn = np.roll(q, -1, axis=0)
    cross = (y * yn < 0) | ((y == 0) & (yn != 0))
    if np.count_nonzero(cross) < 2:
        return float('nan')
    t = y[cross] / (y[cross] - yn[cross])
    xs = q[cross, 0] + t * (qn[cross, 0] - q[cross, 0])
    return 0.5 * float(xs.max() - xs.min())


def contact_radius_3d(q, tris, zcut):
    """Protocol (i): points where mesh edges cross the plane z = zcut; mean
    distance of those points to their centre."""
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    za, zb = q[e[:, 0], 2] - zcut, q[e[:, 1], 2] - zcut
    sel = za * zb < 0
    if not np.any(sel):
        return float('nan')
    t = za[sel] / (za[sel] - zb[sel])
    p = q[e[sel, 0]] + t[:, None] * (q[e[sel, 1]] - q[e[sel, 0]])
    c = p[:, :2].mean(axis=0)
    return float(np.mean(np.linalg.norm(p[:, :2] - c, axis=1)))


def contact_radius_flat_3d(q, tris, tol):
    """Protocol (ii) of Sec. Dynamics: the triangles of the lower half of the
    droplet (all three vertices below the mid-height between the lowest and
    the highest vertex) whose vertices differ in height by less than tol
    (= eps R0) form the flat region; its area chi is taken as a circle's,
    r = sqrt(chi / pi)."""
    z = q[:, 2]
    mid = 0.5 * (z.min() + z.max())
    a, b, c = q[tris[:, 0]], q[tris[:, 1]], q[tris[:, 2]]
    zt = z[tris]
    lower = np.all(zt < mid, axis=1)
    flat = (zt.max(axis=1) - zt.min(axis=1)) < tol
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    chi = float(np.sum(area[lower & flat]))
    return math.sqrt(chi / math.pi)


def contact_radius_flat_2d(q, tol):
    """2D counterpart of protocol (ii): the edges of the lower half whose end
    points differ in height by less than tol; half their total length."""
    y = q[:, 1]
    mid = 0.5 * (y.min() + y.max())
    yn = np.roll(y, -1)
    sel = (y < mid) & (yn < mid) & (np.abs(yn - y) < tol)
    length = np.linalg.norm(np.roll(q, -1, axis=0) - q, axis=1)
    return 0.5 * float(np.sum(length[sel]))


def angle_from_height_3d(ell, volume):
    """eq. (angleh): tan^2(theta/2) = 3 l^3 / (R0^3 - l^3), R0 the radius of
    the sphere of equal volume, l the half-height."""
    R0 = (3.0 * volume / (4.0 * math.pi)) ** (1.0 / 3.0)
    if ell >= R0:
        return math.pi
    return 2.0 * math.atan(math.sqrt(3.0 * ell ** 3 / (R0 ** 3 - ell ** 3)))


def angle_from_height_2d(ell, area):
    """2D counterpart of eq. (angleh): a circular cap of angle theta and
    circle radius Rc has area Rc^2 (theta - sin theta cos theta) and
    half-height l = Rc sin^2(theta/2) (eq. ell), so
    area / l^2 = (theta - sin theta cos theta) / sin^4(theta/2), a decreasing
    function of theta on (0, pi); solved by bisection."""
    target = area / ell ** 2

    def g(th):
        return (th - math.sin(th) * math.cos(th)) / math.sin(0.5 * th) ** 4

    lo, hi = 1e-6, math.pi
    if target <= g(hi):
        return math.pi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def diagnostics(dim, q, qdot, normals, f, phi, F, dropped, xi, tris=None, n=6, m=3):
    """FP64 diagnostics of one state: mass, force balance, volume, contact
    radius at z_cut = h*, measured angle from the half-height, largest
    normal node speed, min height, edge lengths."""
    d = {}
    d["mass"] = float(np.sum(f))
    d["sum_phi"] = phi.sum(axis=0)
    d["sum_F"] = F[:dim].reshape(dim, -1).sum(axis=1)
    d["dropped_F"] = np.asarray(dropped)[:dim]
    hh = q[:, dim - 1]
    d["min_h"] = float(hh.min())
    ell = 0.5 * float(hh.max() - hh.min())
    d["height"] = 2.0 * ell
    zc = h_star(xi, n, m)
    if dim == 2:
        vol = volume_2d(q)
        d["volume"] = vol
        d["contact_radius"] = contact_radius_2d(q, zc)
        d["theta_meas"] = angle_from_height_2d(ell, vol)
        el = np.linalg.norm(np.roll(q, -1, axis=0) - q, axis=1)
    else:
        vol = volume_3d(q, tris)
        d["volume"] = vol
        d["contact_radius"] = contact_radius_3d(q, tris, zc)
        d["theta_meas"] = angle_from_height_3d(ell, vol)
        e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
        el = np.linalg.norm(q[e[:, 1]] - q[e[:, 0]], axis=1)
    d["edge_min"] = float(el.min())
    d["edge_max"] = float(el.max())
    d["max_normal_speed"] = float(np.max(np.abs(np.sum(qdot * normals, axis=1))))
    return d
