"""MI355X-native immersed-boundary lattice Boltzmann wetting solver.

The compute path is the HIP library libiblb.so (C ABI in include/iblb.h).
This package only marshals arguments: PyTorch provides the device
workspace and the stream, numpy holds host-side node arrays.

    from paper_2503_20605_amd import Solver, make_params
    p = make_params(dim=2, nx=128, ny=64, tau=1.0, sigma=0.01,
                    theta_eq_deg=60.0, xi=2.0)
    s = Solver([p], [nodes])          # nodes: (N, 2) float64, CCW polygon
    s.step(1000)
    rho, U, F = s.read_fields(0)
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _lib
from ._lib import (IBLB_BF16, IBLB_F16, IBLB_F32, IBLB_PERIODIC, IBLB_WALL, IblbError,
                   iblb_diag, iblb_params)

__all__ = ["Solver", "MLP", "make_params", "IblbError", "IBLB_F32", "IBLB_F16", "IBLB_BF16",
           "IBLB_PERIODIC", "IBLB_WALL", "STORAGE", "probe_copy_bandwidth"]

STORAGE = {"f32": IBLB_F32, "f16": IBLB_F16, "bf16": IBLB_BF16}
# lattice-kernel variants: 16 kernel forms, each in two block orders
LB_VARIANTS = 32


def make_params(dim=2, nx=128, ny=64, nz=1, bc=None, tau=1.0, sigma=0.01, theta_eq_deg=90.0,
                xi=2.0, n_exp=6, m_exp=3, wetting=True) -> iblb_params:
    """Build an iblb_params record (angle given in degrees)."""
    if bc is None:
        bc = (IBLB_PERIODIC, IBLB_WALL, IBLB_PERIODIC) if dim == 2 else \
             (IBLB_PERIODIC, IBLB_PERIODIC, IBLB_WALL)
    p = iblb_params()
    p.dim, p.nx, p.ny, p.nz = dim, nx, ny, (nz if dim == 3 else 1)
    for a in range(3):
        p.bc[a] = int(bc[a])
    p.tau, p.sigma = float(tau), float(sigma)
    p.theta_eq = math.radians(theta_eq_deg)
    p.xi, p.n_exp, p.m_exp, p.wetting = float(xi), int(n_exp), int(m_exp), int(bool(wetting))
    return p


def params_from(obj) -> iblb_params:
    """iblb_params from any object with the attributes of make_params."""
    return make_params(dim=obj.dim, nx=obj.nx, ny=obj.ny, nz=getattr(obj, "nz", 1),
                       bc=obj.bc, tau=obj.tau, sigma=obj.sigma,
                       theta_eq_deg=obj.theta_eq_deg, xi=obj.xi, n_exp=obj.n_exp,
                       m_exp=obj.m_exp, wetting=obj.wetting)


def probe_copy_bandwidth(nbytes=1 << 30, reps=20, device="cuda"):
    """Attainable device copy bandwidth (GB/s, read + write) on buffers of
    nbytes each."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device=device)
    dst = torch.empty_like(src)
    src.fill_(1)
    out = ctypes.c_double()
    stream = torch.cuda.current_stream(src.device)
    _lib.check(_lib.load().iblb_probe_copy(ctypes.c_void_p(dst.data_ptr()),
                                           ctypes.c_void_p(src.data_ptr()), nbytes, reps,
                                           ctypes.c_void_p(stream.cuda_stream), ctypes.byref(out)))
    return out.value


class Solver:
    """One handle on a batch of droplets.

    params: list of iblb_params; nodes: list of (N, dim) float64 arrays (or
    None for a fluid-only droplet); tris: list of (T, 3) int32 arrays in 3D.
    The device workspace is one torch uint8 tensor; every call runs on
    `stream` (default: torch's current stream)."""

    def __init__(self, params, nodes, tris=None, storage=IBLB_F32, device="cuda", stream=None):
        import torch
        self._torch = torch
        lib = _lib.load()
        self.lib = lib
        n = len(params)
        self.n = n
        self.dim = params[0].dim
        self.Q = 9 if self.dim == 2 else 19
        self.params = list(params)
        self.storage = storage
        self.device = torch.device(device)
        nodes = [None] * n if nodes is None else list(nodes)
        tris = [None] * n if tris is None else list(tris)
        self.n_nodes = [0 if q is None else int(np.asarray(q).shape[0]) for q in nodes]
        self.n_tris = [0 if t is None else int(np.asarray(t).shape[0]) for t in tris]
        P = (iblb_params * n)(*params)
        NN = (ctypes.c_int * n)(*self.n_nodes)
        NT = (ctypes.c_int * n)(*self.n_tris)
        self._P, self._NN, self._NT = P, NN, NT
        nbytes = lib.iblb_workspace_bytes(n, P, NN, NT, storage)
        if nbytes == 0:
            # let create() produce the message
            nbytes = 256
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        ctx = ctypes.c_void_p()
        code = lib.iblb_create(n, P, NN, NT, storage, ctypes.c_void_p(self.ws.data_ptr()),
                               ctypes.c_size_t(nbytes), ctypes.c_void_p(self.stream.cuda_stream),
                               ctypes.byref(ctx))
        _lib.check(code, None)
        self.ctx = ctx
        for d in range(n):
            if nodes[d] is not None and self.n_nodes[d] > 0:
                self.set_interface(d, nodes[d], tris[d])

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            self.lib.iblb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, code):
        return _lib.check(code, self.ctx)

    # -- set-up ------------------------------------------------------------
    def set_interface(self, d, q, tris=None):
        q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).T)
        t = None if tris is None else np.ascontiguousarray(np.asarray(tris, dtype=np.int32))
        self._chk(self.lib.iblb_set_interface(
            self.ctx, d, q.ctypes.data_as(ctypes.c_void_p),
            None if t is None else t.ctypes.data_as(ctypes.c_void_p)))

    def init_rest(self, d=-1):
        self._chk(self.lib.iblb_init_rest(self.ctx, d))

    def cells(self, d):
        p = self.params[d]
        return (p.nz if self.dim == 3 else 1, p.ny, p.nx)

    def init_fields(self, d, rho=None, U=None):
        """Equilibrium populations of droplet d from a density field
        (nz, ny, nx) and a velocity field (dim, nz, ny, nx); None means 1 and
        at rest."""
        torch = self._torch
        sh = self.cells(d)

        def dev(a, shape):
            if a is None:
                return None
            t = torch.as_tensor(np.asarray(a) if not torch.is_tensor(a) else a)
            t = t.to(device=self.device, dtype=torch.float32).contiguous()
            assert tuple(t.shape) == shape, (tuple(t.shape), shape)
            return t

        r = dev(rho, sh)
        u = dev(U, (self.dim,) + sh)
        self._chk(self.lib.iblb_init_fields(self.ctx, d, None if r is None else ctypes.c_void_p(r.data_ptr()),
                                            None if u is None else ctypes.c_void_p(u.data_ptr())))
        self.stream.synchronize()  # the kernel has read r and u

    def write_populations(self, d, fdev):
        """fdev: deviations f - w, shape (Q, nz, ny, nx), any float dtype."""
        t = self._torch.as_tensor(np.asarray(fdev) if not self._torch.is_tensor(fdev) else fdev)
        t = t.to(device=self.device, dtype=self._torch.float64).contiguous()
        assert t.numel() == self.Q * int(np.prod(self.cells(d)))
        self._chk(self.lib.iblb_write_populations(self.ctx, d, ctypes.c_void_p(t.data_ptr())))
        self.stream.synchronize()

    def read_populations(self, d):
        """Deviations f - w of the current post-collision populations."""
        t = self._torch.empty((self.Q,) + self.cells(d), dtype=self._torch.float64,
                              device=self.device)
        self._chk(self.lib.iblb_read_populations(self.ctx, d, ctypes.c_void_p(t.data_ptr())))
        self.stream.synchronize()
        return t

    def set_force_field(self, d, F):
        if F is None:
            self._chk(self.lib.iblb_set_force_field(self.ctx, d, None))
            return
        t = self._torch.as_tensor(F).to(device=self.device, dtype=self._torch.float32)
        t = t[: self.dim].contiguous()
        self._chk(self.lib.iblb_set_force_field(self.ctx, d, ctypes.c_void_p(t.data_ptr())))
        self.stream.synchronize()

    # -- stepping ----------------------------------------------------------
    def step(self, n):
        self._chk(self.lib.iblb_step(self.ctx, int(n)))

    def set_lb_variant(self, variant):
        out = ctypes.c_int()
        self._chk(self.lib.iblb_set_lb_variant(self.ctx, int(variant), ctypes.byref(out)))
        return out.value

    def autotune(self, steps=130, cache_path=None):
        """Time the 32 lattice-kernel variants on the handle's own coupled
        steps and keep the fastest; returns (variant, per-variant ms per
        coupled step, or -1 on a cache hit).  The default runs the step graph
        (64 steps unless set otherwise) twice per timing; every step taken
        here advances the simulation."""
        out = ctypes.c_int()
        ms = (ctypes.c_double * LB_VARIANTS)()
        cp = None if cache_path is None else str(cache_path).encode()
        self._chk(self.lib.iblb_autotune(self.ctx, int(steps), cp, ctypes.byref(out), ms))
        return out.value, list(ms)

    def run_to_rest(self, tol=1e-6, check_every=100, hold=10, max_steps=200000, angle_tol_deg=0.0):
        """Step until every droplet's interface is at rest (see iblb.h):
        normal node speed below tol for `hold` checks and, with
        angle_tol_deg > 0, the measured angle steady within it over those
        checks.  Returns the per-droplet step counts (-1 still moving,
        -2 unstable)."""
        out = (ctypes.c_longlong * self.n)()
        self._chk(self.lib.iblb_run_to_rest(self.ctx, float(tol), math.radians(float(angle_tol_deg)),
                                            int(check_every), int(hold), int(max_steps), out))
        return list(out)

    def set_graph_steps(self, k):
        self._chk(self.lib.iblb_set_graph_steps(self.ctx, int(k)))

    def set_active(self, d, on):
        self._chk(self.lib.iblb_set_active(self.ctx, d, int(bool(on))))

    def set_viscosity_ratio(self, d, lam):
        """Viscosity ratio mu_in / mu_out of droplet d (1: one fluid)."""
        self._chk(self.lib.iblb_set_viscosity_ratio(self.ctx, d, float(lam)))

    def inside_mask(self, d):
        """uint8 device tensor (nz, ny, nx): 1 for the cells of droplet d
        enclosed by its interface at the current node positions."""
        m = self._torch.empty(self.cells(d), dtype=self._torch.uint8, device=self.device)
        self.stream.synchronize()
        self._chk(self.lib.iblb_inside_mask(self.ctx, d, ctypes.c_void_p(m.data_ptr())))
        return m

    def set_membrane_shear(self, d, mu_s):
        """Elastic interface of droplet d with surface shear modulus mu_s,
        stress-free at its current node positions (3D; 0: liquid)."""
        self._chk(self.lib.iblb_set_membrane_shear(self.ctx, d, float(mu_s)))

    def set_node_respacing(self, d, beta):
        """Tangential re-spacing of droplet d's outline at rate beta (2D;
        0: off)."""
        self._chk(self.lib.iblb_set_node_respacing(self.ctx, d, float(beta)))

    def contact_radius(self, d, z_cut, flat_tol):
        """(protocol (i) radius at z_cut, protocol (ii) radius with flatness
        tolerance flat_tol, number of protocol (i) crossings) of droplet d."""
        out = (ctypes.c_double * 3)()
        self._chk(self.lib.iblb_contact_radius(self.ctx, d, float(z_cut), float(flat_tol), out))
        return out[0], out[1], int(out[2])

    def set_timing(self, on):
        """False / 0: off; True / 1: time every lattice launch; n > 1: every
        n-th one (see iblb_set_timing)."""
        self._chk(self.lib.iblb_set_timing(self.ctx, int(on)))

    def last_timing(self):
        """(lattice-kernel duration from events marked by its dispatch, whole
        step), milliseconds, averaged over the last timed step() call."""
        a, b = ctypes.c_double(), ctypes.c_double()
        self._chk(self.lib.iblb_last_timing(self.ctx, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def time_lattice(self, launches=256):
        """Per-launch time (ms) of the lattice kernel replayed back to back
        in a graph (dispatch included).  Advances the populations without
        moving the nodes: a measurement aid, not a simulation step."""
        out = ctypes.c_double()
        self._chk(self.lib.iblb_time_lattice(self.ctx, int(launches), ctypes.byref(out)))
        return out.value

    # -- outputs -----------------------------------------------------------
    def read_fields(self, d):
        torch = self._torch
        sh = self.cells(d)
        rho = torch.empty(sh, dtype=torch.float32, device=self.device)
        U = torch.empty((self.dim,) + sh, dtype=torch.float32, device=self.device)
        F = torch.empty((self.dim,) + sh, dtype=torch.float32, device=self.device)
        self._chk(self.lib.iblb_read_fields(self.ctx, d, ctypes.c_void_p(rho.data_ptr()),
                                            ctypes.c_void_p(U.data_ptr()),
                                            ctypes.c_void_p(F.data_ptr())))
        self.stream.synchronize()
        return rho, U, F

    def read_nodes(self, d):
        N = self.n_nodes[d]
        pos = np.zeros((self.dim, N), dtype=np.float64)
        vel = np.zeros((self.dim, N), dtype=np.float32)
        frc = np.zeros((self.dim, N), dtype=np.float32)
        self._chk(self.lib.iblb_read_nodes(self.ctx, d, pos.ctypes.data_as(ctypes.c_void_p),
                                           vel.ctypes.data_as(ctypes.c_void_p),
                                           frc.ctypes.data_as(ctypes.c_void_p)))
        return pos.T.copy(), vel.T.copy(), frc.T.copy()

    def diagnostics(self, d=0):
        if d == -1:
            arr = (iblb_diag * self.n)()
            self._chk(self.lib.iblb_diagnostics(self.ctx, -1, arr))
            return [a.to_dict(self.dim) for a in arr]
        out = iblb_diag()
        self._chk(self.lib.iblb_diagnostics(self.ctx, d, ctypes.byref(out)))
        return out.to_dict(self.dim)


class MLP:
    """Warm-start network on the device (bf16 matrix-core products, fp32
    master weights, Adam); thin wrapper of the iblb_mlp_* calls."""

    def __init__(self, widths, max_batch, device="cuda", stream=None):
        import torch
        self._torch = torch
        lib = _lib.load()
        self.lib = lib
        self.widths = list(widths)
        self.max_batch = int(max_batch)
        W = (ctypes.c_int * len(widths))(*widths)
        self._W = W
        n = lib.iblb_mlp_workspace_bytes(len(widths) - 1, W, self.max_batch)
        if n == 0:
            raise IblbError(-1, "bad network shape")
        self.device = torch.device(device)
        self.ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        h = ctypes.c_void_p()
        _lib.check_mlp(lib.iblb_mlp_create(len(widths) - 1, W, self.max_batch,
                                           ctypes.c_void_p(self.ws.data_ptr()), n,
                                           ctypes.c_void_p(self.stream.cuda_stream),
                                           ctypes.byref(h)))
        self.h = h
        self.P = lib.iblb_mlp_param_count(h)

    def close(self):
        if getattr(self, "h", None):
            self.lib.iblb_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a):
        t = self._torch.as_tensor(np.asarray(a) if not self._torch.is_tensor(a) else a)
        return t.to(device=self.device, dtype=self._torch.float32).contiguous()

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.P
        _lib.check_mlp(self.lib.iblb_mlp_set_params(self.h, p.ctypes.data_as(ctypes.c_void_p)), self.h)

    def get_params(self):
        p = np.zeros(self.P, dtype=np.float32)
        _lib.check_mlp(self.lib.iblb_mlp_get_params(self.h, p.ctypes.data_as(ctypes.c_void_p)), self.h)
        return p

    def forward(self, x):
        x = self._dev(x)
        y = self._torch.empty((x.shape[0], self.widths[-1]), dtype=self._torch.float32,
                              device=self.device)
        _lib.check_mlp(self.lib.iblb_mlp_forward(self.h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                                 ctypes.c_void_p(y.data_ptr())), self.h)
        self.stream.synchronize()
        return y

    def forward_noalloc(self, x, y):
        """iblb_mlp_forward_noalloc: x (batch, widths[0]) into the caller's
        y (batch, widths[-1]), both device fp32; the library allocates
        nothing (its activations live in a static device array)."""
        _lib.check_mlp(self.lib.iblb_mlp_forward_noalloc(self.h, ctypes.c_void_p(x.data_ptr()),
                                                         x.shape[0], ctypes.c_void_p(y.data_ptr())),
                       self.h)
        return y

    def gradients(self, x, t, want_grads=True):
        x, t = self._dev(x), self._dev(t)
        g = np.zeros(self.P, dtype=np.float32) if want_grads else None
        loss = ctypes.c_double()
        _lib.check_mlp(self.lib.iblb_mlp_gradients(
            self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()), x.shape[0],
            None if g is None else g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss)), self.h)
        return loss.value, g

    def train_step(self, x, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        loss, _ = self.gradients(x, t, want_grads=False)
        _lib.check_mlp(self.lib.iblb_mlp_adam_step(self.h, lr, beta1, beta2, eps), self.h)
        return loss
