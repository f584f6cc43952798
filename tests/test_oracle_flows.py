"""Closed-form flows that pin the oracle's LB update as a whole: the
viscosity mu = rho c_s^2 (tau - dt/2) stated after eqs. (hydro_var1)-(2),
periodic sides and bounce-back walls (Sec. "Numerical results")."""
import math

import numpy as np
import pytest

import oracle as o
import workloads as wl


def _feq_field(dim, rho, U):
    """Equilibrium populations for a velocity field U (3, nz, ny, nx)."""
    _, nz, ny, nx = U.shape
    Q = 9 if dim == 2 else 19
    f = np.empty((Q, nz, ny, nx))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                f[:, k, j, i] = o.equilibrium(dim, rho, U[:dim, k, j, i])
    return f


@pytest.mark.parametrize("tau", [0.7, 1.0])
def test_shear_wave_decays_at_nu_k2(tau):
    """u_x(y) = u0 sin(k y) decays as exp(-nu k^2 t), nu = (tau - 1/2)/3."""
    nx, ny = 2, 64
    k = 2 * math.pi / ny
    y = np.arange(ny) + 0.5
    U = np.zeros((3, 1, ny, nx))
    U[0, 0, :, :] = 1e-4 * np.sin(k * y)[:, None]
    f = _feq_field(2, 1.0, U)
    p = wl.Params(dim=2, nx=nx, ny=ny, bc=(0, 0, 0), tau=tau)
    steps = 400
    r = o.run(p, None, steps, f0=f)
    amp = 2 * np.mean(r["U"][0, 0, :, 0] * np.sin(k * y))
    # amplitude of the velocity reported at the last step (step index
    # steps-1 counted from the first pull, which already is one decay step)
    nu = (tau - 0.5) / 3.0
    want = 1e-4 * math.exp(-nu * k * k * steps)
    assert abs(amp / want - 1) < 2e-3, (amp, want)


def test_poiseuille_exact_at_magic_tau():
    """Body-force channel flow between half-way bounce-back walls at y = 0
    and y = H: u(y) = g y (H - y) / (2 nu).  For BGK this profile is
    reproduced to round-off when tau = 1/2 + sqrt(3/16) (the wall then sits
    exactly half-way), so a wrong wall position, force weight or viscosity
    shows up at once."""
    nx, ny = 2, 12
    tau = 0.5 + math.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3.0
    g = 1e-6
    F = np.zeros((3, 1, ny, nx))
    F[0] = g
    p = wl.Params(dim=2, nx=nx, ny=ny, bc=(0, 1, 0), tau=tau)
    r = o.run(p, None, 6000, F_fixed=F)
    y = np.arange(ny) + 0.5
    want = g * y * (ny - y) / (2 * nu)
    got = r["U"][0, 0, :, 0]
    assert np.max(np.abs(got - want)) / want.max() < 1e-9
    assert np.max(np.abs(r["U"][1])) < 1e-13


def test_poiseuille_other_tau_close():
    nx, ny = 2, 16
    tau = 1.0
    nu = (tau - 0.5) / 3.0
    g = 1e-6
    F = np.zeros((3, 1, ny, nx))
    F[0] = g
    p = wl.Params(dim=2, nx=nx, ny=ny, bc=(0, 1, 0), tau=tau)
    r = o.run(p, None, 8000, F_fixed=F)
    y = np.arange(ny) + 0.5
    want = g * y * (ny - y) / (2 * nu)
    got = r["U"][0, 0, :, 0]
    err = np.max(np.abs(got - want)) / want.max()
    assert 1e-6 < err < 3e-2


def test_poiseuille_3d_channel_magic_tau():
    nx, ny, nz = 2, 2, 10
    tau = 0.5 + math.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3.0
    g = 1e-6
    F = np.zeros((3, nz, ny, nx))
    F[1] = g
    p = wl.Params(dim=3, nx=nx, ny=ny, nz=nz, bc=(0, 0, 1), tau=tau)
    r = o.run(p, None, 5000, F_fixed=F)
    z = np.arange(nz) + 0.5
    want = g * z * (nz - z) / (2 * nu)
    got = r["U"][1, :, 0, 0]
    assert np.max(np.abs(got - want)) / want.max() < 1e-9
