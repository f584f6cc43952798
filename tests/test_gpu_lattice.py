"""GPU parity of the fused lattice kernel against the FP64 oracle, through
the C ABI: pure streaming bit-exact for every storage format, box shape and
boundary mix; collide + Guo source with a prescribed force field within the
fp32 tolerance; closed-form Poiseuille flow."""
import math

import numpy as np
import pytest

import oracle as o
import workloads as wl
from helpers import compare_fields, gpu_run, oracle_dev, weights

pytestmark = pytest.mark.gpu

STREAM_CASES = [
    # dim, (nx, ny, nz), bc
    (2, (37, 23, 1), (0, 1, 0)),       # ragged: partial wavefronts, x wraps
    (2, (64, 8, 1), (0, 0, 0)),        # fully periodic
    (2, (300, 5, 1), (1, 1, 0)),       # walls on both axes, > one 256 tile
    (2, (1, 7, 1), (0, 1, 0)),         # one-cell-wide periodic axis
    (3, (19, 6, 5), (0, 0, 1)),
    (3, (70, 3, 4), (1, 0, 1)),
]


@pytest.mark.parametrize("storage", [0, 1, 2], ids=["f32", "f16", "bf16"])
@pytest.mark.parametrize("dim,shape,bc", STREAM_CASES)
@pytest.mark.parametrize("tile", [0, 2, 3, 4, 6, 8, 10, 11, 12, 13, 14, 15, 16, 25, 31])
def test_pure_streaming_bit_exact(dim, shape, bc, storage, tile):
    nx, ny, nz = shape
    Q = 9 if dim == 2 else 19
    w = weights(dim)
    p = wl.Params(dim=dim, nx=nx, ny=ny, nz=nz, bc=bc, tau=math.inf, wetting=False)
    for seed, steps in ((21, 1), (22, 3), (23, 9)):
        dev = wl.tagged_deviation(Q, nx * ny * nz, seed).reshape(Q, nz, ny, nx)
        print(f"[stream] dim={dim} shape={shape} bc={bc} storage={storage} tile={tile} "
              f"steps={steps}", flush=True)
        g = gpu_run(p, None, steps, storage=storage, f0dev=dev, shape=tile, graph_steps=2)
        f = w[:, None, None, None] + dev
        for _ in range(steps):
            f, _, _ = o.lb_step(dim, nx, ny, nz, bc, math.inf, f, None)
        k = np.rint((f - w[:, None, None, None]) * 1024.0)
        assert np.array_equal(g["fdev"], k / 1024.0)


@pytest.mark.parametrize("dim,shape,bc", [
    (2, (45, 17, 1), (0, 1, 0)),
    (2, (128, 64, 1), (0, 1, 0)),
    (3, (21, 10, 9), (0, 0, 1)),
])
@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_collide_with_force_field_matches_oracle(dim, shape, bc, tau):
    nx, ny, nz = shape
    Q = 9 if dim == 2 else 19
    w = weights(dim)
    rng = np.random.default_rng(31)
    dev = 1e-2 * w[:, None, None, None] * rng.standard_normal((Q, nz, ny, nx))
    F = np.zeros((3, nz, ny, nx))
    F[:dim] = 1e-4 * rng.standard_normal((dim, nz, ny, nx))
    p = wl.Params(dim=dim, nx=nx, ny=ny, nz=nz, bc=bc, tau=tau, wetting=False)
    for steps in (1, 40):
        print(f"[collide] dim={dim} shape={shape} tau={tau} steps={steps}", flush=True)
        g = gpu_run(p, None, steps, f0dev=dev, F_fixed=F, graph_steps=8)
        r = o.run(p, None, steps, f0=w[:, None, None, None] + dev, F_fixed=F)
        drho, du, _ = compare_fields(g, r, dim, f"collide{steps}")
        assert drho <= 1e-6
        assert du <= 1e-5
        assert np.max(np.abs(g["fdev"] - oracle_dev(dim, r["f"]))) <= 1e-7
        assert np.array_equal(g["F"], F[:dim].astype(np.float32).astype(np.float64))


def test_poiseuille_on_gpu():
    nx, ny = 64, 12
    tau = 0.5 + math.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3.0
    g0 = 1e-6
    F = np.zeros((3, 1, ny, nx))
    F[0] = g0
    p = wl.Params(dim=2, nx=nx, ny=ny, bc=(0, 1, 0), tau=tau, wetting=False)
    g = gpu_run(p, None, 6000, F_fixed=F)
    y = np.arange(ny) + 0.5
    want = g0 * y * (ny - y) / (2 * nu)
    got = g["U"][0, 0, :, :]
    err = np.max(np.abs(got - want[:, None])) / want.max()
    print(f"[poiseuille] rel err {err:.3e}", flush=True)
    assert err < 1e-5


def test_rest_state_stays_at_rest_and_mass_exact():
    p = wl.Params(dim=2, nx=96, ny=40, bc=(0, 1, 0), tau=0.9, wetting=False)
    g = gpu_run(p, None, 100)
    assert np.all(g["fdev"] == 0.0)
    assert np.all(g["rho"] == 1.0) and np.all(g["U"] == 0.0)
    d = g["solver"].diagnostics(0)
    assert d["mass"] == 96 * 40


@pytest.mark.parametrize("dim,shape", [(2, (45, 17, 1)), (3, (13, 9, 6))])
@pytest.mark.parametrize("storage", [0, 1, 2], ids=["f32", "f16", "bf16"])
def test_init_fields_is_the_equilibrium(dim, shape, storage):
    """iblb_init_fields against the oracle's equilibrium cell by cell, for a
    random density and velocity field; within one rounding of the storage
    format (relative to the largest deviation)."""
    from helpers import gpu_solver
    nx, ny, nz = shape
    rng = np.random.default_rng(40 + dim)
    rho = (1.0 + 1e-3 * rng.standard_normal((nz, ny, nx))).astype(np.float32)
    U = (1e-2 * rng.standard_normal((dim, nz, ny, nx))).astype(np.float32)
    p = wl.Params(dim=dim, nx=nx, ny=ny, nz=nz, tau=0.8, wetting=False)
    s = gpu_solver([p], storage=storage)
    s.init_fields(0, rho, U)
    got = s.read_populations(0).cpu().numpy()
    w = weights(dim)
    want = np.empty_like(got)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                want[:, z, y, x] = o.equilibrium(dim, float(rho[z, y, x]), U[:, z, y, x].astype(np.float64)) - w
    u = {0: 2.0 ** -23, 1: 2.0 ** -10, 2: 2.0 ** -7}[storage]
    assert np.max(np.abs(got - want)) <= 4 * u * np.max(np.abs(want))
    # null fields: the rest state
    s.init_fields(0)
    assert np.max(np.abs(s.read_populations(0).cpu().numpy())) == 0.0

