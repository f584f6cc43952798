"""Bit-for-bit repeatability of the coupled step on the GPU.

The spread force density (eq. force_spread) is summed in fixed point with
integer atomics, so the order in which the nodes' contributions arrive
cannot change it; every other reduction of the step runs in a fixed order.
Two runs of the same input must therefore agree bit for bit: the spread
field F, the populations, the velocity field and the node positions.  The
3D cases cover both paths of the 3D spreading (chunks summed in LDS, and
chunks too spread out for their LDS box, which add straight to memory)."""
import numpy as np
import pytest

import workloads as wl
from helpers import collect, gpu_run

pytestmark = pytest.mark.gpu


def _same(a, b, dim):
    for k in ("F", "U", "rho", "fdev", "q", "qdot", "phi"):
        assert np.array_equal(a[k], b[k]), (k, float(np.max(np.abs(a[k] - b[k]))))
    assert np.any(a["F"] != 0.0)


def test_3d_runs_repeat_bit_for_bit():
    W = wl.droplet_3d(theta_eq_deg=45.0, small=True)
    print("[det] 3D 64x64x32, 2 x 150 steps", flush=True)
    a = gpu_run(W.params, W.nodes, 150, tris=W.tris, graph_steps=16)
    b = gpu_run(W.params, W.nodes, 150, tris=W.tris, graph_steps=16)
    _same(a, b, 3)


@pytest.mark.parametrize("form", [9, 13])
def test_3d_block_orders_agree_bit_for_bit(form):
    """A lattice-kernel form with its blocks in runs per XCD (variant form)
    and in the storage order of their tiles (form + 16): the order in which
    blocks run changes no cell's update."""
    W = wl.droplet_3d(theta_eq_deg=45.0, small=True)
    print(f"[det] 3D 64x64x32, 80 steps, variants {form} and {form + 16}", flush=True)
    a = gpu_run(W.params, W.nodes, 80, tris=W.tris, graph_steps=16, shape=form)
    b = gpu_run(W.params, W.nodes, 80, tris=W.tris, graph_steps=16, shape=form + 16)
    _same(a, b, 3)


def test_3d_coarse_mesh_direct_path_repeats_bit_for_bit():
    """Coarse cap across the periodic edge: some chunks overflow their LDS
    box and add their taps straight to global memory."""
    p = wl.Params(dim=3, nx=48, ny=44, nz=20, bc=(0, 0, 1), tau=0.9, sigma=0.006,
                  theta_eq_deg=100.0, xi=2.0)
    V, T = wl.cap_mesh(9.0, 90.0, 2.0, 4, (1.0, 22.0))
    a = gpu_run(p, V, 60, tris=T)
    b = gpu_run(p, V, 60, tris=T)
    _same(a, b, 3)


def test_2d_batch_repeats_bit_for_bit():
    from helpers import gpu_solver
    draws = wl.batch_draws(8, seed=3)
    runs = []
    for _ in range(2):
        s = gpu_solver([w.params for w in draws], [w.nodes for w in draws])
        s.set_graph_steps(32)
        s.step(101)
        runs.append([collect(s, d, 2) for d in range(len(draws))])
    for d in range(len(draws)):
        _same(runs[0][d], runs[1][d], 2)
