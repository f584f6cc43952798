"""Streaming pins: with tau = infinity (no relaxation) and no force the LB
update of eq. (LBE) reduces to the pure streaming permutation, with
half-way bounce-back at the walls (Sec. "Numerical results", set-up).  The
expected arrays are built by brute force with numpy rolls and an explicit
wall reflection, independent of the oracle's pull loop."""
import math

import numpy as np
import pytest

import oracle as o
import workloads as wl


def brute_stream(f, c, bc):
    """f (Q, nz, ny, nx) -> streamed copy; walls reflect into the opposite
    population of the same cell."""
    Q = f.shape[0]
    shape = f.shape[1:]
    out = np.empty_like(f)
    axes = {0: 2, 1: 1, 2: 0}  # lattice axis -> numpy axis of (nz, ny, nx)
    opp = [0] + [i + 1 if i % 2 == 1 else i - 1 for i in range(1, Q)]
    for i in range(Q):
        g = f[i].copy()
        for a in range(3):
            if c[i, a] != 0:
                g = np.roll(g, c[i, a], axis=axes[a])
        # cells whose source lies beyond a wall take the reflected value
        mask = np.zeros(shape, dtype=bool)
        for a in range(3):
            if bc[a] == 1 and c[i, a] != 0:
                n = shape[axes[a]]
                sl = [slice(None)] * 3
                sl[axes[a]] = 0 if c[i, a] > 0 else n - 1
                mask[tuple(sl)] = True
        g[mask] = f[opp[i]][mask]
        out[i] = g
    return out


@pytest.mark.parametrize("dim,shape,bc", [
    (2, (1, 6, 9), (0, 1, 0)),
    (2, (1, 5, 4), (0, 0, 0)),
    (2, (1, 4, 5), (1, 1, 0)),
    (3, (5, 4, 3), (0, 0, 1)),
    (3, (3, 3, 4), (0, 0, 0)),
])
def test_pure_streaming_matches_brute_force(dim, shape, bc):
    nz, ny, nx = shape
    Q = 9 if dim == 2 else 19
    c, w = o.lattice(dim)
    dev = wl.tagged_deviation(Q, nx * ny * nz, seed=11).reshape(Q, nz, ny, nx)
    f = w[:, None, None, None] + dev
    got, _, _ = o.lb_step(dim, nx, ny, nz, bc, math.inf, f, None)
    want = brute_stream(f, c, bc)
    assert np.array_equal(got, want)


def test_periodic_streaming_returns_after_box_length():
    nx, ny = 7, 5
    c, w = o.lattice(2)
    f = w[:, None, None, None] + wl.tagged_deviation(9, nx * ny, 12).reshape(9, 1, ny, nx)
    g = f.copy()
    for _ in range(nx * ny):
        g, _, _ = o.lb_step(2, nx, ny, 1, (0, 0, 0), math.inf, g, None)
    assert np.array_equal(g, f)
