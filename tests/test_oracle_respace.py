"""Pins of the oracle's tangential re-spacing of a 2D outline (an addition
to the method for long runs; the paper's outline nodes move with the fluid
only).  The rule moves node j by beta/2 (l_j+ - l_j-) along the unit chord
of its neighbours.  Pinned by what it must do, not by its formula: uniform
spacing is a fixed point; nodes on a straight run stay on it and move by
exactly half the edge-length difference times beta; the rule does not
depend on orientation, position or rotation of the outline; repeated, it
evens out a jittered circle while keeping the nodes on the circle up to
the polygon's own chord error and the enclosed area within it."""
import dataclasses
import math

import numpy as np
import pytest

import oracle


def _circle(R, n, jitter=0.0, seed=0):
    rng = np.random.default_rng(seed)
    a = 2 * math.pi * (np.arange(n) + jitter * rng.uniform(-0.45, 0.45, n)) / n
    return np.stack([R * np.cos(a) + 3.0, R * np.sin(a) - 7.0], axis=1)


def _area(q):
    x, y = q[:, 0], q[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def test_uniform_spacing_is_a_fixed_point():
    q = _circle(40.0, 300)
    dq = oracle.respace_2d(q, 0.7)
    assert np.max(np.abs(dq)) < 1e-12


def test_straight_runs_keep_nodes_on_their_edge():
    # a 20 x 10 rectangle with corners as nodes and unevenly spaced nodes on
    # every edge
    rng = np.random.default_rng(4)
    corners = np.array([[0.0, 0.0], [20.0, 0.0], [20.0, 10.0], [0.0, 10.0]])
    pts = []
    for k in range(4):
        a, b = corners[k], corners[(k + 1) % 4]
        t = np.sort(rng.uniform(0.05, 0.95, 9))
        pts.append(a[None, :])
        pts.append(a[None, :] + t[:, None] * (b - a)[None, :])
    q = np.concatenate(pts)
    beta = 0.6
    dq = oracle.respace_2d(q, beta)
    n = len(q)
    for j in range(n):
        if j % 10 == 0:
            continue  # corners
        a, b = q[j - 1], q[(j + 1) % n]
        e = (b - a) / np.linalg.norm(b - a)
        cross = e[0] * dq[j, 1] - e[1] * dq[j, 0]
        lm, lp = np.linalg.norm(q[j] - a), np.linalg.norm(b - q[j])
        assert abs(cross) < 1e-14
        assert abs(float(np.dot(dq[j], e)) - 0.5 * beta * (lp - lm)) < 1e-14


def test_orientation_translation_and_rotation_invariance():
    q = _circle(25.0, 157, jitter=1.0, seed=2) * np.array([1.0, 0.6])
    dq = oracle.respace_2d(q, 0.4)
    rev = oracle.respace_2d(q[::-1].copy(), 0.4)[::-1]
    assert np.max(np.abs(rev - dq)) < 1e-13
    c, s = math.cos(0.7), math.sin(0.7)
    Rm = np.array([[c, -s], [s, c]])
    moved = oracle.respace_2d(q @ Rm.T + np.array([100.0, -40.0]), 0.4)
    assert np.max(np.abs(moved - dq @ Rm.T)) < 1e-11


def test_repeated_respacing_evens_a_jittered_circle():
    R, n = 50.0, 400
    q = _circle(R, n, jitter=1.0, seed=7)
    h = 2 * math.pi * R / n
    lengths = lambda p: np.linalg.norm(np.roll(p, -1, axis=0) - p, axis=1)
    s0 = np.std(lengths(q)) / np.mean(lengths(q))
    a0 = _area(q)
    for _ in range(3000):
        q = q + oracle.respace_2d(q, 0.5)
    s1 = np.std(lengths(q)) / np.mean(lengths(q))
    r = np.linalg.norm(q - np.array([3.0, -7.0]), axis=1)
    assert s0 > 0.2 and s1 < 1e-3 * s0
    # nodes stay on the circle within a few chord sagittas h^2 / (8 R)
    assert np.max(np.abs(r - R)) < 4 * h * h / (8 * R)
    # the area moves by less than the gap between the circle and its polygon
    assert abs(_area(q) - a0) < 4 * n * h ** 3 / (12 * R)


@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_coupled_run_with_respacing_is_the_plain_run_plus_the_move(beta):
    """orc_run with respace: the last step's positions are the advected
    positions plus the re-spacing of the positions before it."""
    import workloads as wl
    W = wl.droplet_2d_small()
    p = W.params
    a = oracle.run(p, W.nodes, 3)
    p2 = dataclasses.replace(p, respace=beta)
    b2 = oracle.run(p2, W.nodes, 2)
    q_before = b2["q"]
    c = oracle.run(p2, W.nodes, 3)
    step = oracle.run(p2, q_before, 1, f0=b2["f"])
    assert np.array_equal(step["q"], c["q"])
    if beta == 0.0:
        assert np.array_equal(c["q"], a["q"])
    else:
        expect = (q_before + step["qdot"]) + oracle.respace_2d(q_before, beta)
        assert np.max(np.abs(expect - c["q"])) < 1e-12
