"""Host-side geometry of the learned warm start: a predicted outline that
folds back on itself is replaced by the analytic cap before anything runs.
Keeping the nodes above the wall clamps any part of the predicted outline
that dips below it onto one line; if that part also runs backwards in x,
the outline gets a spike of zero width (a 180-degree turn), which no
solver step survives (every learned start that turned unstable on the
MI355X in the time-to-equilibrium runs had one, and no stable start did)."""
import math

import numpy as np
import pytest

import workloads as wl
from paper_2503_20605_amd import warmstart as ws


class _FakeOutput:
    def __init__(self, a):
        self.a = a

    def cpu(self):
        return self

    def numpy(self):
        return self.a


class _FakeNet:
    """Returns fixed (already unscaled) outputs, one row per draw."""

    def __init__(self, rows):
        self.rows = rows

    def forward(self, X):
        assert X.shape == (len(self.rows), ws.WIDTHS[0])
        return _FakeOutput(np.array(self.rows, dtype=np.float32))


def _draws():
    return [w for w in wl.batch_draws(40, seed=6) if w.params.theta_eq_deg < 40.0][:2]


@pytest.mark.parametrize("theta", [20.0, 45.0, 90.0, 135.0, 160.0])
def test_clean_caps_do_not_fold(theta):
    area, xi, nx = 3000.0, 2.0, 400
    ref, rcap, rc = ws.reference(math.radians(theta), area, xi, nx)
    q = ws.outline_from_profile(ref, rcap, 500, ws.H_MIN * xi)
    t = ws.max_turn_deg(q)
    # the contact corner turns by 180 - theta, smoothed over the rays
    assert t <= 180.0 - theta + 1.0
    assert t < ws.MAX_TURN_DEG


def test_max_turn_of_a_spike_is_180():
    q = np.array([[0.0, 0.0], [4.0, 0.0], [2.0, 0.0], [6.0, 0.0], [6.0, 3.0], [0.0, 3.0]])
    assert abs(ws.max_turn_deg(q) - 180.0) < 1e-9
    square = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    assert abs(ws.max_turn_deg(square) - 90.0) < 1e-9


def _base_ray(ref, rcap, xi):
    pts = ref[None, :] + rcap[:, None] * np.stack([np.cos(ws.PHI), np.sin(ws.PHI)], axis=1)
    base = np.where((np.abs(pts[:, 1] - xi) < 1e-6) & (pts[:, 0] < ref[0]))[0]
    return int(base[len(base) // 2])


def test_folded_prediction_is_replaced_by_the_cap():
    draws = _draws()
    assert len(draws) == 2
    rows = []
    for k, w in enumerate(draws):
        p = w.params
        ref, rcap, rc = ws.reference(math.radians(p.theta_eq_deg), ws.polygon_area(w.nodes), p.xi, p.nx)
        o = np.zeros(ws.N_OUT)
        o[:ws.K_RAYS] = 0.002 * np.cos(3 * ws.PHI)       # a mild, foldless change
        if k == 1:
            # a 20 % bump on one ray that ends on the base pushes that point
            # below the wall, down and outwards; clamped back above the wall
            # it runs out and back along one line
            j = _base_ray(ref, rcap, p.xi)
            o[j] = 0.2 * rcap[j] / rc
        rows.append(o)
    scale = (np.zeros(ws.N_OUT), np.ones(ws.N_OUT))
    starts, rejected = ws.predict_starts(_FakeNet(rows), scale, draws)
    assert rejected == [1]
    cap = ws.cap_starts([draws[1]])[0]
    assert np.array_equal(starts[1][0], cap[0]) and np.all(starts[1][1] == 0.0)
    assert ws.max_turn_deg(starts[0][0]) < ws.MAX_TURN_DEG
    assert not np.array_equal(starts[0][0], ws.cap_starts([draws[0]])[0][0])
