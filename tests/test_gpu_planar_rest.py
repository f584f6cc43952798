"""Droplets run to rest on the GPU end at the planar equilibrium outline.

Eight held-out draws of the batch recipe (theta_eq 40-144 deg, xi/R0
0.07-0.11, the recipe's tangential re-spacing on) run to rest in one batch
from their 90-degree caps, fp32 storage, with the rest criterion of the
time-to-equilibrium benchmark.  Each end angle (from the half-height) must
match the angle of the planar equilibrium outline at the droplet's own
theta_eq and xi/R0 (the App. B system in two dimensions, solved by the
oracle's shape solver; the simulated droplets measured 0.01-0.35 deg below
it on the MI355X).  The outline, not theta_eq, is the reference: at these
xi/R0 the wall term's finite range moves the angle measured from the
half-height several degrees away from theta_eq (App. C)."""
import math

import numpy as np
import pytest

import oracle as o
import workloads as wl
from helpers import gpu_solver

pytestmark = pytest.mark.gpu

PICK = (154, 25, 26, 52, 238, 54, 232, 172)
REST = dict(tol=1e-5, angle_tol_deg=0.01, check_every=1000, hold=10)


def test_batch_rests_at_the_planar_outline():
    import statics
    draws = wl.batch_draws(256, seed=6)
    sub = [draws[i] for i in PICK]
    ref = []
    for w in sub:
        R0 = math.sqrt(o.volume_2d(w.nodes) / math.pi)
        s = statics.theory_2d(math.radians(w.params.theta_eq_deg), w.params.xi / R0)
        ref.append(math.degrees(o.angle_from_height_2d(s["ell"], math.pi)))
    print(f"[planar] {len(sub)} droplets to rest (300k-step cap)", flush=True)
    s = gpu_solver([w.params for w in sub], [w.nodes for w in sub])
    s.set_graph_steps(100)
    steps = s.run_to_rest(max_steps=300000, **REST)
    dg = s.diagnostics(-1)
    for k, w in enumerate(sub):
        th = math.degrees(dg[k]["theta_meas"])
        print(f"[planar] draw {PICK[k]}: theta_eq {w.params.theta_eq_deg:.1f}, at rest after {steps[k]} steps, "
              f"angle {th:.3f} against the planar outline's {ref[k]:.3f} deg", flush=True)
        assert steps[k] > 0
        assert abs(th - ref[k]) < 0.6
    # the reference is not theta_eq itself
    assert max(abs(r - w.params.theta_eq_deg) for r, w in zip(ref, sub)) > 3.0
