"""Tangential re-spacing of a 2D outline on the GPU (an addition for long
runs, see iblb_set_node_respacing): parity with the oracle's run with the
same rate, for a lone droplet and inside a batch, through graph replays and
direct launches; and, over a long run, the effect it exists for.  Without
it, a held-out batch draw (224x224, R0 14.4, theta_eq 112 deg, tau 0.61)
reaches its angle within a few thousand steps, then, after some 2e5 steps,
opens a gap of tens of lattice units at a contact corner, loses a third of
its area through it and collapses to about 25 deg (measured on the MI355X
in 2e5-step chunks at node spacings 0.8 and 0.4).  With it, the spacing
stays even and the area and angle stay put."""
import dataclasses

import numpy as np
import pytest

import oracle as o
import workloads as wl
from helpers import collect, compare_fields, gpu_run, gpu_solver

pytestmark = pytest.mark.gpu


def _uneven(R, n, xc, drop):
    return np.delete(wl.cap_polygon(R, 90.0, 2.0, n, xc), drop, axis=0)


def test_respacing_matches_oracle_lone_droplet():
    p = wl.Params(dim=2, nx=96, ny=40, tau=0.7, sigma=0.006, theta_eq_deg=40.0, xi=2.0, respace=0.4)
    q = _uneven(12.0, 94, 48.0, list(range(10, 40, 3)))
    print("[respace] lone 96x40, 300 steps", flush=True)
    g = gpu_run(p, q, 300, graph_steps=16)
    r = o.run(p, q, 300)
    r0 = o.run(dataclasses.replace(p, respace=0.0), q, 300)
    assert np.max(np.abs(r["q"] - r0["q"])) > 0.1
    drho, du, dq = compare_fields(g, r, 2, "respace lone")
    assert drho <= 1e-5 and du <= 1e-5 and dq <= 1e-5


def test_respacing_matches_oracle_in_a_batch():
    ps = [wl.Params(dim=2, nx=96, ny=40, tau=0.7, sigma=0.006, theta_eq_deg=40.0, xi=2.0, respace=0.4),
          wl.Params(dim=2, nx=70, ny=33, tau=1.3, sigma=0.009, theta_eq_deg=140.0, xi=2.0, respace=0.1),
          wl.Params(dim=2, nx=64, ny=32, tau=0.9, sigma=0.005, theta_eq_deg=90.0, xi=2.0)]
    qs = [_uneven(12.0, 94, 48.0, list(range(10, 40, 3))), _uneven(9.0, 71, 35.0, list(range(5, 30, 3))),
          wl.cap_polygon(8.0, 90.0, 2.0, 60, 32.0)]
    print("[respace] batch of 3, 2 x 101 steps", flush=True)
    s = gpu_solver(ps, qs)
    s.set_graph_steps(16)
    s.step(101)
    s.step(101)
    for d in range(3):
        g = collect(s, d, 2)
        r = o.run(ps[d], qs[d], 202)
        drho, du, dq = compare_fields(g, r, 2, f"respace batch{d}")
        assert drho <= 1e-5 and du <= 1e-5 and dq <= 1e-5


def test_respacing_keeps_a_long_run_closed():
    draws = wl.batch_draws(256, seed=6)
    w = draws[68]
    p = w.params
    assert (p.nx, p.ny) == (224, 224) and abs(p.theta_eq_deg - 112.3) < 0.1
    pr = dataclasses.replace(p, respace=0.05)
    s = gpu_solver([pr], [w.nodes])
    s.set_graph_steps(100)
    a0 = abs(float(np.sum(w.nodes[:, 0] * np.roll(w.nodes[:, 1], -1) - np.roll(w.nodes[:, 0], -1) * w.nodes[:, 1]))) / 2
    worst_gap, worst_area, th = 0.0, 0.0, []
    for c in range(8):
        s.step(50000)
        q, _, _ = s.read_nodes(0)
        gap = float(np.max(np.linalg.norm(np.roll(q, -1, axis=0) - q, axis=1)))
        area = abs(float(np.sum(q[:, 0] * np.roll(q[:, 1], -1) - np.roll(q[:, 0], -1) * q[:, 1]))) / 2
        dg = s.diagnostics(0)
        th.append(np.degrees(dg["theta_meas"]))
        worst_gap = max(worst_gap, gap)
        worst_area = max(worst_area, abs(area / a0 - 1.0))
        print(f"[respace] {50000 * (c + 1)} steps: largest gap {gap:.3f}, area change {area / a0 - 1:+.2e}, "
              f"angle {th[-1]:.2f} deg, normal speed {dg['max_normal_speed']:.1e}", flush=True)
    assert dg["status"] == 0
    assert worst_gap < 1.5
    assert worst_area < 0.02
    assert max(th[2:]) - min(th[2:]) < 0.5


def test_respacing_arguments_are_checked():
    from paper_2503_20605_amd import IblbError
    W = wl.droplet_3d(theta_eq_deg=90.0, small=True)
    s3 = gpu_solver([W.params], [W.nodes], [W.tris])
    with pytest.raises(IblbError):
        s3.set_node_respacing(0, 0.1)          # a 3D mesh has no outline to re-space
    p = wl.Params(dim=2, nx=64, ny=32, tau=0.9, sigma=0.005, theta_eq_deg=90.0, xi=2.0)
    s2 = gpu_solver([p], [wl.cap_polygon(8.0, 90.0, 2.0, 60, 32.0)])
    for bad in (-0.1, 1.0, float("nan")):
        with pytest.raises(IblbError):
            s2.set_node_respacing(0, bad)
    with pytest.raises(IblbError):
        s2.set_node_respacing(1, 0.1)          # no such droplet
    s2.set_node_respacing(0, 0.0)
    s2.set_node_respacing(0, 0.999)
