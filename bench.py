"""Benchmark of the coupled IB-LB step on one MI355X.

Workload (default): the 3D droplet, a 256x256x128 D3Q19 box (periodic x and
y, walls at z = 0 and z = 128) holding a hemispherical cap of radius 40 meshed
by a frequency-45 icosphere (20 252 vertices, 40 500 triangles), xi = 4,
sigma = 0.005, tau = 0.8, theta_eq = 90 degrees, fp32 arithmetic and fp32
shifted storage.  A step is the whole coupled method: nodal forces,
spreading, fused stream + collide, interpolation, advection.  Inputs are
resident in HBM before the timed region.

Prints one JSON line: MLUPS of the whole step over exactly --steps timed
steps (value); the roofline of the dominant kernel (the fused lattice
kernel, HBM bound, 152 algorithmic bytes per cell update in fp32) from the
pair of HIP events that each of its launches in the timed region marks at
dispatch; the same steps replayed from a captured graph for comparison;
secondary lines (the 1024x512 D2Q9 step, the lattice kernel alone on boxes
far above the last-level cache); and the FP64 CPU oracle timed on a bounded
sample of the same workload, on one thread and on every thread.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# every TIMING_STRIDE-th lattice launch of the timed region carries events
TIMING_STRIDE = 8


# lattice-kernel forms (variant % 16): block width along x (0: flat runs of
# 256 cells), non-temporal stores, non-temporal loads; variant // 16 is the
# block order (0: one contiguous run of tiles per XCD, 1: storage order)
LB_BX = (256, 128, 64) * 4 + (0,) * 4
LB_NT = (0, 0, 0, 1, 1, 1) * 2 + (0, 1, 0, 1)
LB_NTL = (0,) * 6 + (1,) * 6 + (0, 0, 1, 1)
LB_ORDER = ("xcd-runs", "storage")


def lb_kernel_name(dim, storage, variant, vis=0, one=1):
    """Name of the lattice kernel instance as the kernel trace prints it; one:
    the form for a handle of a single droplet (used unless vis)."""
    k = variant % 16
    return (f"k_lb<{dim}, {storage}, {LB_BX[k]}, {LB_NT[k]}, {LB_NTL[k]}, "
            f"{vis}, {0 if vis else one}>")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_lb_traffic.md")


def code_only(src):
    """C++ source without // comments and with whitespace collapsed."""
    import re
    return re.sub(rb"\s+", b" ", re.sub(rb"//[^\n]*", b"", src)).strip()


def lb_source_hash(lattice_src=None, kernels_src=None, host_src=None):
    """Hash of the lattice kernel's code (lattice.hpp, the part of
    kernels.hpp up to the end of the lattice kernel, and the population
    layout and tile order of iblb.hip; comments and layout left out), to tell
    whether stored counter readings still describe the kernel as built."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2503_20605_amd", "csrc")
    lat = lattice_src if lattice_src is not None else open(os.path.join(csrc, "lattice.hpp"), "rb").read()
    k = kernels_src if kernels_src is not None else open(os.path.join(csrc, "kernels.hpp"), "rb").read()
    hs = host_src if host_src is not None else open(os.path.join(csrc, "iblb.hip"), "rb").read()
    h = hashlib.sha256()
    h.update(code_only(lat))
    h.update(code_only(k[:k.index(b"// Nodes whose coordinates are not finite")]))
    lo = hs.index(b"// Lattice-kernel variants (autotuner candidates)")
    h.update(code_only(hs[lo:hs.index(b"int tiles_of(", lo)]))
    lo = hs.index(b"// Tiles of droplet d in the given shape")
    h.update(code_only(hs[lo:hs.index(b"// ---- kernel dispatch", lo)]))
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, order):
    """HBM-side bytes per launch of `kernel` in block order `order` on
    `workload` from the stored FETCH_SIZE / WRITE_SIZE counter runs (each
    scaled by what the counter reads for a copy of known size), or None when
    there is no reading for this kernel, order and workload or the kernel's
    source changed since."""
    try:
        text = open(TRAFFIC_FILE).read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, ValueError, IndexError):
        return None
    if rec.get("source_hash") != lb_source_hash():
        return None
    for r in rec.get("readings", []):
        if r["kernel"] == kernel and r["workload"] == workload and r["block_order"] == order:
            return round(r["fetch_bytes"] + r["write_bytes"])
    return None


def bytes_per_cell(dim, storage):
    Q = 9 if dim == 2 else 19
    return 2 * Q * (4 if storage == 0 else 2)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--run", type=int, default=1, help="sweep point 0..9 of the 1024x512 set")
    ap.add_argument("--graph-steps", type=int, default=64)
    ap.add_argument("--variant", type=int, default=-1,
                    help="lattice-kernel variant 0..31; -1 autotunes")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the secondary lines (1024x512 D2Q9 step, lattice kernel alone on "
                         "working sets far above the last-level cache)")
    ap.add_argument("--profile-only", action="store_true",
                    help="short run for profilers: no CPU leg, no extra sizes")
    ap.add_argument("--tte", action="store_true",
                    help="time to equilibrium of held-out batch droplets, plain fp32 against fp16 "
                         "storage with the learned warm start, instead of the step rate")
    ap.add_argument("--droplets", type=int, default=256)
    ap.add_argument("--dump", default=None,
                    help="--tte: write every droplet's steps and angles per arm to this JSON file")
    ap.add_argument("--train-draws", type=int, default=512,
                    help="seeded draws whose equilibria train the warm-start network (--tte)")
    ap.add_argument("--max-steps", type=int, default=None,
                    help="step cap: --tte 800000 (per arm), --tanner 150000")
    ap.add_argument("--workload", default="d3q19", choices=["d3q19", "d2q9", "d3q19_spreading"])
    ap.add_argument("--lam", type=float, default=None,
                    help="viscosity ratio mu_in / mu_out (default: the workload's own)")
    ap.add_argument("--mlp", action="store_true",
                    help="time training steps of the warm-start network (4096 samples, widths "
                         "4-256-256-256-1280) on seeded synthetic data")
    ap.add_argument("--spreading", action="store_true",
                    help="contact radius against time on the spreading set-up (240x240x130, "
                         "R0 = 60, viscosity ratio 10) by both protocols, with the exponent of "
                         "the early power law")
    ap.add_argument("--tanner", action="store_true",
                    help="contact radius against time in the late, viscous stage: a hemisphere of "
                         "R0 = 60 spreading towards theta_eq = 22.5 deg (Tanner's law r_c ~ t^(1/10))")
    ap.add_argument("--sweep", action="store_true",
                    help="the ten-run 1024x512 sweep (tau 0.6/1.0 x theta_eq 30-150 deg), 50000 steps "
                         "each: measured angle and contact radius at the end of every run")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="only the FP64 oracle on the host: the oracle-sized 2D and 3D cases, one thread "
                         "and all threads")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="only the lattice kernel alone on the boxes far above the last-level "
                         "cache and the copy probe (short; used for hardware-counter runs)")
    return ap.parse_args()


def spreading(a):
    """Contact radius r_c(t) of a sphere spreading on the substrate (Sec.
    Dynamics set-up: 240x240x130, R0 = 60, xi = 2, lambda = 10) by protocol
    (i) at three z_cut / R0 and protocol (ii) at three eps, until t = t~ =
    sqrt(rho R0^3 / sigma).  The exponent of r_c ~ t^alpha is fitted on a
    log-log scale over 0.05 < t / t~ < 0.5, the window after the initial
    plateau in which the paper finds the inertial law r_c ~ t^(1/2).  The
    eps values are far below the paper's 0.1: with mesh edges of about one
    lattice unit every triangle of the lower half differs in height by less
    than 0.1 R0 = 6, so that value does not single out a flat region here."""
    import numpy as np
    import workloads as wl
    from paper_2503_20605_amd import Solver, params_from
    R0 = 60.0
    zcuts, epss = (0.025, 0.05, 0.1), (0.001, 0.003, 0.01)
    runs = []
    for th in (45.0, 90.0):
        W = wl.droplet_3d_spreading(lam=10.0 if a.lam is None else a.lam, theta_eq_deg=th)
        p = W.params
        t_tilde = math.sqrt(R0 ** 3 / p.sigma)
        s = Solver([params_from(p)], [W.nodes], [W.tris])
        s.set_viscosity_ratio(0, p.lam)
        s.autotune(steps=16)
        every = 50
        n_total = int(math.ceil(t_tilde / every)) * every
        ts = []
        series = {f"i_zcut{z:g}": [] for z in zcuts}
        series.update({f"ii_eps{e:g}": [] for e in epss})
        t0 = time.perf_counter()
        done = 0
        while done < n_total:
            s.step(every)
            done += every
            ts.append(done)
            for k in range(3):
                r1, r2, _ = s.contact_radius(0, zcuts[k] * R0, epss[k] * R0)
                series[f"i_zcut{zcuts[k]:g}"].append(r1 / R0)
                series[f"ii_eps{epss[k]:g}"].append(r2 / R0)
        wall = time.perf_counter() - t0
        d = s.diagnostics(0)
        s.close()
        t = np.array(ts, dtype=np.float64) / t_tilde
        alpha = {}
        for name, r in series.items():
            r = np.array(r, dtype=np.float64)
            sel = (t > 0.05) & (t < 0.5) & np.isfinite(r) & (r > 0)
            alpha[name] = (round(float(np.polyfit(np.log(t[sel]), np.log(r[sel]), 1)[0]), 4)
                           if sel.sum() >= 3 else None)
        runs.append({"theta_eq_deg": th, "t_tilde_steps": round(t_tilde, 1), "steps": n_total,
                     "wall_s": round(wall, 2), "alpha": alpha,
                     "t_over_t_tilde": [round(v, 5) for v in t.tolist()],
                     "rc_over_R0": {k: [None if not math.isfinite(v) else round(v, 5) for v in r]
                                    for k, r in series.items()},
                     "final_theta_meas_deg": round(math.degrees(d["theta_meas"]), 3)})
        print(json.dumps({"theta_eq_deg": th, "alpha": alpha, "wall_s": round(wall, 2)}),
              file=sys.stderr, flush=True)
    print(json.dumps({"metric": "contact-radius exponent of early spreading (inertial law: 1/2)",
                      "workload": W.name, "fit_window_t_over_t_tilde": [0.05, 0.5],
                      "runs": runs}), flush=True)


def tanner(a):
    """Late-stage spreading (Sec. Dynamics): the droplet starts as a
    hemisphere of the volume of a sphere of radius R0 = 60 and spreads towards
    its theta_eq = 22.5 deg cap.  The contact radius is sampled on a
    logarithmic grid of steps by protocol (i) (z_cut = h* + 1, just above the
    film the wall term holds) and protocol (ii) (eps = 0.003); the exponent of
    r_c ~ t^alpha is fitted per decade of steps.  Tanner's law predicts
    alpha = 1/10 once viscous forces and surface tension balance."""
    import numpy as np
    import workloads as wl
    from paper_2503_20605_amd import Solver, params_from
    W = wl.droplet_3d_tanner()
    p = W.params
    R0 = W.meta["R0"]
    s = Solver([params_from(p)], [W.nodes], [W.tris])
    s.autotune(steps=16)
    zc = p.xi * 2.0 ** (1.0 / 3.0) + 1.0
    n_total = a.max_steps or 150000
    marks = sorted({int(round(10 ** e)) for e in np.arange(1.0, math.log10(n_total) + 1e-9, 0.05)})
    ts, ri, rii = [], [], []
    t0 = time.perf_counter()
    done = 0
    for m in marks:
        s.step(m - done)
        done = m
        r1, r2, _ = s.contact_radius(0, zc, 0.003 * R0)
        ts.append(done)
        ri.append(r1)
        rii.append(r2)
        if done % 10000 == 0 or m == marks[-1]:
            print(json.dumps({"steps": done, "r_i": r1, "r_ii": r2}), file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    d = s.diagnostics(0)
    s.close()
    t = np.array(ts, dtype=np.float64)
    fits = {}
    for name, r in (("i", np.array(ri)), ("ii", np.array(rii))):
        for lo in (100, 1000, 10000):
            sel = (t >= lo) & (t <= 10 * lo) & np.isfinite(r) & (r > 0)
            fits[f"{name}_{lo}_{10 * lo}"] = (round(float(np.polyfit(np.log(t[sel]), np.log(r[sel]), 1)[0]), 4)
                                              if sel.sum() >= 3 else None)
    print(json.dumps({"metric": "contact-radius exponent of late spreading (Tanner's law: 1/10)",
                      "workload": W.name, "cells": p.nx * p.ny * p.nz, "vertices": len(W.nodes),
                      "steps": n_total, "wall_s": round(wall, 1),
                      "ms_per_step": round(wall / n_total * 1e3, 4), "z_cut": round(zc, 4),
                      "eps": 0.003, "r_eq_closed_form": round(W.meta["r_eq"], 3), "alpha": fits,
                      "final": {"r_i": ri[-1], "r_ii": rii[-1],
                                "theta_meas_deg": math.degrees(d["theta_meas"]),
                                "max_normal_speed": d["max_normal_speed"]},
                      "series": {"steps": ts, "r_i": [None if not math.isfinite(v) else round(v, 4) for v in ri],
                                 "r_ii": [round(v, 4) for v in rii]}}), flush=True)


def sweep(a):
    """The ten runs of the 1024x512 workload (tau in {0.6, 1.0} x theta_eq in
    {30, 60, 90, 120, 150} deg, initial cap angle theta_eq + U(-5, 5) deg),
    50000 coupled steps each: wall time, the angle from the half-height (2D
    counterpart of eq. angleh) and the contact radius (protocol (i) at h*)
    at the end."""
    import workloads as wl
    from paper_2503_20605_amd import Solver, params_from
    runs = []
    for run in range(10):
        W = wl.droplet_2d_large(run=run)
        p = W.params
        # the variant is picked on a scratch copy of the run (tuning steps
        # advance the simulation), over enough steps to replay the step graph
        s = Solver([params_from(p)], [W.nodes])
        v, _ = s.autotune(steps=130)
        s.close()
        s = Solver([params_from(p)], [W.nodes])
        s.set_lb_variant(v)
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(W.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        d = s.diagnostics(0)
        s.close()
        runs.append({"run": run, "tau": p.tau, "theta_eq_deg": p.theta_eq_deg,
                     "theta0_deg": round(W.meta["theta0_deg"], 3), "steps": W.steps, "lb_variant": v,
                     "wall_s": round(wall, 3),
                     "MLUPS": round(p.nx * p.ny * W.steps / wall / 1e6, 1),
                     "theta_meas_deg": round(math.degrees(d["theta_meas"]), 3),
                     "contact_radius": round(d["contact_radius"], 3),
                     "max_normal_speed": d["max_normal_speed"], "status": d["status"]})
        print(json.dumps(runs[-1]), file=sys.stderr, flush=True)
    print(json.dumps({"metric": "1024x512 sweep: angle from the half-height after 50000 steps",
                      "workload": "d2q9_1024x512_R120_N1024_run0-9", "runs": runs}), flush=True)


def tte(a):
    """Time to equilibrium of held-out batch droplets: the plain solver (fp32
    storage, 90-degree cap, fluid at rest) against fp16 storage with the
    learned warm start, on the same draws and GPU, every arm one batch run
    to rest (droplets freeze as they come to rest).  The network is trained
    in the same run: equilibria of `--train-draws` seeded draws (seed 5)
    generated by the batched solver in fp16, then full-batch Adam on the
    device; held-out draws use seed 6.  Two more arms separate the effects:
    fp16 from the 90-degree cap, fp16 from the analytic equal-area cap."""
    import numpy as np
    import workloads as wl
    from paper_2503_20605_amd import warmstart as ws
    REST = ws.REST
    if a.max_steps is None:
        a.max_steps = 800000
    t0 = time.perf_counter()
    X, Y, S = ws.generate(wl.batch_draws(a.train_draws, seed=5), storage=1, max_steps=a.max_steps,
                          rest=REST, log=log)
    m, scale, hist = ws.fit(X, Y, steps=4000, log=lambda msg: None)
    t_train = time.perf_counter() - t0
    log(f"network trained on {len(X)} equilibria in {t_train:.1f} s (loss {hist[-1][1]:.3e})")
    draws = wl.batch_draws(a.droplets, seed=6)
    res = ws.evaluate_arms(draws, m, scale, a.max_steps, log=log, rest=REST)
    if a.dump:
        # the trained network (parameters and output scaling), the learned
        # start outlines, and which of them turned unstable
        bad = [i for i, x in enumerate(res["f16_learned"]["steps"]) if x == -2]
        np.savez(a.dump + ".net.npz", params=m.get_params(), mean=scale[0], std=scale[1],
                 unstable=np.array(bad, dtype=np.int64),
                 **{f"start_q_{i}": st[0] for i, st in enumerate(res["f16_learned"]["starts"])})
    m.close()
    summary = ws.summarize(draws, res, a.max_steps)
    cells = sum(w.params.nx * w.params.ny for w in draws)
    if a.dump:
        # per-droplet record of every arm, for checks against the planar
        # equilibrium outline (tests/report_tte_planar.py)
        rec = {"rest_criterion": REST, "max_steps": a.max_steps,
               "draws": [{"nx": w.params.nx, "ny": w.params.ny, "tau": w.params.tau, "sigma": w.params.sigma,
                          "theta_eq_deg": w.params.theta_eq_deg, "xi": w.params.xi,
                          "area": float(ws.polygon_area(w.nodes))} for w in draws],
               "arms": {k: {"steps": [int(x) for x in r["steps"]], "theta_deg": [float(x) for x in r["theta"]],
                            "wall_s": r["wall"]} for k, r in res.items()}}
        with open(a.dump, "w") as fh:
            json.dump(rec, fh)
    print(json.dumps({"metric": "time to equilibrium of held-out batch droplets: plain fp32 from the "
                                "90-degree cap against fp16 storage with the learned warm start",
                      "rest_criterion": REST, "droplets": len(draws), "cells": cells,
                      "training": {"draws": a.train_draws, "equilibria": int(len(X)),
                                   "seconds_generate_and_train": round(t_train, 1),
                                   "final_loss": hist[-1][1]},
                      **summary}), flush=True)


MFMA_BF16_PEAK_TFLOPS = 2500.0


def mlp_rate(a):
    """Full-batch training steps (forward, backward, Adam) of the warm-start
    network on seeded synthetic inputs and targets of the training set's
    shape; bf16 matrix-core products with fp32 accumulation."""
    import numpy as np
    import torch
    from paper_2503_20605_amd import MLP
    from paper_2503_20605_amd.warmstart import WIDTHS, _init_params
    rng = np.random.default_rng(11)
    B = 4096
    X = rng.standard_normal((B, WIDTHS[0])).astype(np.float32)
    Y = rng.standard_normal((B, WIDTHS[-1])).astype(np.float32)
    m = MLP(WIDTHS, B)
    m.set_params(_init_params(WIDTHS, 7))
    x, y = m._dev(X), m._dev(Y)
    for _ in range(a.warmup if a.warmup < 200 else 20):
        m.train_step(x, y, 1e-3)
    torch.cuda.synchronize()
    n = min(a.steps, 500)
    t0 = time.perf_counter()
    for _ in range(n):
        loss = m.train_step(x, y, 1e-3)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / n
    macs = B * sum(WIDTHS[i] * WIDTHS[i + 1] for i in range(len(WIDTHS) - 1))
    tflops = 6 * macs / dt / 1e12
    t0 = time.perf_counter()
    for _ in range(50):
        m.forward(x)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / 50
    m.close()
    print(json.dumps({"metric": "warm-start network training step (forward + backward + Adam)",
                      "value": round(dt * 1e3, 4), "unit": "ms", "steps": n,
                      "higher_is_better": False, "dtype": "bf16 products, fp32 accumulation",
                      "data": "synthetic (seeded)",
                      "config": {"workload": "mlp_4-256-256-256-1280_batch4096"},
                      "roofline": {"bound": "mfma", "achieved": round(tflops, 2),
                                   "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": round(tflops / MFMA_BF16_PEAK_TFLOPS, 5), "traffic": None},
                      "forward_ms": round(fwd * 1e3, 4), "final_loss": round(loss, 5)}), flush=True)


def lb_only_rate(dim, nx, ny, nz, storage, steps):
    """Lattice kernel on a big box with no interface (every cell is a plain
    collide + stream), autotuned; its per-launch duration from the events its
    dispatch marks, over `steps` timed steps, and from graph replays of
    back-to-back launches without events."""
    from paper_2503_20605_amd import Solver, make_params
    p = make_params(dim=dim, nx=nx, ny=ny, nz=nz, tau=0.8, wetting=False)
    s = Solver([p], None, storage=storage)
    v, _ = s.autotune(steps=16)
    s.set_timing(True)
    s.step(steps + 1)
    lb_ms, _ = s.last_timing()
    s.set_timing(False)
    # the same kernel replayed back to back from a graph of 64 launches, no
    # events on any of them (median of three replays)
    graph_ms = sorted(s.time_lattice(64) for _ in range(3))[1]
    cells = nx * ny * nz
    gbs = bytes_per_cell(dim, storage) * cells / (lb_ms * 1e-3) / 1e9
    s.close()
    return {"lattice": f"{'D2Q9' if dim == 2 else 'D3Q19'} {nx}x{ny}" + (f"x{nz}" if dim == 3 else ""),
            "storage": ["f32", "f16", "bf16"][storage], "variant": v, "block_order": LB_ORDER[v // 16],
            "working_set_MB": round(bytes_per_cell(dim, storage) * cells / 1e6, 1),
            "lb_us": round(lb_ms * 1e3, 2),
            "MLUPS": round(cells / (lb_ms * 1e-3) / 1e6, 1),
            "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "lb_us_graph": round(graph_ms * 1e3, 2),
            "frac_graph": round(bytes_per_cell(dim, storage) * cells / (graph_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(lb_kernel_name(dim, storage, v),
                                        f"d{dim}q{9 if dim == 2 else 19}_{nx}x{ny}"
                                        + (f"x{nz}" if dim == 3 else "") + "_lattice_only",
                                        LB_ORDER[v // 16])}


def log(msg):
    """Progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(W, steps_one, steps_all):
    """The FP64 oracle on the same workload, on the host: `steps_one`
    coupled steps on one thread and `steps_all` on every thread OpenMP is
    given (the lattice update shares rows among threads).  The set-up of the
    oracle's arrays (a zero-step run) is timed separately and left out."""
    import oracle as o
    p = W.params
    cells = p.nx * p.ny * (p.nz if p.dim == 3 else 1)

    def timed(n):
        t0 = time.perf_counter()
        r = o.run(p, W.nodes, n, tris=W.tris)
        dt = time.perf_counter() - t0
        assert r["status"] == 0
        return dt

    default_threads = o.threads(0)
    all_threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or default_threads
    o.threads(1)
    setup1 = timed(0)
    t1 = timed(steps_one) - setup1
    used = o.threads(all_threads)
    setupn = timed(0)
    tn = timed(steps_all) - setupn
    o.threads(default_threads)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {
        "value": round(cells * steps_all / tn / 1e6, 3), "unit": "MLUPS", "cores": used,
        "kind": "oracle",
        "sample": f"{steps_all} coupled steps of the same {W.name} workload, FP64 oracle on {used} "
                  f"threads ({tn:.1f} s after {setupn:.1f} s of array set-up)",
        "single_thread": {"value": round(cells * steps_one / t1 / 1e6, 3), "unit": "MLUPS",
                          "cores": 1,
                          "sample": f"{steps_one} coupled steps, 1 thread ({t1:.1f} s)"},
        "nproc": os.cpu_count(), "cpus_available": affinity, "cpu_model": cpu_model()}


def cpu_configs(a):
    """The FP64 oracle alone, on the host, on one thread and on all: the
    128x64 D2Q9 droplet run in full (2000 steps), the 1024x512 D2Q9 sweep
    point over its first 500 steps, and the 64x64x32 D3Q19 copy of the 3D
    workload over 1000 steps.  No GPU work."""
    import workloads as wl
    out = {}
    for W, n in ((wl.droplet_2d_small(), 2000), (wl.droplet_2d_large(run=a.run), 500),
                 (wl.droplet_3d(theta_eq_deg=90.0, small=True), 1000)):
        log(f"oracle {W.name}, {n} steps")
        out[W.name] = cpu_baseline(W, n, n)
    print(json.dumps({"metric": "FP64 oracle MLUPS on the host", "configs": out}), flush=True)


def main():
    a = parse()
    if a.cpu_configs:
        cpu_configs(a)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the droplet batch "
                                   "and the single-box path are not sharded across GPUs"}))
        sys.exit(2)
    import torch
    import workloads as wl
    from paper_2503_20605_amd import STORAGE, Solver, params_from

    if a.tte:
        tte(a)
        return
    if a.mlp:
        mlp_rate(a)
        return
    if a.spreading:
        spreading(a)
        return
    if a.tanner:
        tanner(a)
        return
    if a.sweep:
        sweep(a)
        return
    if a.hbm_probe:
        from paper_2503_20605_amd import probe_copy_bandwidth
        res = {"lb_hbm": lb_hbm_boxes(20), "batch256_d2q9_f16": batch_rate(20),
               "copy_1GiB_GBs": round(probe_copy_bandwidth(1 << 30, 5), 1)}
        print(json.dumps(res), flush=True)
        return
    storage = STORAGE[a.storage]
    W = workload_of(a.workload, a.run)
    if a.lam is not None and a.lam != W.params.lam:
        W.params.lam = a.lam
        W.name += f"_lam{a.lam:g}"
    p = W.params
    lam = float(p.lam)
    dim = p.dim
    cells = p.nx * p.ny * (p.nz if dim == 3 else 1)
    log(f"workload {W.name}, storage {a.storage}, {steps_arg(a)}")
    s = Solver([params_from(p)], [W.nodes], None if W.tris is None else [W.tris], storage=storage)
    if lam != 1.0:
        s.set_viscosity_ratio(0, lam)
    s.set_graph_steps(a.graph_steps)
    steps, warm = a.steps, a.warmup
    if a.profile_only:
        steps, warm = min(steps, 200), min(warm, 20)

    # untimed: pick the lattice-kernel variant (its steps are real steps of
    # the run, enough of them to replay the step graph twice per timing),
    # then the warm-up steps
    if a.variant < 0:
        variant, tune_ms = s.autotune(steps=2 * a.graph_steps + 2)
        tune_steps = len(tune_ms) * 2 * (2 * a.graph_steps + 2)
    else:
        variant, tune_ms, tune_steps = s.set_lb_variant(a.variant), None, 0
    s.step(warm)
    torch.cuda.synchronize()
    log(f"variant {variant}; timing {steps} steps")

    # timed region: exactly `steps` coupled steps launched directly on the
    # library's stream; every TIMING_STRIDE-th lattice launch (the first
    # included) is timed by the pair of HIP events its own dispatch marks
    # (events on every launch slow the whole step by about 3 %)
    s.set_timing(TIMING_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lb_ms, step_ms_events = s.last_timing()
    s.set_timing(False)
    ms_per_step = wall / steps * 1e3
    mlups = cells * steps / wall / 1e6

    # the same number of steps replayed from captured graphs (no events),
    # for comparison: graphs of min(steps - 2, graph steps) steps (even), a
    # call of `steps` steps timed five times after one untimed call that
    # builds the graphs it replays; the median is reported
    g = max(2, min(a.graph_steps, (steps - 2) // 2 * 2))
    s.set_graph_steps(g)
    s.step(steps)
    walls = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    wall_g = sorted(walls)[2]
    diag = s.diagnostics(0)
    bpc = bytes_per_cell(dim, storage)
    achieved = bpc * cells / (lb_ms * 1e-3) / 1e9
    lb_name = lb_kernel_name(dim, storage, variant, vis=int(lam != 1.0))
    traffic = measured_traffic(lb_name, W.name, LB_ORDER[variant // 16])

    out = {
        "metric": "MLUPS (coupled IB-LB step) + HBM GB/s fraction of the lattice kernel",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if storage == 0 else f"f32 compute, {a.storage} storage",
        "data": "synthetic (seeded droplet workload)",
        "config": {"workload": W.name,
                   "lattice": (f"D2Q9 {p.nx}x{p.ny}" if dim == 2
                               else f"D3Q19 {p.nx}x{p.ny}x{p.nz}"),
                   "nodes": len(W.nodes),
                   "triangles": None if W.tris is None else len(W.tris),
                   "viscosity_ratio": lam,
                   "tau": p.tau, "theta_eq_deg": p.theta_eq_deg, "sigma": p.sigma, "xi": p.xi,
                   "storage": a.storage, "lb_variant": variant, "block_order": LB_ORDER[variant // 16]},
        "roofline": {"kernel": lb_name + " (fused pull-stream + BGK + Guo)", "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "bytes_per_cell": bpc, "cells_per_launch": cells,
                     "lb_us_per_launch": round(lb_ms * 1e3, 3),
                     "timed_launches": len(range(0, steps - 1, TIMING_STRIDE)),
                     "timing_stride": TIMING_STRIDE,
                     "working_set_MB": round(bpc * cells / 1e6, 1)},
        "step_us_events": round(step_ms_events * 1e3, 3),
        "graph_replay": {"steps": steps, "graph_steps": g, "runs": len(walls),
                         "ms_per_step": round(wall_g / steps * 1e3, 5),
                         "MLUPS": round(cells * steps / wall_g / 1e6, 1),
                         "ms_per_step_runs": [round(w / steps * 1e3, 5) for w in walls]},
        "untimed_steps_before": tune_steps + warm,
        "autotune_step_ms": tune_ms,
        "diag": {"mass": diag["mass"], "theta_meas_deg": math.degrees(diag["theta_meas"]),
                 "volume": diag["volume"]},
    }
    s.close()

    log(f"{out['value']} MLUPS, lattice kernel {out['roofline']['lb_us_per_launch']} us "
        f"({out['roofline']['frac']} of peak)")
    if not a.profile_only:
        from paper_2503_20605_amd import probe_copy_bandwidth
        out["copy_probe_GBs"] = round(probe_copy_bandwidth(1 << 30, 20), 1)
        if not a.no_extra:
            log("secondary lines")
            out["extra"] = extra_workloads(a)
    if not a.no_cpu and not a.profile_only:
        log("CPU oracle baseline")
        # about 10 s of oracle work on one thread and 10 s on all of them
        n1, nn = (4, 40) if dim == 3 else (200, 2000)
        out["cpu_baseline"] = cpu_baseline(W, n1, nn)
    print(json.dumps(out), flush=True)


def steps_arg(a):
    return f"--steps {a.steps} --warmup {a.warmup}"


def workload_of(name, run=1):
    import workloads as wl
    if name == "d3q19":
        return wl.droplet_3d(theta_eq_deg=90.0, small=False)
    if name == "d3q19_spreading":
        return wl.droplet_3d_spreading(lam=10.0)
    return wl.droplet_2d_large(run=run)


def extra_workloads(a):
    """Secondary lines: the 1024x512 D2Q9 coupled step (its two population
    copies, 38 MB, fit the 256 MB last-level cache, so its GB/s is an
    effective figure) and the lattice kernel alone on boxes far above that
    cache in fp32 and fp16 storage."""
    import torch
    from paper_2503_20605_amd import Solver, params_from
    W = workload_of("d2q9", a.run)
    p = W.params
    s = Solver([params_from(p)], [W.nodes])
    v, _ = s.autotune(steps=130)
    s.step(200)
    s.set_timing(TIMING_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(2000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lb_ms, _ = s.last_timing()
    s.set_timing(False)
    s.set_graph_steps(64)
    s.step(2000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(2000)
    torch.cuda.synchronize()
    wall_g = time.perf_counter() - t0
    s.close()
    cells = p.nx * p.ny
    d2 = {"workload": W.name, "lb_variant": v, "steps": 2000,
          "MLUPS": round(cells * 2000 / wall / 1e6, 1),
          "MLUPS_graph_replay": round(cells * 2000 / wall_g / 1e6, 1),
          "lb_us": round(lb_ms * 1e3, 3),
          "effective_GBs": round(72 * cells / (lb_ms * 1e-3) / 1e9, 1)}
    return {"d2q9_1024x512_coupled": d2, "batch256_d2q9_f16": batch_rate(500),
            "lb_hbm": lb_hbm_boxes(100)}


def batch_rate(steps):
    """The 256-droplet batch of uneven 2D boxes (the time-to-equilibrium
    draws, seed 3) in one handle, fp16 storage: coupled steps per second and
    the lattice kernel's per-launch duration from the events its dispatch
    marks.  Its two population copies (about 470 MB) exceed the 256 MB
    last-level cache, so the GB/s is an HBM figure."""
    import torch
    import workloads as wl
    from paper_2503_20605_amd import STORAGE, Solver, params_from
    draws = wl.batch_draws(256, seed=3)
    s = Solver([params_from(w.params) for w in draws], [w.nodes for w in draws], storage=STORAGE["f16"])
    for d, w in enumerate(draws):
        s.set_node_respacing(d, w.params.respace)
    v, _ = s.autotune(steps=16)
    s.set_graph_steps(64)
    s.step(130)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    wall_g = time.perf_counter() - t0
    s.set_timing(TIMING_STRIDE)
    s.step(steps + 1)
    lb_ms, step_ms = s.last_timing()
    s.set_timing(False)
    status = max(s.diagnostics(d)["status"] for d in range(len(draws)))
    s.close()
    cells = sum(w.params.nx * w.params.ny for w in draws)
    bpc = bytes_per_cell(2, 1)
    gbs = bpc * cells / (lb_ms * 1e-3) / 1e9
    name = lb_kernel_name(2, 1, v, one=0)
    return {"workload": "batch256_seed3_d2q9_f16", "droplets": len(draws), "cells": cells,
            "working_set_MB": round(bpc * cells / 1e6, 1), "lb_variant": v, "block_order": LB_ORDER[v // 16],
            "MLUPS_graph_replay": round(cells * steps / wall_g / 1e6, 1),
            "step_us_events": round(step_ms * 1e3, 2), "lb_us": round(lb_ms * 1e3, 2),
            "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(name, "batch256_seed3_d2q9_f16", LB_ORDER[v // 16]),
            "status": status}


def lb_hbm_boxes(steps):
    """The lattice kernel alone on boxes whose two population copies far
    exceed the 256 MB last-level cache: D2Q9 8192x4096 and D3Q19
    256x256x128, fp32 and fp16 storage."""
    return [lb_only_rate(2, 8192, 4096, 1, 0, 2 * steps),
            lb_only_rate(2, 8192, 4096, 1, 1, 2 * steps),
            lb_only_rate(3, 256, 256, 128, 0, steps),
            lb_only_rate(3, 256, 256, 128, 1, steps)]


if __name__ == "__main__":
    main()
