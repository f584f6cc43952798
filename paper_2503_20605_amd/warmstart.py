"""Learned warm start for 2D droplets on a wall.

A small network maps (theta_eq, area, tau, sigma) of a droplet to its
equilibrium: the interface as 256 radial offsets from the equal-area
circular cap of angle theta_eq, and the fluid velocity on a 32x16 grid over
the box.  It is trained on equilibria that the batched solver produces from
seeded parameter draws, with the library's own bf16 matrix-core kernels
(MLP).  Everything here is host-side data preparation; all simulation and
all network arithmetic run in the HIP library.

Geometry.  For a droplet in a box of width nx with the substrate at y = 0:
the reference point is the centroid of the equal-area cap of angle theta_eq
whose flat base lies on y = xi, centred at x = nx / 2.  A shape is stored as
its distance r(phi_k) from that point along 256 rays phi_k = 2 pi k / 256
(the equilibrium shapes are star-shaped about it).

Usage on the GPU:  python -m paper_2503_20605_amd.warmstart <out_dir> generate|train|evaluate
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

K_RAYS = 256
GRID = (16, 32)           # coarse velocity grid (rows in y, columns in x)
N_OUT = K_RAYS + 2 * GRID[0] * GRID[1]
WIDTHS = [4, 256, 256, 256, N_OUT]
U_SCALE = 1e4             # velocity targets are O(1e-6 .. 1e-4) lattice units
U_WEIGHT = 0.3            # weight of the (noise-dominated) velocity outputs in the loss
U_MAX = 1e-3              # predicted velocities are clipped to this magnitude
H_MIN = 0.85              # predicted nodes stay at least this many xi above the wall
MAX_TURN_DEG = 175.0      # a predicted outline turning more sharply than this folds back
PHI = 2.0 * math.pi * np.arange(K_RAYS) / K_RAYS
# rest criterion of the time-to-equilibrium runs (see Solver.run_to_rest):
# normal node speed below 1e-5 and the angle from the half-height steady
# within 0.01 deg over 10 checks 1000 steps apart
REST = dict(tol=1e-5, angle_tol_deg=0.01, check_every=1000, hold=10)


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------

def cap_outline(theta, area, xi, xc, n=4096):
    """Closed CCW outline of the circular cap of angle theta and the given
    area, base on y = xi centred at xc; also its circle radius."""
    rc = math.sqrt(area / (theta - math.sin(theta) * math.cos(theta)))
    yc = xi - rc * math.cos(theta)
    a = np.linspace(0.5 * math.pi - theta, 0.5 * math.pi + theta, n)
    arc = np.stack([xc + rc * np.cos(a), yc + rc * np.sin(a)], axis=1)
    half = rc * math.sin(theta)
    base = np.stack([np.linspace(xc - half, xc + half, n // 4)[1:-1],
                     np.full(n // 4 - 2, xi)], axis=1)
    return np.concatenate([arc, base]), rc


def polygon_centroid(q):
    x, y = q[:, 0], q[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    cr = x * yn - xn * y
    a = 0.5 * cr.sum()
    return np.array([((x + xn) * cr).sum(), ((y + yn) * cr).sum()]) / (6.0 * a)


def polygon_area(q):
    x, y = q[:, 0], q[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def radial_profile(q, p, phi=PHI):
    """Distance from p to the closed polygon q along each ray phi (the
    farthest crossing; a star-shaped outline has exactly one)."""
    a = q
    e = np.roll(q, -1, axis=0) - q
    d = np.stack([np.cos(phi), np.sin(phi)], axis=1)                  # (K, 2)
    ap = a - p                                                        # (N, 2)
    den = d[:, None, 0] * e[None, :, 1] - d[:, None, 1] * e[None, :, 0]
    with np.errstate(divide="ignore", invalid="ignore"):
        s = (ap[None, :, 0] * e[None, :, 1] - ap[None, :, 1] * e[None, :, 0]) / den
        u = (ap[None, :, 0] * d[:, None, 1] - ap[None, :, 1] * d[:, None, 0]) / den
    ok = (np.abs(den) > 1e-14) & (u >= 0) & (u <= 1) & (s > 0)
    s = np.where(ok, s, -np.inf)
    r = s.max(axis=1)
    if not np.all(np.isfinite(r)):
        raise ValueError("outline is not star-shaped about the reference point")
    return r


def reference(theta, area, xi, nx):
    """Reference point, cap profile and cap circle radius of a droplet."""
    cap, rc = cap_outline(theta, area, xi, nx / 2.0)
    p = polygon_centroid(cap)
    return p, radial_profile(cap, p), rc


def outline_from_profile(p, r, n_nodes, h_min):
    """n_nodes points, uniform in arc length, CCW, along the closed curve
    p + r_k (cos phi_k, sin phi_k); heights kept >= h_min."""
    z = p[None, :] + r[:, None] * np.stack([np.cos(PHI), np.sin(PHI)], axis=1)
    zc = np.concatenate([z, z[:1]])
    seg = np.linalg.norm(np.diff(zc, axis=0), axis=1)
    s = np.concatenate([[0.0], np.cumsum(seg)])
    t = np.arange(n_nodes) * (s[-1] / n_nodes)
    out = np.stack([np.interp(t, s, zc[:, 0]), np.interp(t, s, zc[:, 1])], axis=1)
    out[:, 1] = np.maximum(out[:, 1], h_min)
    return out


def coarse_velocity(U):
    """Block means of U (2, ny, nx) on the GRID (ny, nx multiples of it)."""
    _, ny, nx = U.shape
    gy, gx = GRID
    return U.reshape(2, gy, ny // gy, gx, nx // gx).mean(axis=(2, 4))


def fine_velocity(Uc, ny, nx):
    gy, gx = GRID
    return np.repeat(np.repeat(Uc, ny // gy, axis=1), nx // gx, axis=2)


def features(theta, area, tau, sigma):
    """Normalised network inputs."""
    return np.array([theta / math.pi, math.sqrt(area) / 100.0, (tau - 1.05) / 0.45,
                     (sigma - 0.006) / 0.004], dtype=np.float64)


# ---------------------------------------------------------------------------
# solver runs
# ---------------------------------------------------------------------------

def _solver(draws, storage):
    from . import Solver, params_from
    s = Solver([params_from(w.params) for w in draws], [w.nodes for w in draws], storage=storage)
    s.set_graph_steps(100)
    for d, w in enumerate(draws):
        beta = float(getattr(w.params, "respace", 0.0))
        if beta:
            s.set_node_respacing(d, beta)
    return s


def equilibrium_state(s, d, p):
    """Targets of droplet d of solver s at rest: offsets / rc and scaled
    velocity; also its area."""
    theta = math.radians(p.theta_eq_deg)
    q, _, _ = s.read_nodes(d)
    area = polygon_area(q)
    ref, rcap, rc = reference(theta, area, p.xi, p.nx)
    r = radial_profile(q, ref)
    _, U, _ = s.read_fields(d)
    Uc = coarse_velocity(U[:, 0].cpu().numpy().astype(np.float64))
    return np.concatenate([(r - rcap) / rc, U_SCALE * Uc.ravel()]), area


def rest_args(tol, rest):
    """Arguments of Solver.run_to_rest: the normal-speed criterion alone
    (checks every 100 steps, held for 10) unless `rest` gives others."""
    a = dict(tol=tol, check_every=100, hold=10, angle_tol_deg=0.0)
    a.update(rest or {})
    return a


def generate(draws, storage=1, max_steps=100000, tol=1e-6, batch=256, log=print, rest=None):
    """Run every draw from its 90-degree start to rest (or max_steps) and
    return (inputs (n, 4), targets (n, N_OUT), steps (n,))."""
    import torch
    X, Y, S = [], [], []
    for b0 in range(0, len(draws), batch):
        part = draws[b0:b0 + batch]
        s = _solver(part, storage)
        s.autotune(steps=20)
        s.init_rest(-1)
        for d, w in enumerate(part):
            s.set_interface(d, w.nodes)
        t0 = time.perf_counter()
        steps = s.run_to_rest(max_steps=max_steps, **rest_args(tol, rest))
        torch.cuda.synchronize()
        log(f"[generate] droplets {b0}..{b0 + len(part) - 1}: {time.perf_counter() - t0:.1f} s, "
            f"at rest {sum(1 for x in steps if x > 0)}/{len(part)}")
        skipped = 0
        for d, w in enumerate(part):
            if steps[d] == -2:
                skipped += 1
                continue
            try:
                tgt, area = equilibrium_state(s, d, w.params)
            except ValueError:      # outline not star-shaped about the reference
                skipped += 1
                continue
            p = w.params
            X.append(features(math.radians(p.theta_eq_deg), area, p.tau, p.sigma))
            Y.append(tgt)
            S.append(steps[d])
        if skipped:
            log(f"[generate] skipped {skipped} droplets (unstable or not star-shaped)")
        s.close()
    return np.array(X), np.array(Y), np.array(S)


def _init_params(widths, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(widths) - 1):
        bound = 1.0 / math.sqrt(widths[l])
        parts.append(rng.uniform(-bound, bound, size=widths[l] * widths[l + 1]))
        parts.append(np.zeros(widths[l + 1]))
    return np.concatenate(parts).astype(np.float32)


def fit(X, Y, steps=4000, lr=1e-3, seed=7, log=print):
    """Full-batch Adam on the device with the library's network kernels.
    Each output is standardised over the training set (targets clipped to
    5 standard deviations; the velocity outputs scaled down by U_WEIGHT so
    that the interface shape dominates the loss); the learning rate decays
    linearly to 5 %.
    Returns the network, its output scaling (mean, std) and the loss
    history."""
    from . import MLP
    mu = Y.mean(axis=0)
    sd = np.maximum(Y.std(axis=0), 1e-6)
    sd[K_RAYS:] /= U_WEIGHT    # smaller standardised velocity targets weigh less
    Z = np.clip((Y - mu) / sd, -5.0, 5.0)
    m = MLP(WIDTHS, X.shape[0])
    m.set_params(_init_params(WIDTHS, seed))
    x = m._dev(X)
    z = m._dev(Z)
    hist = []
    for k in range(steps):
        loss = m.train_step(x, z, lr * (1.0 - 0.95 * k / steps))
        if k % 500 == 0 or k == steps - 1:
            hist.append((k, loss))
            log(f"[train] step {k} loss {loss:.4e}")
    return m, (mu, sd), hist


def max_turn_deg(q):
    """Largest turning angle (degrees) between consecutive edges of the
    closed outline q: 180 - theta at a contact corner of angle theta, 180
    where the outline folds back on itself."""
    e = np.roll(q, -1, axis=0) - q
    a = np.arctan2(e[:, 1], e[:, 0])
    turn = np.abs((np.roll(a, -1) - a + math.pi) % (2.0 * math.pi) - math.pi)
    return float(np.degrees(turn.max()))


def predict_starts(m, scale, draws):
    """Initial outlines and fluid velocity fields predicted by the network
    (scale: the output mean and std of fit).  Keeping the nodes above the
    wall can fold the predicted outline of a flat droplet back on itself
    near its contact line (a spike of zero width, which no solver step
    survives); such a start is replaced by the analytic prior (cap_starts)
    before anything runs.  Returns the starts and the indices replaced."""
    X = np.array([features(math.radians(w.params.theta_eq_deg), polygon_area(w.nodes),
                           w.params.tau, w.params.sigma) for w in draws])
    out = m.forward(X).cpu().numpy().astype(np.float64) * scale[1] + scale[0]
    starts = []
    for w, o in zip(draws, out):
        p = w.params
        theta = math.radians(p.theta_eq_deg)
        area = polygon_area(w.nodes)
        ref, rcap, rc = reference(theta, area, p.xi, p.nx)
        r = np.maximum(rcap + rc * o[:K_RAYS], 0.05 * rc)
        q = outline_from_profile(ref, r, len(w.nodes), H_MIN * p.xi)
        Uc = np.clip(o[K_RAYS:].reshape(2, *GRID) / U_SCALE, -U_MAX, U_MAX)
        starts.append((q, fine_velocity(Uc, p.ny, p.nx), rc))
    rejected = [i for i, st in enumerate(starts) if max_turn_deg(st[0]) > MAX_TURN_DEG]
    if rejected:
        prior = cap_starts([draws[i] for i in rejected])
        for k, i in enumerate(rejected):
            starts[i] = prior[k]
    return starts, rejected


def cap_starts(draws):
    """The analytic prior: the equal-area cap at theta_eq, fluid at rest."""
    starts = []
    for w in draws:
        p = w.params
        theta = math.radians(p.theta_eq_deg)
        area = polygon_area(w.nodes)
        ref, rcap, rc = reference(theta, area, p.xi, p.nx)
        q = outline_from_profile(ref, rcap, len(w.nodes), H_MIN * p.xi)
        starts.append((q, np.zeros((2, p.ny, p.nx)), rc))
    return starts


def inside_mask(q, ny, nx):
    """Cells whose centre lies inside the closed outline q (even-odd rule),
    one row of cell centres at a time."""
    inside = np.zeros((ny, nx), dtype=bool)
    x0, y0 = q[:, 0], q[:, 1]
    x1, y1 = np.roll(x0, -1), np.roll(y0, -1)
    xc = np.arange(nx) + 0.5
    lo = max(int(np.floor(y0.min())), 0)
    hi = min(int(np.ceil(y0.max())) + 1, ny)
    for j in range(lo, hi):
        y = j + 0.5
        sel = (np.minimum(y0, y1) <= y) & (np.maximum(y0, y1) > y)
        if not np.any(sel):
            continue
        xs = x0[sel] + (y - y0[sel]) * (x1[sel] - x0[sel]) / (y1[sel] - y0[sel])
        inside[j] = (np.searchsorted(np.sort(xs), xc) % 2) == 1
    return inside


def run_from(draws, starts, storage, max_steps, tol=1e-6, log=print, rest=None):
    """Run the batch to rest from given starts (None: the 90-degree caps at
    rest).  Returns wall seconds, steps, measured angles, final outlines."""
    import torch
    s = _solver(draws, storage)
    s.autotune(steps=20)
    s.init_rest(-1)
    for d, w in enumerate(draws):
        if starts is None:
            s.set_interface(d, w.nodes)
        else:
            q, U, rc = starts[d]
            p = w.params
            s.set_interface(d, q)
            drho = 3.0 * p.sigma / rc        # Laplace jump sigma / R, p = rho / 3
            rho = 1.0 + drho * inside_mask(q, p.ny, p.nx)
            s.init_fields(d, rho[None].astype(np.float32), U[:, None].astype(np.float32))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = s.run_to_rest(max_steps=max_steps, **rest_args(tol, rest))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dg = s.diagnostics(-1)
    finals = [s.read_nodes(d)[0] for d in range(len(draws))]
    s.close()
    return wall, steps, [math.degrees(x["theta_meas"]) for x in dg], finals


def shape_error(q_start, q_final, ref):
    """2D counterpart of E_L2 (eq. L2-error_equilibrium) over phi in [0, 2 pi)."""
    a = radial_profile(q_start, ref)
    b = radial_profile(q_final, ref)
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def evaluate_arms(draws, m, scale, max_steps, log=print, rest=None):
    """Run the draws to rest four ways: plain fp32 from the 90-degree cap,
    fp16 from the 90-degree cap, fp16 from the analytic equal-area cap, fp16
    from the network's start (predicted outlines that fold replaced by the
    analytic cap beforehand); plus the learned arm with every start that
    turned unstable rerun from the analytic cap (its wall time charged to
    the learned arm)."""
    res = {}
    arms = [("plain_f32_90deg", 0, None), ("f16_90deg", 1, None),
            ("f16_cap_prior", 1, cap_starts(draws))]
    learned, rejected = predict_starts(m, scale, draws)
    arms.append(("f16_learned", 1, learned))
    for name, storage, starts in arms:
        wall, steps, ang, finals = run_from(draws, starts, storage, max_steps, log=log, rest=rest)
        res[name] = dict(wall=wall, steps=steps, theta=ang, finals=finals, starts=starts,
                         rejected=rejected if name == "f16_learned" else [])
        log(f"[evaluate] {name}: {wall:.1f} s, at rest {sum(1 for x in steps if x > 0)}/"
            f"{len(steps)}")
    lr = res["f16_learned"]
    bad = [i for i, x in enumerate(lr["steps"]) if x == -2]
    fb = dict(lr, steps=list(lr["steps"]), theta=list(lr["theta"]), finals=list(lr["finals"]),
              fallback=len(bad))
    if bad:
        sub = [draws[i] for i in bad]
        wall2, steps2, ang2, fin2 = run_from(sub, cap_starts(sub), 1, max_steps, log=log, rest=rest)
        fb["wall"] = lr["wall"] + wall2
        for k, i in enumerate(bad):
            fb["steps"][i], fb["theta"][i], fb["finals"][i] = steps2[k], ang2[k], fin2[k]
        log(f"[evaluate] f16_learned_with_fallback: {len(bad)} droplets rerun from the cap, "
            f"+{wall2:.1f} s")
    res["f16_learned_with_fallback"] = fb
    return res


def summarize(draws, res, max_steps):
    """Per arm: wall time, droplets at rest, paired step and work ratios
    against the plain arm over the droplets at rest in both, angles against
    the plain arm, the start's shape error against the plain final shape."""
    plain = res["plain_f32_90deg"]
    summary = {"droplets": len(draws), "max_steps": max_steps}
    for name, r in res.items():
        conv = [i for i, x in enumerate(r["steps"]) if x > 0]
        both = [i for i in conv if plain["steps"][i] > 0]
        dth = np.abs(np.array(r["theta"])[both] - np.array(plain["theta"])[both]) if both \
            else np.zeros(0)
        e = {"wall_s": round(r["wall"], 2), "at_rest": len(conv),
             "fallback_reruns": r.get("fallback", 0),
             "folded_starts_replaced_by_cap": len(r.get("rejected", [])),
             "unstable": sum(1 for x in r["steps"] if x == -2),
             "median_steps": float(np.median([r["steps"][i] for i in conv])) if conv else None,
             "theta_vs_plain_within_1deg": int((dth < 1.0).sum()),
             "theta_vs_plain_compared": len(both),
             "theta_vs_plain_max_deg": round(float(dth.max()), 3) if len(dth) else None}
        if both:
            ratio = [r["steps"][i] / plain["steps"][i] for i in both]
            cells = [draws[i].params.nx * draws[i].params.ny for i in both]
            e["paired_at_rest"] = len(both)
            e["paired_median_step_ratio"] = round(float(np.median(ratio)), 4)
            e["paired_work_ratio"] = round(
                sum(c * r["steps"][i] for c, i in zip(cells, both))
                / sum(c * plain["steps"][i] for c, i in zip(cells, both)), 4)
        starts = r["starts"] if r["starts"] is not None else [(w.nodes, None, None) for w in draws]
        errs = []
        for i, w in enumerate(draws):
            p = w.params
            ref, _, _ = reference(math.radians(p.theta_eq_deg), polygon_area(w.nodes), p.xi, p.nx)
            try:
                errs.append(shape_error(starts[i][0], plain["finals"][i], ref))
            except ValueError:
                pass
        e["start_shape_error_median"] = float(np.median(errs)) if errs else None
        summary[name] = e
    summary["speedup_learned_f16_vs_plain_f32"] = round(
        res["plain_f32_90deg"]["wall"] / res["f16_learned"]["wall"], 3)
    summary["speedup_learned_f16_with_fallback_vs_plain_f32"] = round(
        res["plain_f32_90deg"]["wall"] / res["f16_learned_with_fallback"]["wall"], 3)
    return summary


def main(argv):
    out_dir, what = argv[1], argv[2]
    os.makedirs(out_dir, exist_ok=True)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as wl

    def log(msg):
        print(msg, flush=True)

    if what == "generate":
        n_train = int(os.environ.get("IBLB_WARM_TRAIN", "4096"))
        draws = wl.batch_draws(n_train, seed=5)
        X, Y, S = generate(draws, storage=1,
                           max_steps=int(os.environ.get("IBLB_WARM_GEN_STEPS", "800000")), log=log,
                           rest=REST)
        np.savez(os.path.join(out_dir, "train.npz"), X=X.astype(np.float32),
                 Y=Y.astype(np.float32), S=S)
        log(f"[generate] saved {len(X)} equilibria")
    elif what == "train":
        d = np.load(os.environ.get("IBLB_WARM_DATA", os.path.join(out_dir, "train.npz")))
        t0 = time.perf_counter()
        m, scale, hist = fit(d["X"].astype(np.float64), d["Y"].astype(np.float64),
                             steps=int(os.environ.get("IBLB_WARM_STEPS", "8000")), log=log)
        np.savez(os.path.join(out_dir, "net.npz"), params=m.get_params(), mu=scale[0], sd=scale[1])
        json.dump({"loss": hist, "seconds": time.perf_counter() - t0},
                  open(os.path.join(out_dir, "train.json"), "w"))
    elif what == "evaluate":
        from . import MLP
        max_steps = int(os.environ.get("IBLB_WARM_EVAL_STEPS", "800000"))
        n_test = int(os.environ.get("IBLB_WARM_TEST", "512"))
        draws = wl.batch_draws(n_test, seed=6)
        m = MLP(WIDTHS, n_test)
        net = np.load(os.path.join(out_dir, "net.npz"))
        m.set_params(net["params"])
        scale = (net["mu"], net["sd"])
        res = evaluate_arms(draws, m, scale, max_steps, log=log, rest=REST)
        summary = summarize(draws, res, max_steps)
        json.dump(summary, open(os.path.join(out_dir, "evaluate.json"), "w"), indent=1)
        log(json.dumps(summary))
    else:
        raise SystemExit(f"unknown step {what}")


if __name__ == "__main__":
    main(sys.argv)
