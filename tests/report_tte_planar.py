"""End angles of the time-to-equilibrium arms against the planar equilibrium.

Reads the per-droplet record that `bench.py --tte --dump FILE` writes and,
for every droplet at rest in an arm, compares the arm's end angle (from the
half-height) with that of the planar equilibrium outline (the App. B system
in two dimensions, at the droplet's own theta_eq and xi/R0, R0 from the
enclosed area).  The outline's continuation does not converge below
xi/R0 of about 0.06, and above theta_eq of about 145 deg it ends on the
detached branch (a full circle, half-height R0) where the simulated
droplets stay on the wall; those droplets are left out and counted.

    python3 tests/report_tte_planar.py FILE [--workers N]
"""
import argparse
import json
import math
import os
import sys
from multiprocessing import Pool

import numpy as np

sys.path[:0] = [os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                os.path.dirname(os.path.abspath(__file__))]
import oracle as o  # noqa: E402
import statics  # noqa: E402

EPS_MIN = 0.06
THETA_MAX_DEG = 145.0


def planar_angle(args):
    theta_eq_deg, eps = args
    if eps < EPS_MIN or theta_eq_deg > THETA_MAX_DEG:
        return None
    try:
        s = statics.theory_2d(math.radians(theta_eq_deg), eps)
    except RuntimeError:
        return None
    return math.degrees(o.angle_from_height_2d(s["ell"], math.pi))


def main(argv):
    ap = argparse.ArgumentParser()
    ap.add_argument("dump")
    ap.add_argument("--workers", type=int, default=6)
    a = ap.parse_args(argv)
    d = json.load(open(a.dump))
    draws = d["draws"]
    eps = [w["xi"] / math.sqrt(w["area"] / math.pi) for w in draws]
    with Pool(a.workers) as pool:
        ref = pool.map(planar_angle, [(w["theta_eq_deg"], e) for w, e in zip(draws, eps)])
    ok = [r is not None for r in ref]
    asked = sum(e >= EPS_MIN and w["theta_eq_deg"] <= THETA_MAX_DEG for w, e in zip(draws, eps))
    print(f"droplets {len(draws)}; with xi/R0 >= {EPS_MIN} and theta_eq <= {THETA_MAX_DEG} deg: {asked}; "
          f"planar outline solved for {sum(ok)}")
    print("| arm | at rest, outline solved | median abs(theta - planar) deg | 90th pct | max | "
          "median signed deg | above planar |")
    print("|---|---|---|---|---|---|---|")
    for k, arm in d["arms"].items():
        idx = [i for i in range(len(draws)) if ok[i] and arm["steps"][i] > 0]
        dv = np.array([arm["theta_deg"][i] - ref[i] for i in idx])
        if len(dv) == 0:
            continue
        ad = np.abs(dv)
        print(f"| {k} | {len(idx)} | {np.median(ad):.3f} | {np.percentile(ad, 90):.3f} | {ad.max():.3f} | "
              f"{np.median(dv):+.3f} | {int((dv > 0).sum())}/{len(dv)} |")


if __name__ == "__main__":
    main(sys.argv[1:])
