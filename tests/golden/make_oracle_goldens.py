#!/usr/bin/env python3
"""Write stored expected values that are too slow to recompute in a test.

Every value here comes from the FP64 CPU oracle (oracle/) on the seeded
synthetic workloads of paper_2505_22256_amd.workloads; nothing is read from
the GPU library.

  cylinder_theta.json     droplet on a cylinder, 400x400, G_ads in
                          {-0.3 .. 0.3}, 20000 steps: contact angle (Sec. 3.2)
  calibration_theta.json  first 16 runs of the seeded calibration batch,
                          10000 steps: contact angle

Usage: python tests/golden/make_oracle_goldens.py [cylinder|calibration|all]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2505_22256_amd import workloads as W  # noqa: E402


def run(wl, steps):
    o = oracle.Oracle(wl.nx, wl.ny, wl.flags)
    o.set_geometry(wl.solid)
    o.set_params(wl.G_c, wl.G_ads, wl.tau)
    o.set_body_accel(*wl.accel)
    o.init_fields(wl.rho1, wl.rho2)
    o.step(steps)
    try:
        th = o.contact_angle(wl.wall_kind, wl.wall)
    except oracle.OracleError:
        th = None
    m = o.reduce()
    return th, m


def cylinder(steps=20000):
    out = {"_about": "FP64 oracle contact angle, droplet on a cylinder (400x400, R=60 at (200,150), "
                     "drop r=50 at (200,240), tau=1, G_c=0.9), after %d steps; written by "
                     "tests/golden/make_oracle_goldens.py" % steps, "steps": steps, "cases": []}
    for g in W.CYLINDER_SWEEP:
        t0 = time.time()
        th, m = run(W.cylinder_drop(G_ads=g), steps)
        out["cases"].append({"G_ads": g, "theta_deg": th, "mass1": m[0], "mass2": m[1], "max_u": m[4]})
        print(f"cylinder G_ads={g:+.2f} theta={th} ({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, "cylinder_theta.json"), "w") as f:
        json.dump(out, f, indent=1)


def calibration(n=16, steps=10000):
    runs = W.calibration_runs(steps=steps)[:n]
    out = {"_about": "FP64 oracle contact angle of the first %d runs of the seeded calibration batch "
                     "(seed 22256), after %d steps; written by tests/golden/make_oracle_goldens.py"
                     % (n, steps), "steps": steps, "runs": []}
    for r, wl in enumerate(runs):
        t0 = time.time()
        th, m = run(wl, steps)
        out["runs"].append({"index": r, "side": wl.nx, "wall_kind": wl.wall_kind, "G_ads": wl.G_ads,
                            "tau": wl.tau, "theta_deg": th, "mass1": m[0]})
        print(f"calibration run {r} side={wl.nx} kind={wl.wall_kind} theta={th} "
              f"({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, "calibration_theta.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("cylinder", "all"):
        cylinder()
    if what in ("calibration", "all"):
        calibration()
