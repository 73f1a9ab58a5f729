"""Study of the readings that set the wall-force scale, on the oracle alone
(CPU, FP64; a study script beside the tests, not collected by pytest and
not part of the product path).

The paper reports co-current flows within 1.84 % of their analytic
profiles (Sec. 3.1, Eq. 13-14) and spurious currents 50-70 % lower with the
improved adhesion for hydrophilic walls (Sec. 3.2, Fig. 10), without
stating the adhesion strength it used.  This script runs both checks under
alternative readings and prints one JSON line per case:

  * the weights of the adhesion sum S(x) of Eq. 9: the E8 weights (the
    library's reading) or the D2Q9 weights w_i (the oracle's ADH_D2Q9
    exploration flag);
  * the cohesion G_c: 0.9 (the run configurations) or 1.036 (which
    separates the paper's main and dissolved densities 1.02 / 0.05);
  * the adhesion scale G_w2: G_c, or the paper's G_12 = 0.17, with
    lambda = G_w1 / G_w2.

Usage:  python tests/study_readings.py cocurrent [steps]   (100 000 by default)
        python tests/study_readings.py spurious  [steps]   (20 000 by default)
Each case takes from one to several minutes on 8 cores.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import ADH_D2Q9, SCHEME_ORIGINAL, Oracle  # noqa: E402
from paper_2505_22256_amd import workloads as W  # noqa: E402  (seeded input generators only)

# (name, extra flags, G_c, G_w2 or None for G_w2 = G_c)
COCURRENT_READINGS = [
    ("E8, G_c=0.9", 0, 0.9, None),
    ("E8, G_c=1.036", 0, 1.036, None),
    ("D2Q9 w_i, G_c=0.9", ADH_D2Q9, 0.9, None),
    ("D2Q9 w_i, G_c=1.036", ADH_D2Q9, 1.036, None),
    ("E8, G_c=1.036, G_w2=0.17", 0, 1.036, 0.17),
    ("D2Q9 w_i, G_c=1.036, G_w2=0.17", ADH_D2Q9, 1.036, 0.17),
]


def cocurrent_error(flow: str, flags: int, G_c: float, G_w2, lam: float, steps: int) -> dict:
    """Largest deviation of the x-velocity profile (averaged along x) from
    the analytic one, relative to its peak: Couette, the line through the
    wall planes; Poiseuille, the parabola of the total force density and
    the mean total density."""
    wl = W.cocurrent(flow)
    o = Oracle(wl.nx, wl.ny, wl.flags | flags)
    o.set_geometry(wl.solid)
    if G_w2 is None:
        o.set_params(G_c, (lam - 1) * G_c / 2, wl.tau)
    else:
        o.set_params(G_c, 0.0, wl.tau)
        o.set_adhesion(lam * G_w2, G_w2, 0.8)
    o.set_body_accel(*wl.accel)
    if any(v != 0 for v in wl.wall_velocity):
        o.set_wall_velocity(*wl.wall_velocity)
    o.init_fields(wl.rho1, wl.rho2)
    o.step(steps)
    r1, r2, ux, _ = o.get_fields()
    prof = ux[1:-1].mean(axis=1)
    y = np.arange(1, wl.ny - 1) - (wl.ny - 1) / 2.0
    half = (wl.ny - 2) / 2.0
    if flow == "couette":
        ua = wl.wall_velocity[2] * y / half
    else:
        nu = (wl.tau - 0.5) / 3.0
        ua = wl.accel[0] / (nu * (r1 + r2)[1:-1].mean()) * (half ** 2 - y ** 2)
    return {"err": round(float(np.max(np.abs(prof - ua)) / np.max(np.abs(ua))), 4),
            "rho1_core": round(float(r1[wl.ny // 2, 0]), 4), "rho2_wall": round(float(r2[1, 0]), 4),
            "rho1_wall": round(float(r1[1, 0]), 4), "u_wall_row": float(prof[0])}


def spurious(flags: int, lam: float, steps: int) -> dict:
    """Droplet on the cylinder (the library's scheme-comparison case):
    contact angle, largest velocity (the spurious currents) and smallest
    rho_1 after `steps` steps, G_w2 = G_c = 0.9."""
    wl = W.cylinder_drop()
    o = Oracle(wl.nx, wl.ny, wl.flags | flags)
    o.set_geometry(wl.solid)
    o.set_params(wl.G_c, wl.G_ads, wl.tau)
    o.set_adhesion(lam * wl.G_c, wl.G_c, 0.8)
    o.init_fields(wl.rho1, wl.rho2)
    o.step(steps)
    m = o.reduce()
    try:
        th = round(o.contact_angle(wl.wall_kind, wl.wall), 3)
    except Exception:  # no fit: reported as missing
        th = None
    return {"theta": th, "max_u": float(m[4]), "min_rho1": float(m[5]), "nonfinite": int(m[7])}


def main(argv) -> int:
    what = argv[1] if len(argv) > 1 else "cocurrent"
    if what == "cocurrent":
        steps = int(argv[2]) if len(argv) > 2 else 100000
        for name, fl, gc, gw2 in COCURRENT_READINGS:
            for flow in ("couette", "poiseuille"):
                for lam in (0.6, 1.0, 1.4):
                    t0 = time.time()
                    row = {"reading": name, "flow": flow, "lambda": lam}
                    row.update(cocurrent_error(flow, fl, gc, gw2, lam, steps))
                    row["secs"] = round(time.time() - t0, 1)
                    print(json.dumps(row), flush=True)
    elif what == "spurious":
        steps = int(argv[2]) if len(argv) > 2 else 20000
        for rname, rfl in (("E8", 0), ("D2Q9 w_i", ADH_D2Q9)):
            for lam in (0.47, 0.6, 1.35, 1.6):
                for scheme, sfl in (("original", SCHEME_ORIGINAL), ("improved", 0)):
                    t0 = time.time()
                    row = {"reading": rname, "scheme": scheme, "lambda": lam}
                    row.update(spurious(rfl | sfl, lam, steps))
                    row["secs"] = round(time.time() - t0, 1)
                    print(json.dumps(row), flush=True)
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
