#!/usr/bin/env python3
"""Throughput benchmark of the two-component pseudopotential LBM hot path.

One step = one lattice time step of the fused kernel (pull streaming with
bounce-back, densities, E8 cohesion with the second-layer copy, local
adhesion, body force, BGK-Guo collision, store), with the FP64 diagnostics
fused into every 100th step.  With the FP32 default tile two steps run per
launch (the first step's post-collision rows stay in LDS), so HBM moves
fewer bytes per update than the one-step algorithmic count the roofline
uses; `roofline.hbm_bytes_per_update` gives the measured figure.  Workload: the 16384 x 2048 walled microchannel
with 64 square constrictions (side 128), two components as parallel streams,
G_c = 0.9, G_ads = 0.15, tau = 1, body acceleration 2e-6 on both, FP32
deviation storage.  Inputs are resident in HBM before the timed region.

Prints one JSON line: MLUPS (fluid-node updates per second, both components
per update), the HBM roofline fraction of the step kernel (algorithmic
bytes: 2 x 9 populations x (read + write) + 1 byte of geometry per fluid
update), the FP64 CPU oracle on a bounded sample as a baseline, and the
contact-angle error of the reduced-precision storages on the flat-wall
droplet against the FP64 path.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2505_22256_amd import lbm, workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "2-comp D2Q9 MLUPS, % of HBM roofline, contact-angle error vs FP64 oracle"
STORAGES = {"f64": lbm.F64, "f32": lbm.F32, "f16": lbm.F16, "bf16": lbm.BF16}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_constrictions.json")


def rounding_label(args) -> str:
    if args.storage not in ("f16", "bf16"):
        return ""
    return " round-to-nearest-even" if args.nearest else " stochastic rounding"


def copy_bandwidth(nbytes: int = 1 << 31, repeats: int = 5):
    """Read+write bandwidth of a plain device copy (torch's copy kernel) of
    `nbytes`, the best of `repeats` timed copies: what the box delivers for
    the simplest streaming pattern, the practical ceiling beside the 8 TB/s
    peak."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return round(2.0 * 4 * n / (best * 1e-3) / 1e9, 1)


def kernel_source_hash() -> str:
    """Hash of the sources that define the step kernel and its launch
    geometry (the tile is checked separately)."""
    h = hashlib.sha256()
    for name in ("lbm_device.hpp", "lbm_kernels.hpp", "lbm_params.hpp"):
        with open(os.path.join(ROOT, "paper_2505_22256_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    # the compiler flags shape the kernels too
    from paper_2505_22256_amd import build as _build
    h.update(" ".join(_build.FLAGS[:-4]).encode())
    return h.hexdigest()[:16]


def measured_traffic(storage_name: str, tile):
    """HBM bytes per step launch from the committed rocprofv3 counter runs,
    only while they were taken on the current kernel source and tile."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(storage_name)
    if not ent or rec.get("kernel_hash") != kernel_source_hash() or list(ent.get("tile", [])) != list(tile):
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(wl, seconds: float = 12.0, single_seconds: float = 6.0):
    """FP64 oracle on a bounded sample of the same workload: the first 1024
    columns of the channel (periodic in x), stepped until `seconds` pass on
    all the host threads it uses, then for `single_seconds` on one thread
    (the per-core figure)."""
    import oracle  # the oracle: CPU baseline only
    oracle.build(force=False)
    w = 1024
    o = oracle.Oracle(w, wl.ny, wl.flags)
    o.set_geometry(wl.solid[:, :w])
    o.set_params(wl.G_c, wl.G_ads, wl.tau)
    o.set_body_accel(*wl.accel)
    o.init_fields(wl.rho1[:, :w], wl.rho2[:, :w])
    o.step(1)
    nf = int(w * wl.ny - wl.solid[:, :w].sum())

    def timed(limit):
        steps, t0 = 0, time.perf_counter()
        while True:
            o.step(2)
            steps += 2
            el = time.perf_counter() - t0
            if el >= limit:
                return steps, el

    cores = oracle.threads()
    steps, el = timed(seconds)
    prev = oracle.set_threads(1)
    steps1, el1 = timed(single_seconds)
    oracle.set_threads(prev)
    return {"value": round(nf * steps / el / 1e6, 3), "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "single_core_value": round(nf * steps1 / el1 / 1e6, 3),
            "sample": f"constriction channel columns 0..{w - 1} x {wl.ny} rows (periodic in x), "
                      f"{steps} FP64 steps in {el:.1f} s on {cores} threads, {steps1} in {el1:.1f} s on one"}


def precision_check(steps: int = 5000):
    """Contact angle of the flat-wall droplet (100x50, lambda = 13/9) after
    `steps` steps per storage, against the FP64 path (which agrees with the
    FP64 oracle to 1e-12)."""
    wl = W.flat_drop()
    cases = [("f64", lbm.F64, 0), ("f32", lbm.F32, 0), ("f16", lbm.F16, 0),
             ("f16_rne", lbm.F16, lbm.ROUND_NEAREST), ("bf16", lbm.BF16, 0),
             ("bf16_rne", lbm.BF16, lbm.ROUND_NEAREST)]
    th = {}
    for name, st, fl in cases:
        g = lbm.lattice_from_workload(wl, st, fl)
        g.step(steps)
        try:
            th[name] = g.contact_angle(wl.wall_kind, wl.wall)
        except lbm.LbmError:
            th[name] = float("nan")
        g.close()
    ref = th["f64"]
    return {"workload": f"flat-wall droplet 100x50, {steps} steps", "theta_f64_deg": round(ref, 4),
            "theta_err_deg": {k: (round(abs(v - ref), 4) if math.isfinite(v) else None)
                              for k, v in th.items() if k != "f64"}}


def calibration_batch(args):
    """The 512-run contact-angle calibration batch (seed 22256): square
    lattices of side 128..512, flat or cylinder walls, per-run G_ads and tau,
    one launch per step over all runs, HIP graph replays, autotuned tile
    (or the one --tile names).
    With --full, runs the configured 10000 steps and reports the angles
    (and their difference from the FP64 oracle values stored for the first
    16 runs)."""
    import torch
    runs = W.calibration_runs()
    storage = STORAGES[args.storage]
    flags = lbm.ROUND_NEAREST if args.nearest else 0
    for wl in runs:
        wl.flags |= flags
    stream = torch.cuda.Stream()
    b = lbm.Batch(runs, storage)
    b.set_stream(stream.cuda_stream)
    if args.tile in ("default", "auto"):
        tile = b.autotune(4)
    else:
        # a fixed tile (block, seg_rows, sched), e.g. to profile one kernel
        vals = [int(v) for v in args.tile.split(",")]
        b.set_tile(vals[0], vals[1])
        b.set_sched(vals[2] if len(vals) > 2 else 0)
        tile = b.get_tile() + (b.sched,)
    b.use_graph(True, 50)
    n_fluid = b.fluid_nodes
    steps = runs[0].steps if args.full else args.steps
    warm = 0 if args.full else args.warmup
    with torch.cuda.stream(stream):
        b.step(warm)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        b.step(steps)
        ev1.record(stream)
        ev1.synchronize()
    ms = ev0.elapsed_time(ev1)
    mlups = n_fluid * steps / (ms * 1e-3) / 1e6
    out = {"metric": "calibration batch MLUPS (fluid-node updates per second over all runs)",
           "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": warm,
           "ms_per_step": round(ms / steps, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if storage == lbm.F64 else "f32", "data": "synthetic",
           "config": {"workload": f"calibration batch: {len(runs)} runs, sides 128..512, flat/cylinder, "
                                  f"seed 22256, {args.storage} storage" + rounding_label(args),
                      "runs": len(runs), "fluid_nodes": n_fluid,
                      "tile": {"block": tile[0], "seg_rows": tile[1], "sched": tile[2]},
                      "graph_steps": 50}}
    if args.full:
        th = b.contact_angles()
        out["theta_deg"] = {"finite": int(np.isfinite(th).sum()), "min": float(np.nanmin(th)),
                            "max": float(np.nanmax(th))}
        gold = os.path.join(ROOT, "tests", "golden", "calibration_theta.json")
        if os.path.exists(gold):
            with open(gold) as f:
                ref = json.load(f)["runs"]
            errs = [abs(th[r["index"]] - r["theta_deg"]) for r in ref if r["theta_deg"] is not None]
            out["theta_vs_oracle_first_runs"] = {"runs": len(errs), "max_abs_err_deg": round(max(errs), 4),
                                                 "mean_abs_err_deg": round(float(np.mean(errs)), 4)}
    b.close()
    print(json.dumps(out), flush=True)


def saturation_and_front(wl, rho1, rho2):
    """Saturation S1 = fraction of fluid nodes with rho^e > 0, and front
    X_f = last column of the run of columns from x = 0 whose fluid nodes have
    rho^e > 0 for at least half (the channel is periodic in x, so component
    1 that leaks backwards across the seam does not count as the front)."""
    fluid = wl.solid == 0
    pos = fluid & (rho1 > rho2)
    s1 = float(pos.sum()) / float(fluid.sum())
    nf = fluid.sum(axis=0)
    frac = np.where(nf > 0, pos.sum(axis=0) / np.maximum(nf, 1), 1.0)
    low = np.nonzero(frac < 0.5)[0]
    return s1, int(low[0]) - 1 if len(low) else wl.nx - 1


def porous_precision(args):
    """Immiscible displacement in the 2048x1024 porous channel (seed 2505):
    every storage runs the configured steps, recording saturation and front
    every `--record-every` steps, compared with the FP64 device run (which
    the oracle anchors in the GPU tests)."""
    import torch
    wl = W.porous()
    steps = args.steps if args.steps_given else wl.steps
    every = args.record_every
    cases = [("f64", lbm.F64, 0), ("f32", lbm.F32, 0), ("f16", lbm.F16, 0),
             ("f16_rne", lbm.F16, lbm.ROUND_NEAREST), ("bf16", lbm.BF16, 0),
             ("bf16_rne", lbm.BF16, lbm.ROUND_NEAREST)]
    hist, rate = {}, {}
    stream = torch.cuda.Stream()
    for name, st, fl in cases:
        g = lbm.lattice_from_workload(wl, st, fl)
        g.set_stream(stream.cuda_stream)
        g.autotune(2)
        rec, t_gpu = [], 0.0
        for t in range(0, steps, every):
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            g.step(every)
            ev1.record(stream)
            ev1.synchronize()
            t_gpu += ev0.elapsed_time(ev1)
            r1, r2, _, _ = g.get_fields()
            rec.append(saturation_and_front(wl, r1, r2))
        hist[name] = rec
        rate[name] = round(g.fluid_nodes * steps / (t_gpu * 1e-3) / 1e6, 1)
        g.close()
        print(f"[porous] {name}: S1 {rec[-1][0]:.5f} front {rec[-1][1]} ({rate[name]} MLUPS)", file=sys.stderr,
              flush=True)
    ref = hist["f64"]
    out = {"metric": "porous displacement: saturation and front vs FP64", "workload":
           f"porous 2048x1024 (seed 2505, {len(wl.disks)} disks, porosity "
           f"{1 - wl.solid[:, 96:].mean():.3f}), component 1 driven by 1e-6 from x < 64, {steps} steps, "
           f"recorded every {every}", "fluid_nodes": wl.n_fluid,
           "f64_final": {"S1": ref[-1][0], "front_x": ref[-1][1]}, "storages": {}}
    for name, rec in hist.items():
        if name == "f64":
            continue
        ds = max(abs(a[0] - b[0]) for a, b in zip(rec, ref))
        dx = max(abs(a[1] - b[1]) for a, b in zip(rec, ref))
        out["storages"][name] = {"max_abs_dS1": round(ds, 6), "max_abs_dfront": dx, "MLUPS": rate[name]}
    out["f64_MLUPS"] = rate["f64"]
    out["history"] = {k: [[round(a, 6), b] for a, b in v] for k, v in hist.items()}
    print(json.dumps(out), flush=True)


def cylinder_sweep(args):
    """The droplet-on-cylinder sweep (400x400, seven adhesion values, 20000
    steps) in every storage, against the FP64 oracle angles stored in
    tests/golden/cylinder_theta.json (written from the oracle alone)."""
    with open(os.path.join(ROOT, "tests", "golden", "cylinder_theta.json")) as f:
        ref = json.load(f)
    cases = [("f64", lbm.F64, 0), ("f32", lbm.F32, 0), ("f16", lbm.F16, 0),
             ("f16_rne", lbm.F16, lbm.ROUND_NEAREST), ("bf16", lbm.BF16, 0),
             ("bf16_rne", lbm.BF16, lbm.ROUND_NEAREST)]
    rows = []
    for c in ref["cases"]:
        wl = W.cylinder_drop(G_ads=c["G_ads"])
        row = {"G_ads": c["G_ads"], "theta_oracle": round(c["theta_deg"], 4)}
        for name, st, fl in cases:
            g = lbm.lattice_from_workload(wl, st, fl)
            g.step(ref["steps"])
            try:
                row[name] = round(abs(g.contact_angle(wl.wall_kind, wl.wall) - c["theta_deg"]), 4)
            except lbm.LbmError:
                row[name] = None
            g.close()
        rows.append(row)
        print(f"[cylinder] {row}", file=sys.stderr, flush=True)
    worst = {name: max(r[name] for r in rows if r[name] is not None) for name, _, _ in cases}
    print(json.dumps({"metric": "cylinder sweep: |theta - theta_oracle| (deg) per storage",
                      "workload": f"droplet on a cylinder, 400x400, {ref['steps']} steps, G_ads in "
                                  f"{[r['G_ads'] for r in rows]}",
                      "worst_abs_err_deg": worst, "cases": rows}), flush=True)


def scheme_comparison(args):
    """Original (constant G_w1) against improved (local G(x), Eq. 11)
    adhesion on the droplet-on-cylinder case, swept over lambda = G_w1 /
    G_w2 with G_w2 = G_c: contact angle, largest velocity (the spurious
    currents of Sec. 3.2), smallest and largest rho_1, and the mean rho_1
    on the wall under the cylinder, far from the droplet (the mass-transfer
    layer: the dissolved level there is 0.098 without one)."""
    lams = [0.26, 0.35, 0.47, 0.6, 0.88, 1.0, 1.2, 1.35, 1.6]
    steps = args.steps if args.steps_given else 20000
    storage = STORAGES[args.storage]
    wl = W.cylinder_drop()
    cx, cy, Rs = wl.wall
    y, x = np.mgrid[0:wl.ny, 0:wl.nx]
    dist = np.hypot(x - cx, y - cy) - (Rs - 0.5)
    band = (wl.solid == 0) & (dist < 1.5) & (y < cy - 0.5 * (Rs - 0.5))
    rows = []
    for scheme, fl in (("original", lbm.SCHEME_ORIGINAL), ("improved", 0)):
        for lam in lams:
            g = lbm.lattice_from_workload(wl, storage, fl)
            g.set_adhesion(lam * wl.G_c, wl.G_c, 0.8)
            g.step(steps)
            m = g.reduce()
            try:
                th = round(g.contact_angle(wl.wall_kind, wl.wall), 3)
            except lbm.LbmError:
                th = None
            r1 = g.get_fields()[0]
            row = {"scheme": scheme, "lambda": lam, "theta_deg": th, "max_u": float(m[4]),
                   "min_rho1": float(m[5]), "max_rho1": float(m[6]),
                   "wall_rho1_below": round(float(r1[band].mean()), 5), "nonfinite": int(m[7])}
            rows.append(row)
            g.close()
            print(f"[schemes] {row}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "original vs improved adhesion: angle, spurious currents, density extremes, "
                                "wall layer", "workload": f"droplet on a cylinder 400x400, {steps} steps, "
                                f"{args.storage} storage, G_w2 = G_c = 0.9, delta = 0.8", "rows": rows}), flush=True)


def _timed_steps(lat, stream, steps, warmup):
    import torch
    with torch.cuda.stream(stream):
        lat.step(warmup)
        lat.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        lat.step(steps)
        ev1.record(stream)
        ev1.synchronize()
    return ev0.elapsed_time(ev1)


def open_channel(args):
    """The constriction channel with its x edges opened (Zou-He inlet with a
    Poiseuille profile at x = 0, outflow at x = nx-1) against the periodic
    channel, same storage, each at the library's default tile (or both at
    --tile): the cost of the open boundaries on the hot path."""
    import torch
    storage = STORAGES[args.storage]
    steps = args.steps if args.steps_given else 1000
    flags = lbm.ROUND_NEAREST if args.nearest else 0
    out = {}
    for name, wl in (("periodic", W.constrictions()), ("open", W.constrictions(open_ends=True))):
        stream = torch.cuda.Stream()
        lat = lbm.lattice_from_workload(wl, storage, flags)
        lat.set_stream(stream.cuda_stream)
        if args.tile not in ("default", "auto"):
            vals = [int(v) for v in args.tile.split(",")]
            lat.set_tile(vals[0], vals[1], vals[2] if len(vals) > 2 else 0)
        ms = _timed_steps(lat, stream, steps, args.warmup)
        m = lat.reduce()
        out[name] = {"MLUPS": round(lat.fluid_nodes * steps / (ms * 1e-3) / 1e6, 1),
                     "ms_per_step": round(ms / steps, 4), "tile": list(lat.get_tile()),
                     "mass1": float(m[0]), "mass2": float(m[1]), "max_u": float(m[4]),
                     "nonfinite": int(m[7])}
        lat.close()
        print(f"[open] {name} {out[name]}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "open vs periodic constriction channel MLUPS",
                      "workload": f"constrictions 16384x2048, {args.storage} storage{rounding_label(args)}, {steps} steps; open: Zou-He "
                                  "inlet (Poiseuille, peak 0.01) + outflow", "storage": args.storage,
                      "runs": out, "open_over_periodic": round(out["open"]["MLUPS"] / out["periodic"]["MLUPS"], 4)}),
          flush=True)


def cocurrent_flow(args):
    """Co-current two-layer flow between walls (Sec. 3.1): Couette (walls
    sliding at -+0.005) and Poiseuille (body force density 1e-6 on each
    component), 50x100 fluid rows, nu = 0.17, 10000 steps, FP64 and FP32.
    Reports the velocity-profile error against the analytic profiles
    (Couette: linear through the wall planes; Poiseuille: the parabola of
    the total force density and the mean total density) relative to the
    profile's peak, and the FP32 error against FP64."""
    steps = args.steps if args.steps_given else 10000
    rows = []
    for flow in ("couette", "poiseuille"):
        for G_ads in (-0.2, 0.0, 0.2):
            wl = W.cocurrent(flow, G_ads=G_ads)
            prof = {}
            for name, st in (("f64", lbm.F64), ("f32", lbm.F32)):
                g = lbm.lattice_from_workload(wl, st)
                g.step(steps)
                r1, r2, ux, _ = g.get_fields()
                prof[name] = (ux[1:-1].mean(axis=1), (r1 + r2)[1:-1].mean())
                g.close()
            y = np.arange(1, wl.ny - 1) - (wl.ny - 1) / 2.0
            half = (wl.ny - 2) / 2.0
            if flow == "couette":
                ua = wl.wall_velocity[2] * y / half
            else:
                nu = (wl.tau - 0.5) / 3.0
                ua = 2.0 * wl.accel[0] / (2.0 * nu * prof["f64"][1]) * (half ** 2 - y ** 2)
            peak = float(np.max(np.abs(ua)))
            rows.append({"flow": flow, "G_ads": G_ads,
                         "err_vs_analytic": round(float(np.max(np.abs(prof["f64"][0] - ua))) / peak, 5),
                         "f32_vs_f64": float(np.max(np.abs(prof["f32"][0] - prof["f64"][0]))) / peak})
            print(f"[cocurrent] {rows[-1]}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "co-current flow: max velocity-profile error / peak",
                      "workload": f"50x100 channel, two layers (a = 25), nu = 0.17, {steps} steps", "rows": rows}),
          flush=True)


def obstacle_flow(args):
    """A droplet carried by a Zou-He inlet past a square obstacle to an
    outflow (Sec. 3.3, 350x150, Re = 7.5), original against improved
    adhesion: where component 1 ends up.  The paper's Fig. 13 shows the
    original scheme leaving a layer and droplets of component 1 on the
    channel walls and around the obstacle; the improved scheme does not.
    Reported: the droplet's centroid, the mass of component 1 above its
    dissolved level in the wall bands (rows 1-3 and the top three fluid
    rows) and in a 3-node band around the obstacle, the largest rho_1 in
    the wall bands, and the throughput (tiny lattice: launch-bound)."""
    import torch
    steps = args.steps if args.steps_given else 10000
    storage = STORAGES[args.storage]
    rows = []
    for scheme, fl in (("original", lbm.SCHEME_ORIGINAL), ("improved", 0)):
        wl = W.obstacle_drop()
        wl.flags |= fl
        stream = torch.cuda.Stream()
        g = lbm.lattice_from_workload(wl, storage)
        g.set_stream(stream.cuda_stream)
        ms = _timed_steps(g, stream, steps, 0)
        r1, r2, ux, uy = g.get_fields()
        m = g.reduce()
        fluid = wl.solid == 0
        y, x = np.mgrid[0:wl.ny, 0:wl.nx]
        walls = fluid & ((y <= 3) | (y >= wl.ny - 4))
        sq = (np.abs(x - 122.0) < 12.5 + 3) & (np.abs(y - 75.0) < 12.5 + 3) & fluid
        excess = np.clip(r1 - W.RHO_MINOR, 0.0, None)
        drop = fluid & (r1 > r2)
        row = {"scheme": scheme, "t": steps,
               "drop_centroid_x": round(float((x * drop).sum() / max(drop.sum(), 1)), 2),
               "drop_nodes": int(drop.sum()),
               "wall_band_excess_rho1": round(float(excess[walls].sum()), 3),
               "wall_band_max_rho1": round(float(r1[walls].max()), 4),
               "obstacle_band_excess_rho1": round(float(excess[sq].sum()), 3),
               "max_u": float(m[4]), "nonfinite": int(m[7]),
               "MLUPS": round(g.fluid_nodes * steps / (ms * 1e-3) / 1e6, 1)}
        rows.append(row)
        g.close()
        print(f"[obstacle] {row}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "droplet past a square obstacle: component 1 on walls, original vs improved",
                      "workload": f"350x150 channel, square 25 at (122, 75), droplet r = 25 at (55, 75), Zou-He "
                                  f"Poiseuille inlet (Re = 7.5), outflow, G_ads = -0.2, {args.storage} storage, "
                                  f"{steps} steps", "rows": rows}), flush=True)


def sphere_drop(args):
    """The 3-D case of Sec. 3.5: a droplet (r = 45) on a sphere (R = 50) in
    a periodic 200 x 200 x 280 box, D3Q19 with the 92-position stencil.
    Times `--steps` steps (5 repeats, median) at lambda = 0.38 in the chosen
    storage and reports MLUPS and the HBM roofline fraction (algorithmic
    bytes 2 x 19 x (read + write) x element + 1 per fluid update); with
    --full, runs 20000 steps at each lambda of the paper (0.38, 1, 2.1) and
    reports the contact angles."""
    import torch
    storage = STORAGES[args.storage]
    steps = args.steps if args.steps_given else 500
    flags = lbm.ROUND_NEAREST if args.nearest else 0
    wl = W.sphere_drop(lam=0.38)
    stream = torch.cuda.Stream()
    g = lbm.lattice3d_from_workload(wl, storage, flags)
    g.set_stream(stream.cuda_stream)
    if args.tile not in ("default", "auto"):
        vals = [int(v) for v in args.tile.split(",")]
        g.set_tile(*vals)
    reps = 5
    chunk = [max(1, steps // reps)] * reps
    with torch.cuda.stream(stream):
        g.step(args.warmup)
        g.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        evs[0].record(stream)
        for r in range(reps):
            g.step(chunk[r])
            evs[r + 1].record(stream)
        evs[-1].synchronize()
    rep = [evs[r].elapsed_time(evs[r + 1]) / chunk[r] for r in range(reps)]
    ms_step = float(np.median(rep))
    n_fluid, bpu = g.fluid_nodes, g.bytes_per_update
    achieved = bpu * n_fluid / (ms_step * 1e-3) / 1e9
    m = g.reduce()
    out = {"metric": "3-D two-component D3Q19 MLUPS and contact angle on a sphere",
           "workload": f"sphere 200x200x280 (R = 50, droplet r = 45, overlap 15), lambda = 0.38, {args.storage} storage"
                       + rounding_label(args),
           "value": round(n_fluid / (ms_step * 1e-3) / 1e6, 1), "unit": "MLUPS", "fluid_nodes": n_fluid,
           "ms_per_step": round(ms_step, 5), "repeats_ms_per_step": [round(v, 5) for v in rep],
           "tile": list(g.get_tile()),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_update": bpu},
           "mass1": float(m[0]), "mass2": float(m[1]), "max_u": float(m[5]), "nonfinite": int(m[8])}
    g.close()
    if args.full:
        th = {}
        for lam in W.SPHERE_LAMBDAS:
            wl = W.sphere_drop(lam=lam)
            g = lbm.lattice3d_from_workload(wl, storage, flags)
            g.step(wl.steps)
            try:
                th[str(lam)] = round(g.contact_angle(wl.wall_kind, wl.wall), 3)
            except lbm.LbmError as e:
                th[str(lam)] = str(e)
            g.close()
            print(f"[sphere] lambda {lam}: theta {th[str(lam)]}", file=sys.stderr, flush=True)
        out["theta_deg"] = th
        out["steps_full"] = W.sphere_drop().steps
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=7000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--storage", default="f32", choices=sorted(STORAGES))
    ap.add_argument("--nearest", action="store_true",
                    help="f16/bf16: round-to-nearest-even stores instead of the default stochastic rounding")
    ap.add_argument("--diag-every", type=int, default=100)
    ap.add_argument("--tile", default="default",
                    help="default (the library's measured default for the storage), auto (autotune on the "
                         "workload) or BLOCK,ROWS[,SCHED]")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--workload", default="constrictions",
                    choices=["constrictions", "calibration", "porous", "cylinder", "schemes", "open",
                             "cocurrent", "obstacle", "sphere"],
                    help="constrictions: the 16384x2048 channel (default); calibration: the 512-run batch; "
                         "porous: the storage precision study; cylinder: the contact-angle sweep per storage; "
                         "schemes: original against improved adhesion; open: the channel with an inlet and "
                         "an outflow against the periodic one; cocurrent: Couette and Poiseuille layers; "
                         "obstacle: a droplet past a square, original against improved adhesion; sphere: the "
                         "3-D droplet on a sphere (200x200x280)")
    ap.add_argument("--record-every", type=int, default=1000, help="porous: recording interval")
    ap.add_argument("--full", action="store_true", help="calibration: run the configured 10000 steps and "
                    "report contact angles")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (read BYTES, write BYTES) five "
                         "times, to scale HBM byte counters against a known traffic")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 5}))
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU slab "
              "decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)

    args.steps_given = any(a.startswith("--steps") for a in sys.argv[1:])
    if args.workload == "calibration":
        calibration_batch(args)
        return
    if args.workload == "porous":
        porous_precision(args)
        return
    if args.workload == "cylinder":
        cylinder_sweep(args)
        return
    if args.workload == "schemes":
        scheme_comparison(args)
        return
    if args.workload == "open":
        open_channel(args)
        return
    if args.workload == "cocurrent":
        cocurrent_flow(args)
        return
    if args.workload == "obstacle":
        obstacle_flow(args)
        return
    if args.workload == "sphere":
        sphere_drop(args)
        return

    import torch  # device streams and events only

    wl = W.constrictions()
    storage = STORAGES[args.storage]
    flags = lbm.ROUND_NEAREST if args.nearest else 0
    stream = torch.cuda.Stream()
    lat = lbm.lattice_from_workload(wl, storage, flags)
    lat.set_stream(stream.cuda_stream)
    if args.tile == "default":
        block, rows, sched = lat.get_tile()
    elif args.tile == "auto":
        block, rows, sched = lat.autotune(8)
    else:
        vals = [int(v) for v in args.tile.split(",")]
        block, rows, sched = vals[0], vals[1], (vals[2] if len(vals) > 2 else 0)
        lat.set_tile(block, rows, sched)
    lat.set_diag_interval(args.diag_every)
    n_fluid = lat.fluid_nodes
    bpu = lat.bytes_per_update

    # the K timed steps run as 5 equal repeats (the last takes the
    # remainder), each bracketed by HIP events on the library's stream; the
    # step rate is the median repeat's
    reps = 5 if args.steps >= 10 else 1
    chunk = [args.steps // reps] * reps
    chunk[-1] += args.steps - sum(chunk)
    with torch.cuda.stream(stream):
        lat.step(args.warmup)
        lat.synchronize()
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        evs[0].record(stream)
        for r in range(reps):
            lat.step(chunk[r])
            evs[r + 1].record(stream)
        evs[-1].synchronize()
        torch.cuda.synchronize()
    ms = evs[0].elapsed_time(evs[-1])
    rep_ms_step = [evs[r].elapsed_time(evs[r + 1]) / chunk[r] for r in range(reps)]
    diag, t_diag = lat.get_diag() if args.diag_every > 0 else (None, None)
    ms_step = float(np.median(rep_ms_step))
    mlups = n_fluid / (ms_step * 1e-3) / 1e6
    achieved = bpu * n_fluid / (ms_step * 1e-3) / 1e9
    traffic = measured_traffic(args.storage + ("_rne" if args.nearest else ""), (block, rows, sched))
    steps_per_launch = 2 if (sched & lbm.SCHED_TWO_STEP) and storage != lbm.F64 else 1
    lat.close()
    copy_gbs = copy_bandwidth()
    # real HBM rate of the step kernel: counter bytes per launch over the
    # measured time per launch (only while the counters match the kernel)
    hbm_gbs = traffic / (steps_per_launch * ms_step * 1e-3) / 1e9 if traffic else None

    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if storage == lbm.F64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"constrictions {wl.nx}x{wl.ny} (64 squares of side 128, seed 355), "
                               f"G_c=0.9 G_ads=0.15 tau=1 g=2e-6, {args.storage} storage"
                               + rounding_label(args),
                   "nx": wl.nx, "ny": wl.ny, "fluid_nodes": n_fluid, "storage": args.storage,
                   "tile": {"block": block, "seg_rows": rows, "sched": sched},
                   "diag_every": args.diag_every},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_update": bpu, "steps_per_launch": steps_per_launch,
                     "hbm_bytes_per_update": (round(traffic / (steps_per_launch * n_fluid), 1)
                                              if traffic else None),
                     "hbm_measured_gbs": round(hbm_gbs, 1) if hbm_gbs else None,
                     "hbm_measured_frac": round(hbm_gbs / HBM_PEAK_GBS, 4) if hbm_gbs else None,
                     "copy_gbs": copy_gbs, "frac_of_copy": round(achieved / copy_gbs, 4)},
        "repeats_ms_per_step": [round(v, 5) for v in rep_ms_step],
        "timed_ms_total": round(ms, 2),
    }
    if diag is not None:
        out["diagnostics"] = {"t": t_diag, "mass1": diag[0], "mass2": diag[1], "max_u": diag[4],
                              "nonfinite_nodes": int(diag[7])}
    if not args.no_accuracy:
        out["accuracy"] = precision_check()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
