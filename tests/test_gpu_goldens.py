"""Long runs against stored FP64 oracle values (tests/golden/, written by
make_oracle_goldens.py from the oracle alone).

Cylinder sweep (400 x 400, seven adhesion values, 20000 steps): the FP64
device path reproduces the oracle's angle to 1e-6 degrees; FP32 storage
within 0.5 degrees, FP16 and BF16 storage in their default (stochastic)
rounding within 1 degree (the stated tolerances).  Calibration batch: the first 16 runs of the
seeded 512-run batch, advanced together in one FP32 batch with an
autotuned tile and graph replays, within 0.5 degrees of the oracle.
"""
import json
import os

import numpy as np
import pytest

from paper_2505_22256_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("storage,flags,tol", [(0, 0, 1e-6), (1, 0, 0.5), (2, 0, 1.0), (3, 0, 1.0)])
def test_cylinder_sweep_against_oracle(lbm_mod, storage, flags, tol):
    ref = _load("cylinder_theta.json")
    worst = 0.0
    for case in ref["cases"]:
        wl = W.cylinder_drop(G_ads=case["G_ads"])
        g = lbm_mod.lattice_from_workload(wl, storage, flags)
        g.step(ref["steps"])
        th = g.contact_angle(wl.wall_kind, wl.wall)
        g.close()
        err = abs(th - case["theta_deg"])
        worst = max(worst, err)
        assert err < tol, (case["G_ads"], th, case["theta_deg"])
    print(f"storage {storage} flags {flags}: worst angle error {worst:.3g} deg")


def test_calibration_batch_against_oracle(lbm_mod):
    ref = _load("calibration_theta.json")
    n = len(ref["runs"])
    runs = W.calibration_runs(steps=ref["steps"])[:n]
    b = lbm_mod.Batch(runs, lbm_mod.F32)
    b.autotune(2)
    b.use_graph(True, 50)
    b.step(ref["steps"])
    th = b.contact_angles()
    for r in ref["runs"]:
        if r["theta_deg"] is None:
            continue
        assert abs(th[r["index"]] - r["theta_deg"]) < 0.5, (r, th[r["index"]])


def test_batch_autotune_restores_state(lbm_mod):
    runs = W.calibration_runs(nruns=6, steps=100)
    a = lbm_mod.Batch(runs, lbm_mod.F32)
    a.step(7)
    a.set_tile(128, 16)
    a.autotune(1)
    a.step(13)
    c = lbm_mod.Batch(runs, lbm_mod.F32)
    c.step(20)
    for r in range(len(runs)):
        for x, y in zip(a.get_fields(r), c.get_fields(r)):
            assert np.array_equal(x, y), r
