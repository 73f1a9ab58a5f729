"""Host logic: the seeded synthetic workloads and the analysis helpers of
the benchmark.  These hold no LBM arithmetic; the checks pin the recipes
they are documented with (sizes, geometry rules, value ranges, seeds)."""
import math

import numpy as np
import pytest

from paper_2505_22256_amd import workloads as W


def test_coexistence_pair_solves_its_equation():
    """The droplet start densities of the cylinder and calibration runs are
    the bulk coexistence pair of G_c = 0.9 at total density 1.03:
    c_s^2 ln(rho_m / rho_d) = G_c (rho_m - rho_d)."""
    m, d = W.RHO_MAJOR_EQ, W.RHO_MINOR_EQ
    assert abs(m + d - 1.03) < 1e-14
    assert abs(math.log(m / d) / 3.0 - 0.9 * (m - d)) < 1e-12
    assert m > d > 0


def test_flat_drop_recipe():
    wl = W.flat_drop()
    assert (wl.nx, wl.ny) == (100, 50)
    assert wl.solid[0].all() and wl.solid[-1].all() and not wl.solid[1:-1].any()
    y, x = np.mgrid[0:50, 0:100]
    inside = ((x - 50.0) ** 2 + (y - 0.5) ** 2 < 400.0) & (wl.solid == 0)
    assert np.all(wl.rho1[inside] == W.RHO_MAJOR) and np.all(wl.rho2[inside] == W.RHO_MINOR)
    outside = ~inside & (wl.solid == 0)
    assert np.all(wl.rho1[outside] == W.RHO_MINOR) and np.all(wl.rho2[outside] == W.RHO_MAJOR)
    assert np.all(wl.rho1[wl.solid == 1] == 0)
    assert wl.flags == W.PERIODIC_X and wl.wall == (0.5, 0.0, 0.0)


def test_cylinder_mask_has_no_single_voxel_features():
    """Strict voxelisation: every solid row and column of the cylinder is
    at least 3 voxels wide (the pole rows of a <= R^2 mask are one voxel)."""
    wl = W.cylinder_drop()
    rows = wl.solid.sum(axis=1)
    cols = wl.solid.sum(axis=0)
    assert rows[rows > 0].min() >= 3 and cols[cols > 0].min() >= 3
    assert wl.solid[210, 200] == 0 and wl.solid[209, 200] == 1
    assert wl.wall == (200.0, 150.0, 60.5)
    drop = wl.rho1 > 0.5
    assert abs(wl.rho1[drop].max() - W.RHO_MAJOR_EQ) < 1e-15


def test_porous_recipe():
    wl = W.porous()
    assert (wl.nx, wl.ny) == (2048, 1024)
    assert abs((1 - wl.solid[:, 96:].mean()) - 0.70) < 0.01
    d = np.array(wl.disks)
    assert np.all((d[:, 2] >= 8) & (d[:, 2] < 24))
    # every pair of disks keeps a gap of at least 2 lattice units
    for i in range(len(d)):
        gap = np.hypot(d[i + 1:, 0] - d[i, 0], d[i + 1:, 1] - d[i, 1]) - d[i + 1:, 2] - d[i, 2]
        assert np.all(gap >= 2.0)
    assert wl.solid[:, :96][1:-1].sum() == 0
    assert np.all(wl.rho1[1:-1, :64] == W.RHO_MAJOR)
    assert wl.accel == (1e-6, 0.0, 0.0, 0.0)


def test_constrictions_recipe():
    wl = W.constrictions()
    assert (wl.nx, wl.ny) == (16384, 2048)
    body = wl.solid[1:-1].copy()
    # 64 squares of side 128, each attached to the bottom or the top wall
    cols = np.nonzero(body.any(axis=0))[0]
    runs = np.split(cols, np.nonzero(np.diff(cols) > 1)[0] + 1)
    assert len(runs) == 64 and all(len(r) == 128 for r in runs)
    for r in runs:
        c = body[:, r[0]]
        ys = np.nonzero(c)[0] + 1
        assert len(ys) == 128 and (ys[0] == 1 or ys[-1] == 2046)
    assert wl.n_fluid == 32473088
    assert wl.accel == (2e-6, 0.0, 2e-6, 0.0) and wl.G_ads == 0.15


def test_calibration_runs_are_seeded_and_in_range():
    a = W.calibration_runs(nruns=40)
    b = W.calibration_runs(nruns=40)
    for x, y in zip(a, b):
        assert (x.nx, x.wall_kind, x.G_ads, x.tau) == (y.nx, y.wall_kind, y.G_ads, y.tau)
        assert np.array_equal(x.solid, y.solid)
    assert all(w.nx == w.ny and w.nx in (128, 192, 256, 384, 512) for w in a)
    assert all(-0.35 <= w.G_ads <= 0.35 and 0.7 <= w.tau <= 1.2 for w in a)
    assert {w.wall_kind for w in a} == {W.WALL_FLAT, W.WALL_CYLINDER}


def test_saturation_and_front_helper():
    import bench
    wl = W.flat_drop(nx=40, ny=20)
    r1 = np.zeros((20, 40))
    r2 = np.ones((20, 40))
    r1[:, :10] = 1.0
    r2[:, :10] = 0.0
    r1[:, 39] = 1.0  # leaked backwards across the periodic seam: not the front
    r2[:, 39] = 0.0
    s1, front = bench.saturation_and_front(wl, r1, r2)
    assert front == 9
    assert abs(s1 - 11 * 18 / (40 * 18)) < 1e-15
