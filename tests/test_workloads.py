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


def test_poiseuille_inlet_profile():
    """The inlet parabola goes through the halfway wall planes: zero on the
    solid rows, peak u_max midway, symmetric, no transverse part."""
    u = W.poiseuille_profile(102, 0.02)
    assert u.shape == (2, 102)
    assert u[0, 0] == 0.0 and u[0, -1] == 0.0 and np.all(u[1] == 0.0)
    assert np.allclose(u[0, 1:-1], u[0, 1:-1][::-1], rtol=0, atol=1e-17)
    eta = (np.arange(102) - 0.5) / 100
    assert np.allclose(u[0, 1:-1], 0.08 * eta[1:-1] * (1 - eta[1:-1]), rtol=1e-15)
    assert abs(u[0].max() - 0.02 * (1 - (0.5 / 50) ** 2)) < 1e-15


def test_cocurrent_recipes():
    c = W.cocurrent("couette")
    p = W.cocurrent("poiseuille")
    for wl in (c, p):
        assert (wl.nx, wl.ny) == (50, 102)
        assert wl.solid[0].all() and wl.solid[-1].all() and not wl.solid[1:-1].any()
        assert abs(wl.tau - (3 * 0.17 + 0.5)) < 1e-12
        y = np.arange(102)
        core = np.abs(y - 50.5) <= 25
        assert np.all(wl.rho1[1:-1][core[1:-1]] == 1.02) and np.all(wl.rho1[1:-1][~core[1:-1]] == 0.05)
    assert c.wall_velocity == (-0.005, 0.0, 0.005, 0.0) and c.flags == W.PERIODIC_X
    assert p.accel == (1e-6, 0.0, 1e-6, 0.0) and p.flags & W.FORCE_DENSITY
    with pytest.raises(ValueError):
        W.cocurrent("stokes")


def test_obstacle_drop_recipe():
    wl = W.obstacle_drop()
    assert (wl.nx, wl.ny) == (350, 150) and wl.flags == W.INLET | W.OUTFLOW
    inner = wl.solid[1:-1]
    assert inner.sum() == 25 * 25  # the square, |x - 122|, |y - 75| < 12.5
    ys, xs = np.nonzero(inner)
    assert (xs.min(), xs.max(), ys.min() + 1, ys.max() + 1) == (110, 134, 63, 87)
    drop = (wl.rho1 > wl.rho2) & (wl.solid == 0)
    assert abs(drop.sum() - math.pi * 25 ** 2) < 2 * math.pi * 25
    nu = (wl.tau - 0.5) / 3
    assert abs(wl.inlet_u[0].max() - 7.5 * nu / 50 * (1 - (0.5 / 74) ** 2)) < 1e-12


def test_open_constriction_channel_recipe():
    a, b = W.constrictions(nx=512, ny=64, n_squares=2, side=8), W.constrictions(nx=512, ny=64, n_squares=2, side=8,
                                                                               open_ends=True)
    assert np.array_equal(a.solid, b.solid) and np.array_equal(a.rho1, b.rho1)
    assert a.flags == W.PERIODIC_X and b.flags == W.INLET | W.OUTFLOW
    assert b.inlet_u.shape == (2, 64) and b.inlet_u[0].max() <= 0.01
