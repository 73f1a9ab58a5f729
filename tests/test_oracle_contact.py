"""P14 -- the contact-angle measurement of the oracle.

The paper does not state how it reads the contact angle (Sec. 3.2).  The
method used here: interface points where the effective density (Eq. 10)
changes sign along lattice links, placed by linear interpolation, kept only
on links between the largest region of each sign (the droplet and the fluid
around it), points closer than 3 lattice units to the wall dropped, an
algebraic circle fit refined by Gauss-Newton, and the angle between the
fitted circle and the wall.  These tests pin that chain on fields whose contact angle is known by
construction: exact circles, and smooth tanh-profile caps cut by a flat wall
or a cylinder at a prescribed angle.
"""
import math

import numpy as np
import pytest

RHO_M, RHO_D, WIDTH = 0.95, 0.09, 2.0


def test_circle_fit_exact_points(oracle_mod):
    rng = np.random.default_rng(7)
    for _ in range(10):
        a, b, r = rng.uniform(-50, 50), rng.uniform(-50, 50), rng.uniform(5, 80)
        t = rng.uniform(0.2, 2.5) + np.sort(rng.uniform(0, rng.uniform(0.5, 6.0), 40))
        abr = oracle_mod.circle_fit(a + r * np.cos(t), b + r * np.sin(t))
        assert np.allclose(abr, [a, b, r], rtol=0, atol=1e-9 * (1 + r))


def test_circle_fit_noisy_points_are_least_squares(oracle_mod):
    """Gauss-Newton refinement reaches a stationary point of the geometric
    error: perturbing the fitted (a, b, r) never lowers sum (d_i - r)^2."""
    rng = np.random.default_rng(8)
    t = rng.uniform(0.3, 2.8, 60)
    px = 10 + 30 * np.cos(t) + rng.normal(0, 0.3, 60)
    py = -5 + 30 * np.sin(t) + rng.normal(0, 0.3, 60)
    a, b, r = oracle_mod.circle_fit(px, py)
    cost = lambda a_, b_, r_: np.sum((np.hypot(px - a_, py - b_) - r_) ** 2)
    c0 = cost(a, b, r)
    for d in np.eye(3) * 1e-4:
        assert cost(a + d[0], b + d[1], r + d[2]) >= c0 - 1e-12
        assert cost(a - d[0], b - d[1], r - d[2]) >= c0 - 1e-12


def _cap_fields(nx, ny, centre, r):
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    s = np.tanh((r - np.hypot(x - centre[0], y - centre[1])) / WIDTH)
    rho1 = 0.5 * (RHO_M + RHO_D) + 0.5 * (RHO_M - RHO_D) * s
    rho2 = 0.5 * (RHO_M + RHO_D) - 0.5 * (RHO_M - RHO_D) * s
    return rho1, rho2


@pytest.mark.parametrize("theta", [20, 40, 60, 90, 120, 140, 160])
def test_flat_wall_angle_of_synthetic_cap(oracle_mod, theta):
    th = math.radians(theta)
    r = max(30.0, 15.0 / (1 - math.cos(th)))
    yw = 0.5
    yc = yw - r * math.cos(th)
    half = r * math.sin(th) if theta <= 90 else r
    nx = int(2 * half + 40)
    ny = int(yc + r + 12)
    solid = np.zeros((ny, nx), np.uint8)
    solid[0] = 1
    solid[-1] = 1
    r1, r2 = _cap_fields(nx, ny, (nx / 2, yc), r)
    o = oracle_mod.Oracle(nx, ny, oracle_mod.PERIODIC_X)
    o.set_geometry(solid)
    o.set_params(0.9, 0.0, 1.0)
    o.init_fields(np.where(solid, 0, r1), np.where(solid, 0, r2))
    got = o.contact_angle(0, (yw, 0.0, 0.0))
    assert abs(got - theta) < 0.3, (theta, got)


@pytest.mark.parametrize("theta", [20, 45, 90, 135, 160])
def test_cylinder_angle_of_synthetic_cap(oracle_mod, theta):
    th = math.radians(theta)
    R, r = 30.0, 25.0
    Rs = R + 0.5
    d = math.sqrt(Rs * Rs + r * r - 2 * Rs * r * math.cos(th))
    n = 160
    C = (80.0, 60.0)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    solid = (((x - C[0]) ** 2 + (y - C[1]) ** 2) <= R * R).astype(np.uint8)
    r1, r2 = _cap_fields(n, n, (C[0], C[1] + d), r)
    o = oracle_mod.Oracle(n, n, oracle_mod.PERIODIC_X | oracle_mod.PERIODIC_Y)
    o.set_geometry(solid)
    o.set_params(0.9, 0.0, 1.0)
    o.init_fields(np.where(solid, 0, r1), np.where(solid, 0, r2))
    got = o.contact_angle(1, (C[0], C[1], Rs))
    assert abs(got - theta) < 0.3, (theta, got)


def test_interface_points_respect_wall_exclusion(oracle_mod):
    nx, ny = 120, 60
    solid = np.zeros((ny, nx), np.uint8)
    solid[0] = 1
    solid[-1] = 1
    r1, r2 = _cap_fields(nx, ny, (60.0, 0.5), 30.0)
    o = oracle_mod.Oracle(nx, ny, oracle_mod.PERIODIC_X)
    o.set_geometry(solid)
    o.set_params(0.9, 0.0, 1.0)
    o.init_fields(np.where(solid, 0, r1), np.where(solid, 0, r2))
    px, py = o.interface_points(0, (0.5, 0, 0))
    assert len(px) > 50
    assert np.all(py - 0.5 >= 3.0)
    # every point lies on the prescribed circle to within the interpolation error
    assert np.max(np.abs(np.hypot(px - 60.0, py - 0.5) - 30.0)) < 0.05


def _blob(r1, r2, centre, r, inside_positive):
    """Overwrite a small tanh blob of the given sign into the fields."""
    ny, nx = r1.shape
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    s = np.tanh((r - np.hypot(x - centre[0], y - centre[1])) / WIDTH)
    m = s > -0.999
    sign = 1.0 if inside_positive else -1.0
    r1 = np.where(m, 0.5 * (RHO_M + RHO_D) + sign * 0.5 * (RHO_M - RHO_D) * s, r1)
    r2 = np.where(m, 0.5 * (RHO_M + RHO_D) - sign * 0.5 * (RHO_M - RHO_D) * s, r2)
    return r1, r2


def _cyl_oracle(oracle_mod, solid, r1, r2, n):
    o = oracle_mod.Oracle(n, n, oracle_mod.PERIODIC_X | oracle_mod.PERIODIC_Y)
    o.set_geometry(solid)
    o.set_params(0.9, 0.0, 1.0)
    o.init_fields(np.where(solid, 0, r1), np.where(solid, 0, r2))
    return o


@pytest.mark.parametrize("theta", [60, 110])
def test_pocket_and_satellite_do_not_enter_the_fit(oracle_mod, theta):
    """A component-2 pocket trapped inside the droplet next to the wall and
    a separate satellite droplet change nothing: the points come only from
    the interface between the largest region of each sign, so the angle and
    the point set equal those of the bare cap."""
    th = math.radians(theta)
    R, r = 30.0, 25.0
    Rs = R + 0.5
    d = math.sqrt(Rs * Rs + r * r - 2 * Rs * r * math.cos(th))
    n = 160
    C = (80.0, 60.0)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    solid = (((x - C[0]) ** 2 + (y - C[1]) ** 2) < R * R).astype(np.uint8)
    r1, r2 = _cap_fields(n, n, (C[0], C[1] + d), r)
    bare = _cyl_oracle(oracle_mod, solid, r1, r2, n)
    th_bare = bare.contact_angle(1, (C[0], C[1], Rs))
    px0, py0 = bare.interface_points(1, (C[0], C[1], Rs))
    # pocket: negative blob of radius 5 centred 9 above the cylinder top,
    # inside the droplet; satellite: positive blob of radius 6 far away
    r1b, r2b = _blob(r1, r2, (C[0], C[1] + R + 9.0), 5.0, inside_positive=False)
    r1b, r2b = _blob(r1b, r2b, (20.0, 150.0), 6.0, inside_positive=True)
    dirty = _cyl_oracle(oracle_mod, solid, r1b, r2b, n)
    px1, py1 = dirty.interface_points(1, (C[0], C[1], Rs))
    assert len(px1) == len(px0)
    assert np.allclose(np.sort(px1), np.sort(px0), atol=1e-9)
    assert abs(dirty.contact_angle(1, (C[0], C[1], Rs)) - th_bare) < 1e-9
    assert abs(th_bare - theta) < 0.3


def test_largest_region_picks_the_bigger_droplet(oracle_mod):
    """Two droplets on a flat wall: the points are those of the larger one."""
    nx, ny = 200, 60
    solid = np.zeros((ny, nx), np.uint8)
    solid[0] = 1
    solid[-1] = 1
    r1, r2 = _cap_fields(nx, ny, (60.0, 0.5), 25.0)
    r1, r2 = _blob(r1, r2, (150.0, 0.5), 12.0, inside_positive=True)
    o = oracle_mod.Oracle(nx, ny, oracle_mod.PERIODIC_X)
    o.set_geometry(solid)
    o.set_params(0.9, 0.0, 1.0)
    o.init_fields(np.where(solid, 0, r1), np.where(solid, 0, r2))
    px, py = o.interface_points(0, (0.5, 0, 0))
    assert np.all(px < 100)
    assert abs(o.contact_angle(0, (0.5, 0, 0)) - 90.0) < 0.3
