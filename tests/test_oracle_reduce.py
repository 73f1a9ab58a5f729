"""Pins of the oracle's whole-lattice diagnostics, of the literal-velocity
reading and of its thread-count independence.

The diagnostics (M_1, M_2, P_x, P_y, max |u|, min and max rho_1, the count
of non-finite nodes) are checked against states whose values are known in
closed form: a uniform mixture moving at a fixed velocity (Eq. 6 makes it a
fixed point of the collision), a field with two prescribed densities, and a
single node moving in a fluid at rest.  The velocity readings are checked
against the one-step momentum balance of Guo's forcing scheme (Eq. 1-2, 5,
7): after one step of a uniform fluid under a body force F = rho g the
momentum is rho g (Guo's half-force shift) or (1 - 1/(2 tau)) rho g
(the literal u = j / rho of Eq. 4-5).
"""
import numpy as np

from paper_2505_22256_amd import workloads as W

EPS = np.finfo(float).eps


def _d2q9_feq(rho, ux, uy):
    """Second-order equilibrium of Eq. 6, written out independently of the
    oracle (D2Q9 weights 4/9, 1/9, 1/36; c_s^2 = 1/3)."""
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    eu = ex * ux + ey * uy
    return w * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy))


def _uniform_flow(oracle_mod, r1, r2, U, nx=11, ny=9, G_c=0.9):
    o = oracle_mod.Oracle(nx, ny, oracle_mod.PERIODIC_X | oracle_mod.PERIODIC_Y)
    o.set_geometry(np.zeros((ny, nx), np.uint8))
    o.set_params(G_c, 0.1, 0.8)
    f = np.empty((2, 9, ny, nx))
    for k, r in enumerate((r1, r2)):
        f[k] = _d2q9_feq(r, *U)[:, None, None]
    o.set_populations(f)
    return o


def test_reduce_uniform_flow_closed_form(oracle_mod):
    """A uniform two-component mixture at equilibrium with velocity U has
    no force (every stencil difference vanishes) and is a fixed point of
    the collision and of periodic streaming.  So at any time
    M_k = N rho_k, P = N (rho_1 + rho_2) U, max |u| = |U|,
    min rho_1 = max rho_1 = rho_1.  U_x != U_y and rho_2 != 0 make a
    swapped momentum component or a momentum weighted by one component
    fail."""
    r1, r2, U = 0.83, 0.21, (0.031, -0.017)
    nx, ny = 11, 9
    N = nx * ny
    o = _uniform_flow(oracle_mod, r1, r2, U, nx, ny)
    for steps in (0, 7):
        o.step(steps)
        out = o.reduce()
        rt = r1 + r2
        assert abs(out[0] - N * r1) < 64 * EPS * N * r1
        assert abs(out[1] - N * r2) < 64 * EPS * N * r2
        assert abs(out[2] - N * rt * U[0]) < 1e-13 * N * rt
        assert abs(out[3] - N * rt * U[1]) < 1e-13 * N * rt
        assert abs(out[4] - np.hypot(*U)) < 1e-14
        assert abs(out[5] - r1) < 16 * EPS and abs(out[6] - r1) < 16 * EPS
        assert out[7] == 0


def test_reduce_min_max_of_prescribed_densities(oracle_mod):
    """At t = 0 (f = w rho, u = 0 up to the half-force shift) the density
    extremes are the prescribed values over fluid nodes only: a solid node
    (which outputs 0) must not become the minimum, and a solid node's
    prescribed density must not become the maximum."""
    nx, ny = 12, 10
    solid = np.zeros((ny, nx), np.uint8)
    solid[4:6, 3:5] = 1
    rho1 = np.full((ny, nx), 0.5)
    rho1[1, 1] = 0.125
    rho1[8, 10] = 0.875
    rho1[4, 3] = 5.0  # solid: ignored
    rho2 = np.full((ny, nx), 0.25)
    o = oracle_mod.Oracle(nx, ny, 3 | oracle_mod.SCHEME_ORIGINAL)
    o.set_geometry(solid)
    o.set_params(0.0, 0.0, 1.0)
    o.init_fields(rho1, rho2)
    out = o.reduce()
    fluid = solid == 0
    assert out[5] == 0.125 or abs(out[5] - 0.125) < 8 * EPS
    assert abs(out[6] - 0.875) < 8 * EPS
    assert abs(out[0] - rho1[fluid].sum()) < 1e-13 * rho1[fluid].sum()
    assert abs(out[1] - 0.25 * fluid.sum()) < 1e-13 * 0.25 * fluid.sum()
    # G_c = 0 and no body force: nothing moves at t = 0
    assert out[2] == 0 and out[3] == 0 and out[4] == 0


def test_reduce_max_speed_of_one_moving_node(oracle_mod):
    """One node at equilibrium with velocity (0.03, -0.04) in a mixture at
    rest of the same densities: the densities are uniform (the
    equilibrium's zeroth moment is rho to rounding), so forces vanish to
    rounding and max |u| = 0.05 while P = (rho_1 + rho_2) (0.03, -0.04)."""
    nx, ny = 10, 8
    r1, r2 = 0.7, 0.3
    o = oracle_mod.Oracle(nx, ny, 3)
    o.set_geometry(np.zeros((ny, nx), np.uint8))
    o.set_params(0.9, 0.0, 1.0)
    f = np.empty((2, 9, ny, nx))
    for k, r in enumerate((r1, r2)):
        f[k] = _d2q9_feq(r, 0.0, 0.0)[:, None, None]
        f[k, :, 5, 6] = _d2q9_feq(r, 0.03, -0.04)
    o.set_populations(f)
    out = o.reduce()
    assert abs(out[4] - 0.05) < 1e-14
    assert abs(out[2] - (r1 + r2) * 0.03) < 1e-14
    assert abs(out[3] + (r1 + r2) * 0.04) < 1e-14
    assert out[5] == out[6] or abs(out[6] - out[5]) < 8 * EPS


def test_reduce_counts_non_finite_nodes(oracle_mod):
    """The last diagnostic counts fluid nodes whose density or velocity is
    not finite; they are left out of every other entry.  An infinite
    rho_1 at one node makes that node's rho_1 and u non-finite, and the
    velocity of each of its 24 E8 neighbours too (their cohesion force
    takes -G_c psi Sum W psi e with an infinite psi: 0 * inf is NaN even at
    G_c = 0): 25 nodes."""
    nx, ny = 12, 12
    o = oracle_mod.Oracle(nx, ny, 3 | oracle_mod.SCHEME_ORIGINAL)
    o.set_geometry(np.zeros((ny, nx), np.uint8))
    o.set_params(0.0, 0.0, 1.0)
    o.init_fields(np.full((ny, nx), 0.6), np.full((ny, nx), 0.4))
    f = o.get_populations()
    f[0, 1, 6, 5] = 1e308
    f[0, 3, 6, 5] = 1e308  # rho_1 overflows to inf at (5, 6)
    o.set_populations(f)
    out = o.reduce()
    assert out[7] == 25
    assert abs(out[0] - 0.6 * (nx * ny - 25)) < 1e-12
    assert abs(out[1] - 0.4 * (nx * ny - 25)) < 1e-12
    assert out[6] < 0.6 + 1e-15


def test_velocity_readings_after_one_forced_step(oracle_mod):
    """R7 -- a uniform periodic mixture at rest under a body acceleration g
    (force F_k = rho_k g, no stencil force).  Guo's scheme: collision
    momentum j* = j + (1 - 1/(2 tau)) F + (rho u - j)/tau.
      default u = (j + F/2)/rho: u(0) = g/2, j(1) = F, u(1) = 3g/2;
      VEL_LITERAL u = j/rho:     u(0) = 0,  j(1) = (1 - 1/(2 tau)) F,
                                 u(1) = (1 - 1/(2 tau)) g."""
    nx, ny, tau = 7, 6, 0.8
    g = (2e-5, -3e-5)
    for flags, u0, u1 in ((0, 0.5, 1.5), (oracle_mod.VEL_LITERAL, 0.0, 1 - 1 / (2 * tau))):
        o = oracle_mod.Oracle(nx, ny, 3 | flags)
        o.set_geometry(np.zeros((ny, nx), np.uint8))
        o.set_params(0.9, 0.0, tau)
        o.set_body_accel(g[0], g[1], g[0], g[1])
        o.init_fields(np.full((ny, nx), 0.9), np.full((ny, nx), 0.1))
        _, _, ux, uy = o.get_fields()
        assert np.max(np.abs(ux - u0 * g[0])) < 1e-18 and np.max(np.abs(uy - u0 * g[1])) < 1e-18
        o.step(1)
        _, _, ux, uy = o.get_fields()
        assert np.max(np.abs(ux - u1 * g[0])) < 1e-15, (flags, ux[0, 0], u1 * g[0])
        assert np.max(np.abs(uy - u1 * g[1])) < 1e-15, (flags, uy[0, 0], u1 * g[1])


def test_results_do_not_depend_on_thread_count(oracle_mod):
    """The oracle's row loops are split over OpenMP threads, and no sum
    crosses a thread: populations, diagnostics and the contact angle are
    bitwise the same on one thread and on several."""
    wl = W.flat_drop(nx=60, ny=30, radius=12)
    prev = oracle_mod.set_threads(1)
    try:
        res = {}
        for nt in (1, 4):
            oracle_mod.set_threads(nt)
            o = oracle_mod.Oracle(wl.nx, wl.ny, wl.flags)
            o.set_geometry(wl.solid)
            o.set_params(wl.G_c, wl.G_ads, wl.tau)
            o.init_fields(wl.rho1, wl.rho2)
            o.step(300)
            res[nt] = (o.get_populations(), o.reduce(), o.contact_angle(0, (0.5, 0, 0)))
        assert np.array_equal(res[1][0], res[4][0])
        assert np.array_equal(res[1][1], res[4][1])
        assert res[1][2] == res[4][2]
    finally:
        oracle_mod.set_threads(prev)
