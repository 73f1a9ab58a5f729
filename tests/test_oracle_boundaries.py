"""Pins of the oracle's open and moving boundaries: sliding walls (the
Couette set-up of Sec. 3.1), the Zou-He velocity inlet and the outflow of
Sec. 3.3, and the E8 stencil next to an open edge (Sec. 2.4, Table 1).

Each pin is fixed by something other than the oracle's own formulas: the
exact linear Couette profile, the moments that define a velocity
boundary, the equilibrium fixed point of uniform flow, the equality of the
two populations the zero-gradient outflow makes equal, and symmetry.
"""
import numpy as np
import pytest

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WQ = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _feq(rho, ux, uy):
    """Second-order D2Q9 equilibrium, c_s^2 = 1/3 (textbook form)."""
    eu = EX[:, None, None] * ux + EY[:, None, None] * uy
    return WQ[:, None, None] * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (ux ** 2 + uy ** 2))


def _channel(ny, nx):
    s = np.zeros((ny, nx), np.uint8)
    s[0] = 1
    s[-1] = 1
    return s


@pytest.mark.parametrize("tau,ub,ut", [(1.0, 0.01, -0.02), (0.7, 0.005, -0.005), (1.6, 0.0, 0.03)])
def test_couette_profile_is_exactly_linear(oracle_mod, tau, ub, ut):
    """Plane Couette flow between walls sliding at ub (bottom) and ut (top):
    the steady state of BGK with halfway bounce-back and Ladd's moving-wall
    term is the linear profile through the wall planes y = 1/2 and
    y = ny - 3/2, for any tau, to rounding; mass is conserved."""
    nx, ny = 5, 12
    o = oracle_mod.Oracle(nx, ny, oracle_mod.PERIODIC_X | oracle_mod.SCHEME_ORIGINAL)
    o.set_geometry(_channel(ny, nx))
    o.set_params(0.0, 0.0, tau)  # no cohesion, no adhesion: one effective fluid
    o.set_wall_velocity(ub, 0.0, ut, 0.0)
    o.init_fields(np.ones((ny, nx)), np.zeros((ny, nx)))
    m0 = o.reduce()[0]
    o.step(6000)
    rho1, _, ux, uy = o.get_fields()
    y = np.arange(1, ny - 1)
    ua = ub + (ut - ub) * (y - 0.5) / (ny - 2)
    assert np.max(np.abs(ux[1:-1] - ua[:, None])) < 1e-13
    assert np.max(np.abs(uy)) < 1e-13
    assert abs(o.reduce()[0] - m0) < 1e-12 * m0


def test_moving_wall_momentum_input(oracle_mod):
    """One step from rest next to a wall sliding at U: a fluid node on the
    wall receives, for each diagonal link from the wall, the reflected
    population plus 6 w_i rho (e_i . U) (Ladd), so its x momentum after the
    step is 2 * 6 * (1/36) * rho * U = rho U / 3 from the bottom wall."""
    nx, ny = 6, 9
    U, rho = 0.02, 1.3
    o = oracle_mod.Oracle(nx, ny, oracle_mod.PERIODIC_X | oracle_mod.SCHEME_ORIGINAL)
    o.set_geometry(_channel(ny, nx))
    o.set_params(0.0, 0.0, 1.0)
    o.set_wall_velocity(U, 0.0, 0.0, 0.0)
    o.init_fields(np.full((ny, nx), rho), np.zeros((ny, nx)))
    o.step(1)
    f = o.get_populations().reshape(2, 9, ny, nx)
    jx = (f[0] * EX[:, None, None]).sum(0)
    assert np.allclose(jx[1], rho * U / 3, rtol=1e-14, atol=0)
    assert np.max(np.abs(jx[2:-1])) == 0.0


def test_zou_he_inlet_imposes_the_row_velocity(oracle_mod):
    """At every inlet node the populations after streaming have the
    prescribed velocity: sum_i f_i e_i / sum_i f_i = (U, V) of the row, per
    component, whatever the known populations are (random state, walls,
    forces on)."""
    nx, ny = 12, 9
    o = oracle_mod.Oracle(nx, ny, oracle_mod.INLET | oracle_mod.OUTFLOW)
    o.set_geometry(_channel(ny, nx))
    o.set_params(0.9, 0.1, 1.0)
    rng = np.random.default_rng(1)
    U = rng.uniform(0.0, 0.05, ny)
    V = rng.uniform(-0.02, 0.02, ny)
    o.set_inlet_velocity(U, V)
    o.init_fields(1 + 0.1 * rng.random((ny, nx)), 0.1 + 0.1 * rng.random((ny, nx)))
    o.step(3)
    f = o.get_populations().reshape(2, 9, ny, nx)[:, :, 1:-1, 0]
    for k in range(2):
        rho = f[k].sum(0)
        assert np.max(np.abs((f[k] * EX[:, None]).sum(0) / rho - U[1:-1])) < 1e-15
        assert np.max(np.abs((f[k] * EY[:, None]).sum(0) / rho - V[1:-1])) < 1e-15


def test_uniform_flow_is_a_fixed_point(oracle_mod):
    """Uniform flow at the inlet velocity, in equilibrium, through an open
    channel (periodic in y): the collision leaves equilibrium unchanged,
    interior streaming keeps it uniform, Zou-He rebuilds exactly the
    equilibrium's unknowns and the outflow copies uniform values, so the
    state stays put to rounding."""
    nx, ny, U = 12, 7, 0.03
    o = oracle_mod.Oracle(nx, ny, oracle_mod.PERIODIC_Y | oracle_mod.INLET | oracle_mod.OUTFLOW |
                          oracle_mod.SCHEME_ORIGINAL)
    o.set_geometry(np.zeros((ny, nx), np.uint8))
    o.set_params(0.0, 0.0, 0.8)
    o.set_inlet_velocity(np.full(ny, U), np.zeros(ny))
    f = np.zeros((2, 9, ny, nx))
    f[0] = _feq(np.full((ny, nx), 1.0), U, 0.0)
    f[1] = _feq(np.full((ny, nx), 0.2), U, 0.0)
    o.init_fields(np.ones((ny, nx)), np.ones((ny, nx)))
    o.set_populations(f)
    o.step(200)
    assert np.max(np.abs(o.get_populations().reshape(f.shape) - f)) < 1e-15


def test_outflow_copies_the_upstream_neighbour(oracle_mod):
    """Zero normal gradient: after streaming, the populations entering the
    outflow column from outside (directions 3, 6, 7) equal those of the
    column upstream in the same row, exactly (both come from the same
    post-collision value)."""
    nx, ny = 11, 9
    o = oracle_mod.Oracle(nx, ny, oracle_mod.INLET | oracle_mod.OUTFLOW)
    o.set_geometry(_channel(ny, nx))
    o.set_params(0.9, -0.1, 0.9)
    o.set_inlet_velocity(np.full(ny, 0.02), np.zeros(ny))
    rng = np.random.default_rng(2)
    o.init_fields(1 + 0.1 * rng.random((ny, nx)), 0.1 + 0.1 * rng.random((ny, nx)))
    o.step(4)
    f = o.get_populations().reshape(2, 9, ny, nx)
    for i in (3, 6, 7):
        # rows whose source row y - e_iy is fluid
        rows = range(2, ny - 2)
        for y in rows:
            assert np.array_equal(f[:, i, y, -1], f[:, i, y, -2]), (i, y)


def test_open_edge_stencil_uniform_field_has_no_force(oracle_mod):
    """A uniform mixture in an open channel (periodic in y): the ghost
    positions beyond the inlet and outflow read the uniform value, so the
    cohesion and adhesion forces vanish at every node, edges included
    (with zeros beyond the edge they would not)."""
    nx, ny = 10, 8
    o = oracle_mod.Oracle(nx, ny, oracle_mod.PERIODIC_Y | oracle_mod.INLET | oracle_mod.OUTFLOW)
    o.set_geometry(np.zeros((ny, nx), np.uint8))
    o.set_params(0.9, 0.2, 1.0)
    o.set_inlet_velocity(np.zeros(ny), np.zeros(ny))
    o.init_fields(np.full((ny, nx), 0.7), np.full((ny, nx), 0.3))
    for x in (0, 1, nx - 2, nx - 1):
        out = o.node_forces(x, 3).ravel()
        assert np.all(out[:8] == 0.0), x


def test_open_edge_second_layer_copy(oracle_mod):
    """A field that varies only across the channel, g_k(y).  The node one
    column inside an open edge misses the second-layer positions two
    columns out.  Those at (2, 0) and (2, +-1) copy, by Table 1 (Sec. 2.4),
    the in-domain first-layer nodes of the same rows, which hold what an
    x-uniform extension would; those at (2, +-2) copy the diagonal
    first-layer nodes, one row nearer.  So the cohesion differs from an
    interior node's by exactly the two diagonal terms,
    -G_c psi_k W(8) e_n [g(y+-1) - g(y+-2)], W(8) = 1/5040, and the
    adhesion (walls continue through the ghosts) not at all."""
    nx, ny, Gc = 12, 12, 0.9
    o = oracle_mod.Oracle(nx, ny, oracle_mod.INLET | oracle_mod.OUTFLOW)
    o.set_geometry(_channel(ny, nx))
    o.set_params(Gc, 0.15, 1.0)
    o.set_inlet_velocity(np.zeros(ny), np.zeros(ny))
    yy = np.arange(ny)
    g1 = 0.5 + 0.4 * np.tanh((yy - 5.3) / 1.7)
    g = [g1, 1.03 - g1]
    o.init_fields(np.repeat(g[0][:, None], nx, 1), np.repeat(g[1][:, None], nx, 1))
    mid, W8 = nx // 2, 1.0 / 5040.0
    for y in range(3, ny - 3):
        ref = o.node_forces(mid, y)
        for x, sgn in ((1, -1.0), (nx - 2, 1.0)):
            got = o.node_forces(x, y)
            for k in range(2):
                h = g[1 - k]
                dp, dm = h[y + 1] - h[y + 2], h[y - 1] - h[y - 2]
                pre = -Gc * g[k][y] * W8
                want = ref[k] + pre * np.array([sgn * 2 * (dp + dm), 2 * (dp - dm)])
                assert np.allclose(got[k], want, rtol=0, atol=1e-15), (x, y, k)
            assert np.array_equal(got[2:4], ref[2:4]), (x, y)
    for y in (1, 2, ny - 3, ny - 2):
        s_mid = o.adhesion_vector(mid, y)
        for x in (0, 1, nx - 2, nx - 1):
            assert np.array_equal(o.adhesion_vector(x, y), s_mid), (x, y)


def test_open_boundaries_need_a_non_periodic_x(oracle_mod):
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.Oracle(10, 10, oracle_mod.PERIODIC_X | oracle_mod.INLET)
    o = oracle_mod.Oracle(10, 10, oracle_mod.INLET)
    with pytest.raises(oracle_mod.OracleError):
        o.set_inlet_velocity(np.full(10, 1.0), np.zeros(10))
