"""Pins of the oracle's wall treatment: the adhesion vector S(x) (Eq. 9 on
the E8 stencil), cohesion next to a wall with the second-layer copy of
Sec. 2.4 / Table 1, and the link and source tables against a brute-force
geometric construction.

Closed forms for a flat wall below fluid (wall row y = 0, periodic in x),
from the E8 weights W(1)=4/21, W(2)=4/45, W(4)=1/60, W(5)=2/315, W(8)=1/5040:
  row 1: the unavailable positions are every e with e_y < 0, so
         S_y = -(W1 + 2 W2 + 2 W4 + 2*2 W8 + 2 W5 + 2*2 W5) = -37/84;
  row 2: only e_y = -2 is unavailable: S_y = -(2 W4 + 2*2 W8 + 2*2 W5) = -5/84;
  row 3 and above: S = 0.
"""
import itertools

import numpy as np
import pytest

from paper_2505_22256_amd import workloads as W

S_ROW1 = -37.0 / 84.0
S_ROW2 = -5.0 / 84.0


def _flat(oracle_mod, flags=0, nx=12, ny=12, a=0.8, b=0.2, Gc=0.9):
    solid = np.zeros((ny, nx), np.uint8)
    solid[0] = 1
    solid[-1] = 1
    o = oracle_mod.Oracle(nx, ny, oracle_mod.PERIODIC_X | flags)
    o.set_geometry(solid)
    o.set_params(Gc, 0.0, 1.0)
    o.init_fields(np.where(solid, 0, a), np.where(solid, 0, b))
    return o


def test_flat_wall_adhesion_vector(oracle_mod):
    """P5 -- S(x) = sum W s(x+e) e next to a flat wall."""
    o = _flat(oracle_mod)
    for x in (0, 5, 11):
        assert np.allclose(o.adhesion_vector(x, 1), [0, S_ROW1], rtol=0, atol=1e-16)
        assert np.allclose(o.adhesion_vector(x, 2), [0, S_ROW2], rtol=0, atol=1e-16)
        assert np.all(o.adhesion_vector(x, 3) == 0) and np.all(o.adhesion_vector(x, 6) == 0)
        # the top wall mirrors the bottom one
        assert np.allclose(o.adhesion_vector(x, 10), [0, -S_ROW1], rtol=0, atol=1e-16)
        assert np.allclose(o.adhesion_vector(x, 9), [0, -S_ROW2], rtol=0, atol=1e-16)


def test_flat_wall_cohesion_with_second_layer_copy(oracle_mod):
    """P6 -- uniform densities a, b next to a flat wall.
    Row 1: unavailable first-layer positions give 0 and their second-layer
    partners copy them, so F_1 = -G a b (-S_row1) = -G a b 37/84 along y.
    Row 2: the copy fills the y = 0 positions from row 1, so F = 0 exactly
    up to rounding (without the copy it would be -G a b 5/84).
    Adhesion force = -G_w rho S with G_w1 = G_w2 = G_c at G_ads = 0."""
    a, b, G = 0.8, 0.2, 0.9
    o = _flat(oracle_mod, a=a, b=b, Gc=G)
    p1 = o.node_forces(4, 1)
    assert abs(p1[0, 1] - (-G * a * b * 37 / 84)) < 1e-15 and p1[0, 0] == 0
    assert abs(p1[1, 1] - (-G * b * a * 37 / 84)) < 1e-15
    assert abs(p1[2, 1] - (-G * a * S_ROW1)) < 1e-15     # adhesion comp 1 (lambda = 1)
    assert abs(p1[3, 1] - (-G * b * S_ROW1)) < 1e-15
    p2 = o.node_forces(4, 2)
    assert abs(p2[0, 1]) < 1e-16 and abs(p2[1, 1]) < 1e-16
    assert abs(p2[2, 1] - (-G * a * S_ROW2)) < 1e-15
    p3 = o.node_forces(4, 3)
    assert np.all(np.abs(p3[:4]) < 1e-16)

    off = _flat(oracle_mod, flags=oracle_mod.E8_COPY_OFF, a=a, b=b, Gc=G)
    q2 = off.node_forces(4, 2)
    assert abs(q2[0, 1] - (-G * a * b * 5 / 84)) < 1e-15
    assert abs(off.node_forces(4, 1)[0, 1] - (-G * a * b * 37 / 84)) < 1e-15

    selfp = _flat(oracle_mod, flags=oracle_mod.WALLPSI_SELF, a=a, b=b, Gc=G)
    # own value substituted for the wall: a uniform field sees no gradient
    assert np.all(np.abs(selfp.node_forces(4, 1)[:2]) < 1e-16)
    assert np.all(np.abs(selfp.node_forces(4, 2)[:2]) < 1e-16)


def test_adhesion_uses_local_parameter_only_for_component_1(oracle_mod):
    """Eq. 9-11: component 1 uses G(x) of Eq. 11 evaluated at the node's
    effective density (Eq. 10); component 2 keeps G_w2."""
    a, b = 0.9, 0.3
    o = _flat(oracle_mod, a=a, b=b)
    o.set_adhesion(1.3, 0.9, 0.8)
    re = (a - b) / (a + b)
    G1 = oracle_mod.local_G(re, 1.3, 0.9, 0.8)
    p = o.node_forces(3, 1)
    assert abs(p[2, 1] - (-G1 * a * S_ROW1)) < 1e-15
    assert abs(p[3, 1] - (-0.9 * b * S_ROW1)) < 1e-15
    orig = _flat(oracle_mod, flags=oracle_mod.SCHEME_ORIGINAL, a=a, b=b)
    orig.set_adhesion(1.3, 0.9, 0.8)
    q = orig.node_forces(3, 1)
    assert abs(q[2, 1] - (-1.3 * a * S_ROW1)) < 1e-15


def test_body_force_forms(oracle_mod):
    a, b = 0.7, 0.4
    o = _flat(oracle_mod, a=a, b=b)
    o.set_body_accel(1e-3, -2e-3, 3e-3, 4e-3)
    p = o.node_forces(5, 5)
    assert np.allclose(p[4], [a * 1e-3, -a * 2e-3], rtol=1e-15)
    assert np.allclose(p[5], [b * 3e-3, b * 4e-3], rtol=1e-15)
    d = _flat(oracle_mod, flags=oracle_mod.FORCE_DENSITY, a=a, b=b)
    d.set_body_accel(1e-3, -2e-3, 3e-3, 4e-3)
    assert np.allclose(d.node_forces(5, 5)[4], [1e-3, -2e-3], rtol=1e-15)


# --------------------------------------------------------------------------
# P17: tables against a brute-force geometric construction
# --------------------------------------------------------------------------

D2Q9 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def _padded_available(solid, flags, pad=2):
    """Availability on a padded grid: wrap periodic axes, mark the outside
    as unavailable along the others."""
    ny, nx = solid.shape
    fluid = (solid == 0).astype(np.int8)
    mode_y = "wrap" if flags & 2 else "constant"
    mode_x = "wrap" if flags & 1 else "constant"
    g = np.pad(fluid, ((pad, pad), (0, 0)), mode=mode_y)
    g = np.pad(g, ((0, 0), (pad, pad)), mode=mode_x)
    return g  # g[y + pad, x + pad] = available(x, y)


def _brute_tables(solid, flags):
    ny, nx = solid.shape
    pad = 2
    av = _padded_available(solid, flags, pad)
    def padax(a, widths, periodic):
        return np.pad(a, widths, mode="wrap") if periodic else \
            np.pad(a, widths, mode="constant", constant_values=-1)

    idx = padax(np.arange(nx * ny).reshape(ny, nx), ((pad, pad), (0, 0)), flags & 2)
    idx = padax(idx, ((0, 0), (pad, pad)), flags & 1)
    link = np.zeros((ny, nx), np.uint8)
    nw, srcs = [], []
    offsets = [(dx, dy) for dy in range(-2, 3) for dx in range(-2, 3) if (dx, dy) != (0, 0)]
    for y, x in itertools.product(range(ny), range(nx)):
        if solid[y, x]:
            continue
        for i in range(1, 9):
            ex, ey = D2Q9[i]
            if not av[y - ey + pad, x - ex + pad]:
                link[y, x] |= 1 << (i - 1)
        if all(av[y + dy + pad, x + dx + pad] for dx, dy in offsets):
            continue
        nw.append(y * nx + x)
        # resolve by geometry: an unavailable position at distance 2 takes the
        # neighbour one step along (sign dx, sign dy), which resolves to its
        # own node or, if unavailable, to zero (-1).
        res = {}
        for dx, dy in offsets:
            if max(abs(dx), abs(dy)) == 1:
                res[(dx, dy)] = idx[y + dy + pad, x + dx + pad] if av[y + dy + pad, x + dx + pad] else -1
        for dx, dy in offsets:
            if max(abs(dx), abs(dy)) == 2:
                if av[y + dy + pad, x + dx + pad]:
                    res[(dx, dy)] = idx[y + dy + pad, x + dx + pad]
                else:
                    res[(dx, dy)] = res[(int(np.sign(dx)), int(np.sign(dy)))]
        srcs.append(res)
    return link, nw, srcs


@pytest.mark.parametrize("seed,flags", [(s, f) for s in range(6) for f in (0, 1, 2, 3)])
def test_tables_against_brute_force(oracle_mod, seed, flags):
    rng = np.random.default_rng(100 + seed)
    nx, ny = int(rng.integers(5, 13)), int(rng.integers(5, 13))
    solid = (rng.random((ny, nx)) < 0.25).astype(np.uint8)
    o = oracle_mod.Oracle(nx, ny, flags)
    o.set_geometry(solid)
    link, lst, src = o.get_tables()
    blink, bnw, bsrc = _brute_tables(solid, flags)
    assert np.array_equal(link, blink)
    assert lst.tolist() == bnw
    ex, ey, _, _ = oracle_mod.e8()
    for row, res in zip(src, bsrc):
        for n in range(24):
            assert row[n] == res[(int(ex[n]), int(ey[n]))]


def test_curved_wall_second_layer_is_copied(oracle_mod):
    """A fluid node near a staircase cylinder: every unavailable
    second-layer position reads exactly the value its Table 1 partner reads."""
    wl = W.cylinder_drop(nx=40, ny=40, R=8.0, centre=(20.0, 15.0), r_drop=6.0,
                         drop_centre=(20.0, 28.0))
    o = oracle_mod.Oracle(wl.nx, wl.ny, wl.flags)
    o.set_geometry(wl.solid)
    link, lst, src = o.get_tables()
    _, _, _, cp = oracle_mod.e8()
    copied = 0
    for node, row in zip(lst, src):
        y, x = divmod(int(node), wl.nx)
        for n in range(8, 24):
            px, py = x + oracle_mod.e8()[0][n], y + oracle_mod.e8()[1][n]
            if wl.solid[py % wl.ny, px % wl.nx]:
                assert row[n] == row[cp[n]]
                copied += 1
    assert copied > 50


def test_d2q9_weight_reading_of_the_adhesion_vector(oracle_mod):
    """The alternative reading of Eq. 9's w_i (D2Q9 weights over the eight
    links, an exploration flag of the oracle only): on a flat wall below,
    S = (0, -(1/9 + 2/36)) = (0, -1/6) on the first fluid row and 0 from
    the second row on."""
    nx, ny = 9, 8
    solid = np.zeros((ny, nx), np.uint8)
    solid[0] = 1
    o = oracle_mod.Oracle(nx, ny, oracle_mod.PERIODIC_X | oracle_mod.ADH_D2Q9)
    o.set_geometry(solid)
    o.set_params(0.9, 0.1, 1.0)
    o.init_fields(np.full((ny, nx), 0.5), np.full((ny, nx), 0.5))
    assert np.allclose(o.adhesion_vector(4, 1), [0.0, -1.0 / 6.0], rtol=0, atol=1e-16)
    for y in (2, 3, 4):
        assert np.all(o.adhesion_vector(4, y) == 0.0)
