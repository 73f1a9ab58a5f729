"""Full-size checks on the 16384 x 2048 constriction channel, in the launch
configuration the benchmark times (the library's default tile: two fused
steps per launch for FP32 and FP16), and on the 2048 x 1024 porous
channel of the precision study (FP64, anchored at t = 1000).

The oracle cannot step the whole lattice in test time, so it checks sampled
nodes one by one: the update of node x from t to t+1 reads only positions
within Chebyshev distance 3 of x (pull sources at distance 1, whose forces
read the E8 stencil at distance 2 around them), so the oracle stepped n
times on the (6n+1) x (6n+1) window of f(t) around x (taken from the device)
must reproduce the device's f(x, t+n); n is the number of steps the
device fuses into one launch.  Whole-lattice properties (mass conservation, no
non-finite value) are checked at full size.
"""
import numpy as np
import pytest

from paper_2505_22256_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def channel():
    return W.constrictions()


def _samples(wl, n_each=16, seed=7):
    rng = np.random.default_rng(seed)
    fluid = np.argwhere(wl.solid == 0)
    # nodes next to a solid (within distance 3) exercise bounce-back,
    # the second-layer copy and the adhesion force
    from scipy.ndimage import binary_dilation
    near = binary_dilation(wl.solid.astype(bool), iterations=3) & (wl.solid == 0)
    near_idx = np.argwhere(near)
    seam = fluid[(fluid[:, 1] < 3) | (fluid[:, 1] >= wl.nx - 3)]
    pick = lambda a: a[rng.choice(len(a), n_each, replace=False)]
    return np.concatenate([pick(fluid), pick(near_idx), pick(seam)])


def _oracle_steps(oracle_mod, wl, f_win, y0, x0, h, w, n=1):
    ys = np.arange(y0, y0 + h)
    xs = (x0 + np.arange(w)) % wl.nx
    mask = wl.solid[np.ix_(ys, xs)]
    o = oracle_mod.Oracle(w, h, 0)  # the window edges do not reach the centre in n steps
    o.set_geometry(mask)
    o.set_params(wl.G_c, wl.G_ads, wl.tau)
    o.set_body_accel(*wl.accel)
    o.set_populations(f_win)
    o.step(n)
    return o.get_populations()


# Tolerances: FP64 storage and arithmetic, 1e-12 relative (rounding order
# only).  FP32 storage and arithmetic, a few ulps of the largest
# population (~0.45): 2e-6 relative.  FP16 and BF16 store the deviation
# g = f - w rho0 with rho0 the mean density (0.5 here), so |g| <= ~0.25:
# an FP16 ulp there is 2^-12 (2.4e-4, 5.4e-4 of the largest population
# 0.45); stochastic rounding (the default) errs by less than one ulp,
# nearest-even by half of one; 8e-4 allows either after two fused steps.
# BF16 (8 significant bits): an ulp of 2^-9 at |g| = 0.25, 4.3e-3 of the
# largest population; 8e-3 allows it.
RNE = 1024
FULL_TOLS = [(0, 0, 1e-12), (1, 0, 2e-6), (2, 0, 8e-4), (3, 0, 8e-3), (2, RNE, 8e-4), (3, RNE, 8e-3)]


@pytest.mark.parametrize("storage,flags,tol", FULL_TOLS)
def test_sampled_nodes_against_oracle(oracle_mod, lbm_mod, channel, storage, flags, tol):
    wl = channel
    g = lbm_mod.lattice_from_workload(wl, storage, flags)
    n = 2 if g.get_tile()[2] & lbm_mod.SCHED_TWO_STEP else 1
    rad = 3 * n
    g.step(40)
    samples = _samples(wl)
    before = []
    for (y, x) in samples:
        y0 = max(0, y - rad)
        h = min(wl.ny, y + rad + 1) - y0
        w = 2 * rad + 1
        before.append((y0, x - rad, h, w, g.get_populations_window(x - rad, y0, w, h)))
    g.step(n)  # one launch
    worst = 0.0
    for (y, x), (y0, x0, h, w, f_win) in zip(samples, before):
        after = g.get_populations_window(x, y, 1, 1)[:, :, 0, 0]
        ref = _oracle_steps(oracle_mod, wl, f_win, y0, x0, h, w, n)[:, :, y - y0, rad]
        scale = np.max(np.abs(ref))
        err = np.max(np.abs(after - ref)) / scale
        worst = max(worst, err)
        assert err < tol, (int(y), int(x), err)
    print(f"storage {storage}: worst relative error over {n} step(s) {worst:.2e}, {len(samples)} nodes")


def test_porous_fp64_anchor_at_1000_steps(oracle_mod, lbm_mod):
    """The FP64 device run that the precision study compares the reduced
    storages with: after 1000 steps on the porous channel (14 % of fluid
    nodes near a wall), sampled nodes advance one more step exactly as the
    oracle advances their 7 x 7 windows (1e-12 relative)."""
    wl = W.porous()
    g = lbm_mod.lattice_from_workload(wl, lbm_mod.F64)
    g.autotune(1)
    g.step(1000)
    samples = _samples(wl, n_each=24, seed=11)
    before = []
    for (y, x) in samples:
        y0 = max(0, y - 3)
        h = min(wl.ny, y + 4) - y0
        before.append((y0, x - 3, h, 7, g.get_populations_window(x - 3, y0, 7, h)))
    g.step(1)
    for (y, x), (y0, x0, h, w, f_win) in zip(samples, before):
        after = g.get_populations_window(x, y, 1, 1)[:, :, 0, 0]
        ref = _oracle_steps(oracle_mod, wl, f_win, y0, x0, h, w)[:, :, y - y0, 3]
        assert np.max(np.abs(after - ref)) <= 1e-12 * np.max(np.abs(ref)), (int(y), int(x))
    m = g.reduce()
    assert m[7] == 0


def test_full_lattice_mass_and_finiteness(lbm_mod, channel):
    wl = channel
    g = lbm_mod.lattice_from_workload(wl, lbm_mod.F32)
    g.step(1)  # default tile: the benchmark configuration
    m0 = g.reduce()
    g.step(200)
    m1 = g.reduce()
    assert m1[7] == 0
    for k in (0, 1):
        assert abs(m1[k] - m0[k]) / m0[k] < 1e-5
    # the body force drives both components along +x
    assert m1[2] > 0


def _open_samples(wl, seed=5):
    """Random fluid and near-wall nodes, plus nodes of the four columns at
    each open edge (the Zou-He unknowns, the outflow copy, the E8 ghosts
    and Table 1 copies beyond the edge)."""
    rng = np.random.default_rng(seed)
    base = _samples(wl, n_each=12, seed=seed)[:24]
    edge_cols = [0, 1, 2, 3, wl.nx - 4, wl.nx - 3, wl.nx - 2, wl.nx - 1]
    ys = rng.integers(1, wl.ny - 1, size=len(edge_cols))
    ys[:2] = 1           # the inlet corner on the bottom wall
    ys[-2:] = wl.ny - 2  # the outflow corner on the top wall
    edge = np.array([(y, x) for y, x in zip(ys, edge_cols) if wl.solid[y, x] == 0])
    return np.concatenate([base, edge])


@pytest.mark.parametrize("moving", [False, True])
@pytest.mark.parametrize("storage,tol", [(st, tol) for st, fl, tol in FULL_TOLS if fl == 0])
def test_open_channel_sampled_nodes_against_oracle(oracle_mod, lbm_mod, storage, tol, moving):
    """The channel with a Zou-He inlet and an outflow instead of periodic x,
    in the launch configuration of the open-channel benchmark (default
    tile, boundary kernel instances): sampled nodes, open-edge columns
    included, advance one launch as the oracle advances their windows; a
    window that reaches an open edge carries that edge (and the inlet
    velocities of its rows).  With `moving`, every wall (channel walls and
    constrictions) also slides at u_x = 0.01: the same velocity in both
    halves, so that a window takes it whatever rows it covers."""
    wl = W.constrictions(open_ends=True)
    if moving:
        wl.wall_velocity = (0.01, 0.0, 0.01, 0.0)
    g = lbm_mod.lattice_from_workload(wl, storage)
    n = 2 if g.get_tile()[2] & lbm_mod.SCHED_TWO_STEP else 1
    # the dependence radius is 3 per step; at least 4, so that a window cut
    # by an open edge still has the 5 columns a lattice needs
    rad = max(3 * n, 4)
    g.step(41)
    samples = _open_samples(wl)
    before = []
    for (y, x) in samples:
        y0, x0 = max(0, y - rad), max(0, x - rad)
        h, w = min(wl.ny, y + rad + 1) - y0, min(wl.nx, x + rad + 1) - x0
        before.append((y0, x0, h, w, g.get_populations_window(x0, y0, w, h)))
    g.step(n)
    for (y, x), (y0, x0, h, w, f_win) in zip(samples, before):
        flags = (W.INLET if x0 == 0 else 0) | (W.OUTFLOW if x0 + w == wl.nx else 0)
        o = oracle_mod.Oracle(w, h, flags)
        o.set_geometry(wl.solid[y0:y0 + h, x0:x0 + w])
        o.set_params(wl.G_c, wl.G_ads, wl.tau)
        o.set_body_accel(*wl.accel)
        o.set_inlet_velocity(wl.inlet_u[0, y0:y0 + h], wl.inlet_u[1, y0:y0 + h])
        if moving:
            o.set_wall_velocity(*wl.wall_velocity)
        o.set_populations(f_win)
        o.step(n)
        ref = o.get_populations()[:, :, y - y0, x - x0]
        after = g.get_populations_window(x, y, 1, 1)[:, :, 0, 0]
        err = np.max(np.abs(after - ref)) / np.max(np.abs(ref))
        assert err < tol, (int(y), int(x), err)
