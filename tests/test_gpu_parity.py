"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances
  FP64 storage and arithmetic: relative 1e-12 on populations and densities
    after 1000 steps (the two sides differ only in the rounding order of
    the same formulas).
  FP32 (deviation storage, FP32 arithmetic): density error at most 1e-4 of
    the field maximum.
  FP16 / BF16 storage: contact angle within 1 degree of the FP64 oracle.
  Integer work (tables) and invariances (tiling, batching, checkpoints):
    bit-exact.
"""
import numpy as np
import pytest

from paper_2505_22256_amd import workloads as W

pytestmark = pytest.mark.gpu

REL64 = 1e-12


def _pair(oracle_mod, lbm_mod, wl, storage, flags_extra=0, pops=None, tile=None, adhesion=None):
    # stochastic rounding concerns reduced-precision storage only; the FP64
    # oracle has no such flag
    o = oracle_mod.Oracle(wl.nx, wl.ny, (wl.flags | flags_extra) & ~(lbm_mod.ROUND_STOCHASTIC | lbm_mod.ROUND_NEAREST))
    g = lbm_mod.Lattice(wl.nx, wl.ny, storage, wl.flags | flags_extra)
    for s in (o, g):
        s.set_geometry(wl.solid)
        s.set_params(wl.G_c, wl.G_ads, wl.tau)
        if adhesion is not None:
            s.set_adhesion(*adhesion)
        s.set_body_accel(*wl.accel)
        if pops is None:
            s.init_fields(wl.rho1, wl.rho2)
        else:
            s.set_populations(pops)
    if tile is not None:
        g.set_tile(*tile)
    return o, g


def _relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_fp64_flat_drop_1000_steps(oracle_mod, lbm_mod):
    """Flat-wall droplet (100x50, improved scheme, lambda = 13/9), FP64."""
    wl = W.flat_drop()
    o, g = _pair(oracle_mod, lbm_mod, wl, lbm_mod.F64, tile=(64, 8))
    o.step(1000)
    g.step(1000)
    assert g.time == 1000
    assert _relmax(g.get_populations(), o.get_populations()) < REL64
    for a, b in zip(g.get_fields(), o.get_fields()):
        assert np.max(np.abs(a - b)) < REL64 * max(np.max(np.abs(b)), 1e-3)


FLAG_CASES = [0, 4, 8, 16, 32, 64, 4 | 8 | 16]


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("extra", FLAG_CASES)
def test_fp64_random_geometry_random_populations(oracle_mod, lbm_mod, seed, extra):
    """Random blobs and a non-equilibrium start, with every reading flag;
    periodic and walled variants alternate with the seed."""
    periodic = (W.PERIODIC_X | W.PERIODIC_Y) if seed % 2 == 0 else W.PERIODIC_X
    wl = W.random_small(seed, nx=23 + seed, ny=17 + 2 * seed, flags=periodic, walls=seed % 2 == 1)
    f0 = W.random_populations(seed + 50, wl)
    o, g = _pair(oracle_mod, lbm_mod, wl, lbm_mod.F64, flags_extra=extra, pops=f0,
                 tile=(64, 4 + seed))
    o.step(200)
    g.step(200)
    assert _relmax(g.get_populations(), o.get_populations()) < REL64


def _speckled(seed, nx, ny, flags, frac=0.25):
    """Random masks with a quarter of the nodes solid, placed one by one:
    most solid features are a single voxel thick, so second-layer stencil
    positions often lie just beyond a one-node wall (Sec. 2.4, Table 1:
    the copy then takes the first-layer value on the near side), and
    fluid nodes enclosed on several sides are common."""
    rng = np.random.default_rng(seed)
    solid = (rng.random((ny, nx)) < frac).astype(np.uint8)
    y, x = np.mgrid[0:ny, 0:nx]
    inside = (x - nx * rng.uniform(0.3, 0.7)) ** 2 + (y - ny * rng.uniform(0.3, 0.7)) ** 2 < (min(nx, ny) / 3) ** 2
    rho1 = np.where(solid != 0, 0.0, np.where(inside, 1.0, 0.03))
    rho2 = np.where(solid != 0, 0.0, np.where(inside, 0.03, 1.0))
    return W.Workload("speckled", nx, ny, flags, solid, rho1, rho2, G_c=0.9,
                      G_ads=float(rng.uniform(-0.3, 0.3)), tau=float(rng.uniform(0.8, 1.2)),
                      accel=(1e-5, -2e-5, -1e-5, 3e-5), steps=200)


@pytest.mark.parametrize("seed,periodic", [(0, 3), (1, 1), (2, 0), (3, 2)])
@pytest.mark.parametrize("extra", [0, 8, 16])
def test_fp64_one_voxel_features(oracle_mod, lbm_mod, seed, periodic, extra):
    """Dynamics on speckled masks (one-voxel-thick solids everywhere), from
    random populations, with the Table 1 copy, without it (E8_COPY_OFF) and
    with WALLPSI_SELF: 200 steps of the device against the oracle at 1e-12
    (two tiles, so strip and segment edges cut through the speckle)."""
    wl = _speckled(700 + seed, 37 + 3 * seed, 29 + 2 * seed, periodic)
    f0 = W.random_populations(710 + seed, wl, amplitude=0.1)
    ref = None
    for tile in ((64, 5), (128, 16)):
        o, g = _pair(oracle_mod, lbm_mod, wl, lbm_mod.F64, flags_extra=extra, pops=f0, tile=tile)
        if ref is None:
            o.step(200)
            ref = o.get_populations()
            assert np.all(np.isfinite(ref))
        g.step(200)
        assert _relmax(g.get_populations(), ref) < REL64, tile


def test_fp64_multitile_ragged_nonperiodic(oracle_mod, lbm_mod):
    """Several strips and segments with ragged tails, no periodic axis
    (outside = solid), random blobs."""
    wl = W.random_small(11, nx=301, ny=71, flags=0, n_blobs=12, walls=False)
    f0 = W.random_populations(12, wl)
    for tile in ((64, 8), (128, 13), (256, 71)):
        o, g = _pair(oracle_mod, lbm_mod, wl, lbm_mod.F64, pops=f0, tile=tile)
        o.step(150)
        g.step(150)
        assert _relmax(g.get_populations(), o.get_populations()) < REL64, tile


def test_fp64_cylinder_shortened(oracle_mod, lbm_mod):
    """Droplet on the staircase cylinder (400x400), 200 steps."""
    wl = W.cylinder_drop(G_ads=-0.2)
    o, g = _pair(oracle_mod, lbm_mod, wl, lbm_mod.F64)
    o.step(200)
    g.step(200)
    for a, b in zip(g.get_fields(), o.get_fields()):
        assert np.max(np.abs(a - b)) < REL64 * max(np.max(np.abs(b)), 1e-3)


@pytest.mark.parametrize("seed,flags", [(s, f) for s in range(4) for f in (0, 1, 2, 3)])
def test_tables_bit_exact(oracle_mod, lbm_mod, seed, flags):
    rng = np.random.default_rng(300 + seed)
    nx, ny = int(rng.integers(5, 40)), int(rng.integers(5, 30))
    solid = (rng.random((ny, nx)) < 0.2).astype(np.uint8)
    for extra in (0, 8, 16):
        o = oracle_mod.Oracle(nx, ny, flags | extra)
        o.set_geometry(solid)
        g = lbm_mod.Lattice(nx, ny, lbm_mod.F32, flags | extra)
        g.set_geometry(solid)
        g.set_params(0.9, 0.0, 1.0)
        g.init_fields(np.where(solid, 0, 0.7), np.where(solid, 0, 0.3))
        ol, on, osrc = o.get_tables()
        gl, gn, gsrc = g.get_tables()
        assert np.array_equal(ol, gl)
        assert np.array_equal(on, gn)
        assert np.array_equal(osrc, gsrc)


def test_tables_cylinder_bit_exact(oracle_mod, lbm_mod):
    wl = W.cylinder_drop()
    o = oracle_mod.Oracle(wl.nx, wl.ny, wl.flags)
    o.set_geometry(wl.solid)
    _, g = _pair(oracle_mod, lbm_mod, wl, lbm_mod.F16)
    for a, b in zip(o.get_tables(), g.get_tables()):
        assert np.array_equal(a, b)


def test_reduce_matches_oracle(oracle_mod, lbm_mod):
    wl = W.flat_drop()
    o, g = _pair(oracle_mod, lbm_mod, wl, lbm_mod.F64)
    o.step(300)
    g.step(300)
    ro, rg = o.reduce(), g.reduce()
    for q in (0, 1, 4, 5, 6):
        assert abs(rg[q] - ro[q]) <= 1e-12 * abs(ro[q])
    for q in (2, 3):  # momenta: near zero, compare against the mass scale
        assert abs(rg[q] - ro[q]) <= 1e-12 * ro[0]
    assert rg[7] == 0


def test_contact_angle_matches_oracle(oracle_mod, lbm_mod):
    wl = W.flat_drop()
    o, g = _pair(oracle_mod, lbm_mod, wl, lbm_mod.F64)
    o.step(1500)
    g.step(1500)
    to = o.contact_angle(0, wl.wall)
    tg = g.contact_angle(0, wl.wall)
    assert abs(tg - to) < 1e-8


def test_contact_angle_of_synthetic_cap(lbm_mod):
    """Same construction as the oracle's pin: a tanh cap cut by a flat wall
    at a known angle, read back by the device fit."""
    nx, ny, r, theta = 160, 60, 40.0, 60.0
    yc = 0.5 - r * np.cos(np.radians(theta))
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    s = np.tanh((r - np.hypot(x - nx / 2, y - yc)) / 2.0)
    solid = np.zeros((ny, nx), np.uint8)
    solid[0] = 1
    solid[-1] = 1
    g = lbm_mod.Lattice(nx, ny, lbm_mod.F64, lbm_mod.PERIODIC_X)
    g.set_geometry(solid)
    g.set_params(0.9, 0.0, 1.0)
    g.init_fields(np.where(solid, 0, 0.52 + 0.43 * s), np.where(solid, 0, 0.52 - 0.43 * s))
    assert abs(g.contact_angle(0, (0.5, 0, 0)) - theta) < 0.3


@pytest.mark.parametrize("storage", [0, 1, 2, 3])
def test_uniform_fluid_stays_exactly_at_rest(lbm_mod, storage):
    nx, ny = 70, 40
    g = lbm_mod.Lattice(nx, ny, storage, 3)
    g.set_geometry(np.zeros((ny, nx), np.uint8))
    g.set_params(0.9, 0.1, 0.8)
    g.init_fields(np.full((ny, nx), 0.91), np.full((ny, nx), 0.13))
    g.step(30)
    r1, r2, ux, uy = g.get_fields()
    assert np.all(ux == 0) and np.all(uy == 0)
    assert np.all(r1 == r1[0, 0]) and np.all(r2 == r2[0, 0])


def test_tiling_does_not_change_results(lbm_mod):
    wl = W.cylinder_drop(G_ads=0.1, nx=200, ny=180, R=30, centre=(100, 70), r_drop=25,
                         drop_centre=(100, 115))
    ref = None
    for tile in ((64, 8, 0), (128, 32, 1), (256, 64, 2), (256, 7, 3), (256, 0, 0), (128, 0, 1), (256, 0, 5), (64, 0, 4)):
        g = lbm_mod.lattice_from_workload(wl, lbm_mod.F32)
        g.set_tile(*tile)
        g.step(100)
        f = g.get_populations()
        if ref is None:
            ref = f
        else:
            assert np.array_equal(f, ref), tile


def test_fp32_flat_drop_density(oracle_mod, lbm_mod):
    wl = W.flat_drop()
    o, g = _pair(oracle_mod, lbm_mod, wl, lbm_mod.F32)
    o.step(1000)
    g.step(1000)
    ro, go = o.get_fields(), g.get_fields()
    for k in (0, 1):
        assert np.max(np.abs(go[k] - ro[k])) <= 1e-4 * np.max(np.abs(ro[k]))


@pytest.mark.parametrize("storage,flags,tol", [(1, 0, 0.5), (2, 0, 1.0), (3, 0, 1.0), (2, 128, 1.0)])
def test_reduced_storage_contact_angle(oracle_mod, lbm_mod, storage, flags, tol):
    """Flat-wall droplet after 5000 steps: contact angle against the FP64
    oracle, 0.5 degree for FP32 storage and 1 degree for FP16 / BF16
    storage in their default rounding (stochastic; giving the flag
    explicitly is the same).  (With LBM_ROUND_NEAREST the FP16 / BF16 runs
    miss by 5 / 11 degrees: the rounding error of a steady state repeats
    every step and drains mass; see the next test.)"""
    wl = W.flat_drop()
    o, g = _pair(oracle_mod, lbm_mod, wl, storage, flags_extra=flags)
    o.step(5000)
    g.step(5000)
    to = o.contact_angle(0, wl.wall)
    tg = g.contact_angle(0, wl.wall)
    assert abs(tg - to) < tol, (to, tg)


@pytest.mark.parametrize("storage,bound", [(2, 1e-3), (3, 8e-3)])
def test_stochastic_rounding_removes_mass_drift(oracle_mod, lbm_mod, storage, bound):
    """The oracle conserves each component's mass to rounding.  Nearest-even
    FP16 / BF16 storage loses mass steadily (linear in the step count);
    stochastic rounding is unbiased, so its mass only random-walks.  Size of
    that walk: each stored deviation |g| ~ 0.1-0.2 carries a rounding error
    of standard deviation ulp/sqrt(6); 4500 values per component per step
    over 3000 steps give a relative standard deviation of about 2e-3 for
    BF16 (ulp 2^-10 at that size) and 2.5e-4 for FP16 (ulp 2^-13).  The
    bound is four of those; the drift must also be well below nearest-even's."""
    wl = W.flat_drop()
    o = oracle_mod.Oracle(wl.nx, wl.ny, wl.flags)
    o.set_geometry(wl.solid)
    o.set_params(wl.G_c, wl.G_ads, wl.tau)
    o.init_fields(wl.rho1, wl.rho2)
    m0 = o.reduce()[:2]
    drift = {}
    for fl in (lbm_mod.ROUND_NEAREST, 0):
        g = lbm_mod.lattice_from_workload(wl, storage, fl)
        assert bool(g.flags_in_effect() & lbm_mod.ROUND_STOCHASTIC) == (fl == 0)
        g.step(3000)
        m = g.reduce()[:2]
        drift[fl] = np.max(np.abs(m - m0) / m0)
    assert drift[0] < 0.25 * drift[lbm_mod.ROUND_NEAREST], drift
    assert drift[0] < bound, drift


def test_rounding_flags_in_effect(lbm_mod):
    """16-bit storage rounds stochastically unless LBM_ROUND_NEAREST is
    given; FP32 and FP64 carry neither bit; both bits together are
    refused."""
    SR, RNE = lbm_mod.ROUND_STOCHASTIC, lbm_mod.ROUND_NEAREST
    want = {(lbm_mod.F16, 0): SR, (lbm_mod.BF16, 0): SR, (lbm_mod.F16, SR): SR, (lbm_mod.BF16, RNE): RNE,
            (lbm_mod.F32, 0): 0, (lbm_mod.F32, SR): 0, (lbm_mod.F64, RNE): 0}
    for (storage, fl), bits in want.items():
        g = lbm_mod.Lattice(16, 12, storage, 3 | fl)
        assert g.flags_in_effect() & (SR | RNE) == bits, (storage, fl)
        assert g.flags_in_effect() & 3 == 3
        g.close()
    for storage in (lbm_mod.F16, lbm_mod.F32):
        with pytest.raises(lbm_mod.LbmError):
            lbm_mod.Lattice(16, 12, storage, SR | RNE)


def test_checkpoint_resume_is_bitwise(lbm_mod, tmp_path):
    wl = W.flat_drop()
    a = lbm_mod.lattice_from_workload(wl, lbm_mod.F16)
    a.step(70)
    path = str(tmp_path / "ck.bin")
    a.save(path)
    a.step(50)
    b = lbm_mod.Lattice(wl.nx, wl.ny, lbm_mod.F16, wl.flags)
    b.load(path)
    assert b.time == 70
    b.step(50)
    assert np.array_equal(a.get_populations(), b.get_populations())


def test_populations_window_matches_full(lbm_mod):
    wl = W.cylinder_drop(nx=120, ny=110, R=20, centre=(60, 40), r_drop=18, drop_centre=(60, 70))
    g = lbm_mod.lattice_from_workload(wl, lbm_mod.F32)
    g.step(20)
    full = g.get_populations()
    win = g.get_populations_window(110, 100, 20, 15)  # wraps both axes
    xs = (110 + np.arange(20)) % 120
    ys = (100 + np.arange(15)) % 110
    assert np.array_equal(win, full[:, :, ys][:, :, :, xs])


def test_errors_and_call_order(lbm_mod):
    L = lbm_mod
    with pytest.raises(L.LbmError) as e:
        L.Lattice(4, 10)
    assert e.value.code == L.EINVAL
    g = L.Lattice(10, 10, L.F32, 3)
    with pytest.raises(L.LbmError) as e:
        g.step(1)
    assert e.value.code == L.ESTATE
    g.set_geometry(np.zeros((10, 10), np.uint8))
    for bad in ((0.9, 0.0, 0.5), (0.9, -0.45, 1.0), (0.9, -0.6, 1.0), (float("nan"), 0, 1)):
        with pytest.raises(L.LbmError) as e:
            g.set_params(*bad)
        assert e.value.code == L.EINVAL
    with pytest.raises(L.LbmError) as e:
        g.set_adhesion(1.0, 1.0, 0.8)  # before set_params
    assert e.value.code == L.ESTATE
    g.set_params(0.9, 0.0, 1.0)
    with pytest.raises(L.LbmError) as e:
        g.set_adhesion(1.0, -1.0, 0.8)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LbmError) as e:
        g.init_fields(np.full((10, 10), np.nan), np.ones((10, 10)))
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LbmError) as e:
        g.set_tile(100, 4)
    assert e.value.code == L.EINVAL
    g.init_fields(np.full((10, 10), 0.5), np.full((10, 10), 0.5))
    g.step(3)
    with pytest.raises(L.LbmError) as e:
        g.contact_angle(0, (0.5, 0, 0))  # no interface
    assert e.value.code == L.EUNSTABLE


def _pocket_workload():
    """Tanh cap on a cylinder at 110 degrees, with a component-2 pocket
    inside the droplet next to the wall and a satellite droplet."""
    n, R, r, C, theta = 160, 30.0, 25.0, (80.0, 60.0), 110.0
    Rs = R + 0.5
    d = np.sqrt(Rs * Rs + r * r - 2 * Rs * r * np.cos(np.radians(theta)))
    y, x = np.mgrid[0:n, 0:n].astype(float)
    solid = (((x - C[0]) ** 2 + (y - C[1]) ** 2) < R * R).astype(np.uint8)
    s = np.tanh((r - np.hypot(x - C[0], y - C[1] - d)) / 2.0)
    for (cx, cy, rb, sign) in ((C[0], C[1] + R + 9.0, 5.0, -1.0), (20.0, 150.0, 6.0, 1.0)):
        sb = np.tanh((rb - np.hypot(x - cx, y - cy)) / 2.0)
        s = np.where(sb > -0.999, sign * sb, s)
    rho1 = np.where(solid, 0, 0.52 + 0.43 * s)
    rho2 = np.where(solid, 0, 0.52 - 0.43 * s)
    return W.Workload("pocket", n, n, W.PERIODIC_X | W.PERIODIC_Y, solid, rho1, rho2, G_c=0.9, G_ads=0.0,
                      tau=1.0, wall_kind=W.WALL_CYLINDER, wall=(C[0], C[1], Rs))


def test_contact_angle_ignores_pocket_and_satellite(oracle_mod, lbm_mod):
    """The device labels the phase regions (union-find) and fits only the
    interface between the largest region of each sign, as the oracle does
    (breadth-first labelling): same angle, single context and batch."""
    wl = _pocket_workload()
    o, g = _pair(oracle_mod, lbm_mod, wl, lbm_mod.F64)
    to = o.contact_angle(wl.wall_kind, wl.wall)
    assert abs(to - 110.0) < 0.3
    assert abs(g.contact_angle(wl.wall_kind, wl.wall) - to) < 1e-9
    b = lbm_mod.Batch([W.flat_drop(nx=64, ny=40, radius=12), wl], lbm_mod.F64)
    assert abs(b.contact_angles()[1] - to) < 1e-9


def _small_runs():
    runs = [W.flat_drop(nx=64, ny=40, radius=12, G_ads=0.1, tau=0.8),
            W.cylinder_drop(G_ads=-0.2, nx=96, ny=90, R=14, centre=(48, 34), r_drop=18,
                            drop_centre=(48, 60), tau=1.1),
            W.flat_drop(nx=130, ny=47, radius=15, G_ads=-0.25, tau=1.0),
            W.random_small(7, nx=37, ny=29)]
    runs[3].wall_kind, runs[3].wall = 0, (0.5, 0.0, 0.0)
    return runs


@pytest.mark.parametrize("storage,flags,two,block", [(1, 0, False, 128), (2, 128, False, 128), (0, 0, False, 128),
                                                      (1, 0, True, 128), (2, 128, True, 128), (3, 0, True, 128),
                                                      (1, 0, True, 256)])
def test_batch_equals_single_runs_bitwise(lbm_mod, storage, flags, two, block):
    runs = _small_runs()
    for wl in runs:
        wl.flags |= flags
    b = lbm_mod.Batch(runs, storage)
    b.set_tile(block, 16)
    if two:
        b.set_sched(8)  # two fused steps per launch
    b.use_graph(True, 10)
    b.step(57)  # five graph replays and seven single launches
    singles = []
    for wl in runs:
        g = lbm_mod.lattice_from_workload(wl, storage)
        g.set_tile(64, 8)
        g.step(57)
        singles.append(g)
    for r, g in enumerate(singles):
        for a, c in zip(b.get_fields(r), g.get_fields()):
            assert np.array_equal(a, c), r
    th = b.contact_angles()
    for r in (0, 1, 2):
        assert th[r] == singles[r].contact_angle(runs[r].wall_kind, runs[r].wall)


def test_batch_against_oracle_fp64(oracle_mod, lbm_mod):
    runs = _small_runs()[:3]
    b = lbm_mod.Batch(runs, lbm_mod.F64)
    b.step(120)
    for r, wl in enumerate(runs):
        o = oracle_mod.Oracle(wl.nx, wl.ny, wl.flags)
        o.set_geometry(wl.solid)
        o.set_params(wl.G_c, wl.G_ads, wl.tau)
        o.init_fields(wl.rho1, wl.rho2)
        o.step(120)
        for a, c in zip(b.get_fields(r), o.get_fields()):
            assert np.max(np.abs(a - c)) < REL64 * max(np.max(np.abs(c)), 1e-3)


def test_fused_diagnostics_match_reduce(lbm_mod):
    wl = W.flat_drop()
    g = lbm_mod.lattice_from_workload(wl, lbm_mod.F64)
    g.set_diag_interval(50)
    g.step(100)  # records at t = 0 and t = 50
    d, t = g.get_diag()
    assert t == 50
    h = lbm_mod.lattice_from_workload(wl, lbm_mod.F64)
    h.step(50)
    r = h.reduce()
    for q in (0, 1, 4, 5, 6, 7):
        assert abs(d[q] - r[q]) <= 1e-12 * max(abs(r[q]), 1.0)
