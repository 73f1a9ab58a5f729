"""Two fused time steps per launch (LBM_SCHED_TWO_STEP) against one step
per launch: the populations must be bitwise identical, for every storage
that allows it, with and without stochastic rounding, periodic and walled
lattices, several tile shapes (also with the first step's rows pulled
again at their finish, LBM_SCHED_REPULL), odd step counts and fused
diagnostics (the steps that record diagnostics run alone); FP64 in its
64- and 128-thread strips.  The FP64 oracle parity tests pin one step per
launch (their explicit tiles) and two (FP64's default)."""
import numpy as np
import pytest

from paper_2505_22256_amd import workloads as W

pytestmark = pytest.mark.gpu

TWO = 8
REPULL = 16


def _cases():
    return [W.random_small(11, nx=37, ny=29),
            W.random_small(12, nx=61, ny=23, flags=W.PERIODIC_X, walls=True),
            W.random_small(13, nx=300, ny=41, flags=0, walls=True),
            W.flat_drop(nx=130, ny=47, radius=15, G_ads=-0.25),
            W.cylinder_drop(G_ads=0.2, nx=96, ny=90, R=14, centre=(48, 34), r_drop=18, drop_centre=(48, 60))]


@pytest.mark.parametrize("storage,flags", [(0, 0), (1, 0), (2, 0), (2, 1024), (3, 0), (3, 1024)])
def test_two_step_is_bitwise_one_step(lbm_mod, storage, flags):
    tiles = [(128, 16, TWO), (64, 8, TWO | 2), (128, 0, TWO), (128, 32, TWO | 3), (64, 0, TWO | 4),
             (256, 24, TWO | 2), (256, 0, TWO), (128, 24, TWO | REPULL | 2), (64, 32, TWO | REPULL | 2),
             (64, 7, TWO | REPULL | 1), (128, 0, TWO | REPULL)]
    if storage == lbm_mod.F64:  # FP64 fuses in 64- or 128-thread strips only
        tiles = [t for t in tiles if t[0] != 256]
    for ci, wl in enumerate(_cases()):
        ref = lbm_mod.lattice_from_workload(wl, storage, flags)
        ref.set_tile(256, 16, 0)
        ref.step(37)
        f_ref = ref.get_populations()
        for tile in tiles:
            g = lbm_mod.lattice_from_workload(wl, storage, flags)
            g.set_tile(*tile)
            g.step(37)
            assert np.array_equal(g.get_populations(), f_ref), (ci, tile)
            g.close()


@pytest.mark.parametrize("storage", [1, 0])
@pytest.mark.parametrize("steps,every,t_diag", [(23, 5, 20), (22, 7, 21), (9, 1, 8), (40, 4, 36)])
def test_two_step_with_fused_diagnostics(lbm_mod, steps, every, t_diag, storage):
    """Diagnostics due on the first or the second of two fused steps are
    recorded inside the fused launch (first step: core nodes only, the halo
    is computed twice); they equal the one-step records to rounding and the
    populations stay bitwise equal."""
    wl = W.random_small(21, nx=70, ny=33, flags=W.PERIODIC_X, walls=True)
    a = lbm_mod.lattice_from_workload(wl, storage)
    a.set_tile(256, 16, 0)
    a.set_diag_interval(every)
    a.step(steps)
    b = lbm_mod.lattice_from_workload(wl, storage)
    b.set_tile(128, 16, TWO | 2)
    b.set_diag_interval(every)
    b.step(steps)
    assert np.array_equal(a.get_populations(), b.get_populations())
    da, ta = a.get_diag()
    db, tb = b.get_diag()
    assert ta == tb == t_diag
    for q in range(8):
        assert abs(da[q] - db[q]) <= 1e-12 * max(abs(da[q]), 1.0), q


def test_repull_needs_two_steps(lbm_mod):
    g = lbm_mod.Lattice(20, 20, lbm_mod.F32, 3)
    with pytest.raises(lbm_mod.LbmError):
        g.set_tile(128, 16, REPULL)
    g.set_tile(128, 16, TWO | REPULL)
    assert tuple(g.get_tile()) == (128, 16, TWO | REPULL)


def test_fp64_two_step_limits(lbm_mod):
    """FP64 fuses two steps in 64- and 128-thread strips; a 256-thread strip
    is refused."""
    for flags in (3, lbm_mod.INLET | lbm_mod.OUTFLOW):
        g = lbm_mod.Lattice(20, 20, lbm_mod.F64, flags)
        assert tuple(g.get_tile()) == (64, 48, TWO | 2)
        g.set_tile(128, 16, TWO)
        g.set_tile(64, 0, TWO)
        with pytest.raises(lbm_mod.LbmError) as e:
            g.set_tile(256, 16, TWO)
        assert e.value.code == lbm_mod.EINVAL


def test_fp64_two_step_with_walls_starting_to_slide(lbm_mod):
    """FP64 with two fused steps whose walls start sliding between calls
    (the steps after that run in the boundary instance of the fused
    kernel): the results of single steps, bitwise."""
    wl = W.random_small(23, nx=50, ny=30, flags=W.PERIODIC_X, walls=True)
    out = []
    for tile in ((256, 16, 0), (64, 16, TWO | 2)):
        g = lbm_mod.lattice_from_workload(wl, lbm_mod.F64)
        g.set_tile(*tile)
        g.step(6)
        g.set_wall_velocity(0.01, 0.0, -0.01, 0.0)
        g.step(9)
        out.append(g.get_populations())
        g.close()
    assert np.array_equal(out[0], out[1])
