"""CPU checks of the C-ABI library: it loads, and it exports every symbol
that include/lbm.h and include/lbm3d.h declare (no compute calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions(headers=("lbm.h", "lbm3d.h")):
    names = []
    for h in headers:
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?\**\s*\**\b(lbm(?:3d)?_[a-z0-9_]+)\s*\(",
                            text, flags=re.M)
    return sorted(set(names))


def test_every_header_is_checked():
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == ["lbm.h", "lbm3d.h"]


def test_header_declares_the_boundary():
    names = _declared_functions()
    for core in ("lbm_create", "lbm_set_geometry", "lbm_set_params", "lbm_step", "lbm_get_fields",
                 "lbm_reduce", "lbm_contact_angle", "lbm_get_tables", "lbm_batch_create"):
        assert core in names
    assert len(names) >= 30
    for core in ("lbm3d_create", "lbm3d_set_geometry", "lbm3d_step", "lbm3d_get_fields", "lbm3d_reduce",
                 "lbm3d_contact_angle", "lbm_reduce_noalloc"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2505_22256_amd import build, lbm
    build.build(force=False)
    L = ctypes.CDLL(lbm.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2505_22256_amd import lbm
    assert set(_declared_functions()) == set(lbm.SIGNATURES)


def test_binding_refuses_missing_library(tmp_path):
    from paper_2505_22256_amd import lbm
    saved = lbm._lib
    try:
        lbm._lib = None
        try:
            lbm.load_library(str(tmp_path / "absent.so"))
        except RuntimeError as e:
            assert "not built" in str(e)
        else:
            raise AssertionError("missing library must raise")
    finally:
        lbm._lib = saved


def test_flag_and_code_values_match_the_header():
    from paper_2505_22256_amd import lbm
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    for name in ("PERIODIC_X", "PERIODIC_Y", "SCHEME_ORIGINAL", "E8_COPY_OFF", "WALLPSI_SELF",
                 "VEL_LITERAL", "FORCE_DENSITY", "ROUND_STOCHASTIC", "INLET", "OUTFLOW", "SCHED_ALIGN", "SCHED_BANDS", "SCHED_XCD_SLABS", "SCHED_TWO_STEP", "F64", "F32", "F16", "BF16", "EINVAL", "ESTATE",
                 "EDEVICE", "EUNSTABLE", "WALL_FLAT", "WALL_CYLINDER", "ROUND_NEAREST"):
        m = re.search(r"LBM_%s\s*=\s*(-?\d+)" % name, text)
        assert m, name
        assert int(m.group(1)) == getattr(lbm, name), name
    text3 = open(os.path.join(ROOT, "include", "lbm3d.h")).read()
    for name in ("PERIODIC_Z", "WALL_FLAT", "WALL_SPHERE"):
        m = re.search(r"LBM3D_%s\s*=\s*(-?\d+)" % name, text3)
        assert m, name
        assert int(m.group(1)) == getattr(lbm, "L3_" + name), name


def test_population_bytes():
    """Size of one caller-provided population buffer (host arithmetic only):
    18 elements of the storage type per node, 0 for refused sizes."""
    from paper_2505_22256_amd import lbm
    assert lbm.lbm_population_bytes(7, 5, lbm.F64) == 7 * 5 * 18 * 8
    assert lbm.lbm_population_bytes(16384, 2048, lbm.F32) == 16384 * 2048 * 18 * 4
    assert lbm.lbm_population_bytes(9, 6, lbm.F16) == 9 * 6 * 18 * 2
    assert lbm.lbm_population_bytes(9, 6, lbm.BF16) == 9 * 6 * 18 * 2
    assert lbm.lbm_population_bytes(4, 6, lbm.F32) == 0
    assert lbm.lbm_population_bytes(9, 6, 7) == 0
