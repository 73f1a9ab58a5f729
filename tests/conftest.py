"""Shared pytest configuration.

Markers
  gpu   needs an MI355X (gfx950) and the built HIP library; parity and
        device-side checks.  Everything else runs on the CPU.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU run (oracle physics), skipped with -m 'not slow'")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    """Name every GPU case on the real stderr before it runs, so that a run
    that ends abruptly still shows which case was on the device."""
    if request.node.get_closest_marker("gpu") is not None:
        sys.__stderr__.write(f"[gpu case] {request.node.nodeid}\n")
        sys.__stderr__.flush()
    yield


@pytest.fixture(scope="session")
def lbm_mod():
    from paper_2505_22256_amd import lbm
    lbm.load_library()
    return lbm
