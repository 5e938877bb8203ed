import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def _ensure_cpu_libs():
    """The oracle and the input generator are plain C; build them if nothing is built yet."""
    import oracle
    from paper_2304_09953_amd import inputs
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    if not os.path.exists(inputs.LIB_PATH):
        from paper_2304_09953_amd import build as pkg_build
        pkg_build.build_inputs()


_ensure_cpu_libs()


@pytest.fixture(scope="session")
def p48():
    from paper_2304_09953_amd import inputs as I
    return I.workload("pocket48-lib100")


@pytest.fixture(scope="session")
def p48_grid(p48):
    import oracle
    return oracle.build_grids(p48.pockets[0])


@pytest.fixture(scope="session")
def p48_ligs(p48):
    return p48.ligands()
