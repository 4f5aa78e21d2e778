import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def wave_mod():
    """The HIP binding.  Builds the library if nothing is built yet; the
    binding itself raises if the library cannot be loaded."""
    from paper_2204_03775_amd import wave

    if not os.path.exists(wave.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    return wave
