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
    """The FP64 oracle (built on first load if nothing is built yet)."""
    import oracle

    return oracle


@pytest.fixture(scope="session")
def wave_mod():
    """The HIP binding.  Builds the library if nothing is built yet; the
    binding itself raises if the library cannot be loaded."""
    if not os.path.exists(os.path.join(ROOT, "paper_2204_03775_amd", "libwave.so")):
        import __graft_entry__

        __graft_entry__.build()
    from paper_2204_03775_amd import wave

    return wave
