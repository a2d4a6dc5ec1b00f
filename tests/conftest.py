import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_libraries():
    """Build the oracle and the input generator if they are not built yet."""
    import oracle
    from paper_2407_07463_amd import synth

    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    if not os.path.exists(synth._LIB_PATH):
        from paper_2407_07463_amd import _build

        _build.build_synth()
    yield


@pytest.fixture(scope="session")
def drops512():
    """The benchmark workload (512^3, 8 FP64 tracers, seeded), generated once
    per session for the full-size parity tests."""
    from paper_2407_07463_amd import synth

    return synth.drops512(order=8, workers=16)
