"""pytest configuration: the ``gpu`` marker and in-tree native builds.

Tests marked ``gpu`` call the HIP library through its C ABI and need an
MI355X; everything else runs on the CPU.  Native libraries are built in-tree
only when they are missing (``__graft_entry__.build()`` rebuilds them).
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X; runs the HIP path through the C ABI")


@pytest.fixture(scope="session", autouse=True)
def _native_libs():
    import oracle
    from paper_1504_07499_amd import _build

    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build(force=True)
    if not os.path.exists(_build.geom_lib_path()):
        _build.build_geom()
    yield
