import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: larger CPU cases")
    config.addinivalue_line("markers", "sym_expanded: symmetric CSR planned as expanded full rows on small systems")


@pytest.fixture(autouse=True)
def _symmetric_plans(request, monkeypatch):
    """Small symmetric-CSR systems are planned as expanded full rows by
    default (the library's choice where launches bound the iteration).  The
    tests keep the scatter plans (compact blocks, coloured ranges) on small
    systems too, so that every edge case reaches those kernels; tests of the
    expanded plan carry the `sym_expanded` marker."""
    if request.node.get_closest_marker("sym_expanded") is None:
        monkeypatch.setenv("CGMI_SYM_EXPAND", "0")
