import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.lib()
    return oracle


def pytest_terminal_summary(terminalreporter):
    gu = sys.modules.get("gpu_util")
    if gu is None:
        return
    st = gu.RELERR_STATS
    if st["columns"]:
        terminalreporter.write_line(
            f"normwise relative error: {st['columns']} columns checked against ||y_ref||, "
            f"{st['scale_denominator']} of them divided by the cancellation scale (||y_ref|| tiny)")
