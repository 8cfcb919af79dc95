import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for p in (ROOT, os.path.dirname(os.path.abspath(__file__))):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU statistics test")


def pytest_terminal_summary(terminalreporter):
    """Errors against the FP64 oracle that the GPU tests recorded."""
    gc = sys.modules.get("gpu_common")
    if gc is None or not getattr(gc, "MEASURED", None):
        return
    terminalreporter.section("measured errors against the FP64 oracle (worst per test)")
    for (test, what), v in sorted(gc.MEASURED.items()):
        terminalreporter.write_line(f"{v:10.3e}  {what:32s} {test}")
