import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """List every FP64 comparison that missed 1e-12 against the FP64 oracle
    and was accepted against the long-double oracle (tests/parity_checks.py)."""
    mod = sys.modules.get("tests.parity_checks")
    fb = getattr(mod, "FALLBACKS", None) if mod else None
    if fb is None:
        return
    terminalreporter.write_sep("-", f"FP64 long-double fallbacks: {len(fb)}")
    for label, e, e_gpu, e_or in fb:
        terminalreporter.write_line(f"{label}: gpu vs fp64 oracle {e:.2e}; vs long double gpu {e_gpu:.2e}, "
                                    f"fp64 oracle {e_or:.2e}")
