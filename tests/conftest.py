import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Report every parity tie of the session (decisions whose margin is
    below the tie bound, which a different rounding order may flip)."""
    try:
        import parity
    except ImportError:
        return
    ties = parity.TIES
    terminalreporter.write_sep("-", f"parity ties: {len(ties)}")
    for t in ties:
        terminalreporter.write_line(f"  {t['what']}: imf {t['imf']} sift {t['sift']}: "
                                    f"{t['detail']}")
