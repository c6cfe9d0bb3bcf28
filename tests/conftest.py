import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def read_golden(name):
    """Parse tests/golden/<name>: 'key value' lines; '...' suffix kept as a
    flag meaning 'only the printed digits are pinned'."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split(None, 1)
            prefix = val.endswith("...")
            out[key] = (val[:-3] if prefix else val, prefix)
    return out


def matches_printed(value, printed):
    """True when `value` agrees with a printed decimal: exactly when the
    documentation printed the full number, else to the printed digits."""
    text, prefix = printed
    ref = float(text)
    if not prefix:
        return value == ref
    decimals = len(text.split(".")[1]) if "." in text else 0
    return abs(value - ref) < 10.0 ** (-decimals)
