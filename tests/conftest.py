import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-side oracle runs")


def golden_path(name):
    return os.path.join(ROOT, "tests", "golden", name)


def load_golden_matrix(name):
    rows, extra = [], []
    with open(golden_path(name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                if rows and line.startswith("#"):
                    extra.append(None)
                continue
            vals = [float(x) for x in line.split()]
            if extra:
                extra.append(vals)
            else:
                rows.append(vals)
    return rows, [e for e in extra if e is not None]
