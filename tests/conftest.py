import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) device")
    config.addinivalue_line("markers", "slow: CPU test that runs for more than a few seconds")


def load_paper_values():
    """Values printed in the paper: {key: (value, unit, citation)}."""
    out = {}
    with open(os.path.join(GOLDEN, "paper_values.txt")) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            key, val, unit, cite = line.split(None, 3)
            out[key] = (float(val), float(unit), cite.strip())
    return out


def load_coexistence_table():
    """Rows of tests/golden/coexistence.txt keyed by T/Tc."""
    eps = (0.0, 1.0, 1.86, 2.0)
    rows = {}
    with open(os.path.join(GOLDEN, "coexistence.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [float(x) for x in line.split()]
            r = {"T": v[1], "spinodal": (v[2], v[3]), "maxwell": (v[4], v[5], v[6])}
            for k, e in enumerate(eps):
                g, l = v[7 + 2 * k], v[8 + 2 * k]
                r[("eq9", e)] = None if np.isnan(g) else (g, l)
            rows[round(v[0], 3)] = r
    return rows


@pytest.fixture(scope="session")
def paper_values():
    return load_paper_values()


@pytest.fixture(scope="session")
def coexistence_table():
    return load_coexistence_table()
