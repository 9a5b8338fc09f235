import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: oracle cases that take tens of seconds")


def golden(name):
    return os.path.join(ROOT, "tests", "golden", name)


def read_remarks():
    out = {}
    with open(golden("paper_remarks.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, val = line.split()[:2]
            out[key] = float(val)
    return out


def read_test3():
    """{(scaling, primal, H/h): (lit, cond)} of the paper's Test 3 slab
    table (None where the paper reports out of memory)."""
    out = {}
    with open(golden("paper_test3_slab.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            sc, pr, hh, lit, cond = line.split()[:5]
            out[(sc, pr, int(hh))] = None if lit == "oom" else (float(lit), float(cond))
    return out
