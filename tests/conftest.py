import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run through the C-ABI on the device)")
    config.addinivalue_line("markers", "slow: long CPU test")


GOLDEN = os.path.join(ROOT, "tests", "golden")


def load_example31():
    """Example 3.1 fixture: returns A, B, [(lambda, x)]."""
    import numpy as np
    A, B, eig = [], [], []
    with open(os.path.join(GOLDEN, "example31.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tag, *vals = line.split()
            vals = [float(v) for v in vals]
            if tag == "A":
                A.append(vals)
            elif tag == "B":
                B.append(vals)
            elif tag == "EIG":
                eig.append((vals[0], np.array(vals[1:], dtype=np.complex128)))
    return (np.array(A, dtype=np.complex128), np.array(B, dtype=np.complex128), eig)
