import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def normwise(a, b):
    """max over cells |a-b| / max over cells |b|, per leading-axis row (a
    conserved variable); rows where b is identically zero use the absolute
    difference."""
    import numpy as np
    a = np.asarray(a, float).reshape(a.shape[0], -1)
    b = np.asarray(b, float).reshape(b.shape[0], -1)
    den = np.abs(b).max(axis=1)
    num = np.abs(a - b).max(axis=1)
    return np.where(den > 0, num / np.where(den > 0, den, 1), num)
