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


def normwise_state(a, b, ns, rho_c):
    """normwise() for a conserved state, with the momentum rows measured
    against max(max|b|, rho_c): a pressure roundoff of eps*p per cell
    produces momentum errors of order eps*rho*c per acoustic time whatever
    the flow speed, so a flow near rest has a tiny max|rho u| that measures
    roundoff amplification rather than disagreement."""
    import numpy as np
    a = np.asarray(a, float).reshape(a.shape[0], -1)
    b = np.asarray(b, float).reshape(b.shape[0], -1)
    den = np.abs(b).max(axis=1)
    den[ns:ns + 3] = np.maximum(den[ns:ns + 3], rho_c)
    num = np.abs(a - b).max(axis=1)
    return np.where(den > 0, num / np.where(den > 0, den, 1), num)


EPS = 2.0 ** -52


def flux_floor(U, p, xi_max, ns):
    """Rounding bound of a conservative flux difference, per conserved
    variable: 100 eps xi_max max|F_v|, with |F_v| bounded by |U_v| |u| (+ p for
    momentum, + p |u| for energy).  A face flux is a handful of terms of size
    max|F|; the difference of two faces times the metric carries an error of
    a few ulps of max|F| xi, whatever the size of the difference itself."""
    import numpy as np
    U = np.asarray(U, float)
    rho = U[:ns].sum(axis=0)
    speed = np.sqrt((U[ns:ns + 3] ** 2).sum(axis=0)) / rho
    F = np.abs(U) * speed[None]
    F[ns:ns + 3] += p[None]
    F[ns + 3] += p * speed
    return 100 * EPS * xi_max * F.max(axis=1)


def rhs_close(a, b, floor, rel=1e-12):
    """Per conserved variable: max|a-b| <= max(rel max|b|, floor).  Returns
    (ok, ratio) with ratio = max|a-b| / max(rel max|b|, floor)."""
    import numpy as np
    a = np.asarray(a, float).reshape(a.shape[0], -1)
    b = np.asarray(b, float).reshape(b.shape[0], -1)
    lim = np.maximum(rel * np.abs(b).max(axis=1), floor)
    r = np.abs(a - b).max(axis=1) / np.where(lim > 0, lim, 1)
    return bool(np.all(r <= 1.0)), r


def golden(name):
    """Rows of a cited text fixture under tests/golden/ (comment lines
    starting with '#' skipped), each split on commas."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    with open(path) as fh:
        return [ln.strip().split(",") for ln in fh if ln.strip() and not ln.startswith("#")]
