import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built HIP library")


@pytest.fixture(scope="session")
def c1_oracle():
    """Unit sphere, 80 order-4 patches (N = 1200), all rows of the oracle."""
    from oracle.refelem import nodes
    from oracle.geometry import Geometry
    from oracle.ops import Oracle
    import lbinputs as I
    uv = nodes(4)
    X, Xu, Xv = I.sphere_patches(1, uv)
    g = Geometry(X, Xu, Xv, 4)
    return Oracle(g)


def rel_l2(a, b, w=None):
    a = np.asarray(a)
    b = np.asarray(b)
    if w is None:
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
    w = np.asarray(w)
    d = ((a - b) ** 2).reshape(len(w), -1).sum(1)
    r = (b ** 2).reshape(len(w), -1).sum(1)
    return float(np.sqrt((w * d).sum() / (w * r).sum()))


def max_row(a, b):
    """Largest row error relative to the largest row of b: max_i |a_i - b_i| / max_i |b_i|
    (rows: the first axis; a row's norm is the Euclidean norm of its entries)."""
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    d = np.linalg.norm((a - b).reshape(len(b), -1), axis=1)
    r = np.linalg.norm(b.reshape(len(b), -1), axis=1)
    return float(d.max() / r.max())
