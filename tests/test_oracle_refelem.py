"""Pins of the oracle's reference element (Section 4 discretization): exactness
on polynomials of total degree <= k against closed-form monomial integrals and
derivatives, which a wrong basis, node or weight formula would fail."""
from math import factorial

import numpy as np
import pytest

from oracle.refelem import RefElem, nodes, conical_rule


def monomials(k):
    return [(a, b) for a in range(k + 1) for b in range(k + 1 - a)]


def exact_int(a, b):
    # integral over T0 of u^a v^b = a! b! / (a + b + 2)!
    return factorial(a) * factorial(b) / factorial(a + b + 2)


@pytest.mark.parametrize("k", range(1, 8))
def test_nodes_interior_unisolvent(k):
    uv = nodes(k)
    assert uv.shape == ((k + 1) * (k + 2) // 2, 2)
    assert (uv > 0).all() and (uv.sum(1) < 1).all()
    re = RefElem(k, k + 2)
    assert np.linalg.cond(re.V) < 1e3


@pytest.mark.parametrize("k", range(1, 8))
def test_weights_positive_and_exact(k):
    re = RefElem(k, k + 2)
    assert (re.w_ref > 0).all()
    for a, b in monomials(k):
        f = re.uv[:, 0] ** a * re.uv[:, 1] ** b
        assert abs(re.w_ref @ f - exact_int(a, b)) < 1e-14


@pytest.mark.parametrize("k", [2, 4, 6, 7])
def test_interpolation_and_derivatives_exact(k):
    re = RefElem(k, k + 3)
    rng = np.random.default_rng(k)
    pts = rng.uniform(0, 1, (40, 2))
    pts = pts[pts.sum(1) < 1]
    pts = np.vstack([pts, [[0, 0], [1, 0], [0, 1]]])   # vertices included
    L = re.interp(pts)
    for a, b in monomials(k):
        fn = re.uv[:, 0] ** a * re.uv[:, 1] ** b
        assert np.abs(L @ fn - pts[:, 0] ** a * pts[:, 1] ** b).max() < 1e-12
        du = a * re.uv[:, 0] ** max(a - 1, 0) * re.uv[:, 1] ** b if a > 0 else 0 * fn
        dv = b * re.uv[:, 0] ** a * re.uv[:, 1] ** max(b - 1, 0) if b > 0 else 0 * fn
        assert np.abs(re.Du @ fn - du).max() < 1e-11
        assert np.abs(re.Dv @ fn - dv).max() < 1e-11


@pytest.mark.parametrize("q", [3, 6, 10])
def test_conical_rule_exact(q):
    U, W = conical_rule(q)
    for a in range(2 * q - 1):
        for b in range(2 * q - 1 - a):
            assert abs(W @ (U[:, 0] ** a * U[:, 1] ** b) - exact_int(a, b)) < 1e-15
