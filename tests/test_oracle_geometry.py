"""Pins of the oracle's discrete geometry (Section 2 surface calculus, Section 4
weights/normals/mean curvature): areas and mean curvatures with closed forms,
converging under refinement."""
import numpy as np
import pytest
from scipy.special import ellipeinc, ellipkinc

import lbinputs as I
from oracle.geometry import Geometry
from oracle.refelem import nodes


def ellipsoid_area(a, b, c):
    # a >= b >= c (Legendre's form)
    phi = np.arccos(c / a)
    m = a * a * (b * b - c * c) / (b * b * (a * a - c * c))
    s = np.sin(phi)
    return 2 * np.pi * c * c + 2 * np.pi * a * b / s * (ellipeinc(phi, m) * s * s + ellipkinc(phi, m) * np.cos(phi) ** 2)


def test_sphere_area_normals_curvature_converge():
    k = 4
    errs = []
    for nsub in (1, 2):
        X, Xu, Xv = I.sphere_patches(nsub, nodes(k))
        g = Geometry(X, Xu, Xv, k)
        assert np.abs(g.n - g.x).max() < 1e-13          # outward normal = position
        errs.append((abs(g.area - 4 * np.pi), np.abs(g.H - 1).max()))
    assert errs[0][0] < 2e-4 and errs[0][1] < 3e-2
    assert errs[1][0] < errs[0][0] / 30                  # ~h^(k+2)
    assert errs[1][1] < errs[0][1] / 8                   # ~h^(k-1)


def test_torus_area_and_curvature():
    k, R, r = 5, 2.0, 0.7
    X, Xu, Xv = I.torus_patches(R, r, 12, 24, nodes(k))
    g = Geometry(X, Xu, Xv, k)
    assert abs(g.area - 4 * np.pi ** 2 * R * r) < 1e-8 * g.area
    Hex = I.torus_mean_curvature(g.x, R, r)
    assert np.abs(g.H - Hex).max() < 1e-4
    # outward orientation
    rho = np.linalg.norm(g.x[:, :2], axis=1, keepdims=True)
    centre = np.concatenate([g.x[:, :2] / rho * R, 0 * g.x[:, 2:]], 1)
    assert ((g.x - centre) * g.n).sum(1).min() > 0


def test_ellipsoid_area():
    k = 6
    X, Xu, Xv = I.ellipsoid_patches(2, nodes(k), (1.0, 1.5, 2.0))
    g = Geometry(X, Xu, Xv, k)
    ex = ellipsoid_area(2.0, 1.5, 1.0)
    assert abs(g.area - ex) < 1e-7 * ex


def test_near_lists_contain_self_and_close_patches():
    k = 4
    X, Xu, Xv = I.sphere_patches(1, nodes(k))
    g = Geometry(X, Xu, Xv, k)
    nl = g.near_lists()
    for i, l in enumerate(nl):
        assert g.patch_of[i] in l
        d = np.linalg.norm(g.x[i] - g.c, axis=1)
        assert set(np.nonzero(d < g.eta * g.R)[0]) | {g.patch_of[i]} == set(l)
