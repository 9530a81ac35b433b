"""Pins of the oracle's near/far split and of its self-patch rule that do not
restate the oracle's own formulas.

Near lists and patch radii (Section 4, the Near/Far split, read as
Near(x) = {l : |x - c_l| < eta R_l}): the centre c_l is the area centroid of
patch l and R_l the largest distance from it to a point of the patch.  Both
are recomputed here from the analytic chart alone, sampled densely (a 24 x 24
collapsed Gauss rule from numpy for the centroid, a barycentric lattice with
vertices and edges for the radius), and the oracle's values and lists must
agree with them up to the chart's interpolation error; the property the
split exists for, every point of a far patch at distance >= (eta - 1) R_l,
is checked by brute force over the dense samples.

Self rule (Duffy triangles, sinh-graded edge variable, principal value of
the gradient, the displacement from the node formed as the integral of the
chart's derivative along the ray): the default 16 radial x 12 edge points
against 24 x 20.  The S column agrees to 3e-13 (sphere, order 4) .. 3e-11
(ellipsoid, order 6) of its largest entry, the gradient and S' columns to
5e-12 .. 6e-11, S''+D' to 5e-11 .. 1e-9: on the interpolated chart the
target's given normal is not exactly orthogonal to the chart's tangents, so
the S''+D' kernel keeps a 1/r^2 part whose coefficient is the chart's
interpolation error (odd in direction, a principal value that Gauss rules
resolve only algebraically), far below the discretization error of these
surfaces (1e-5 .. 1e-7).  Translating the surface leaves the self integrals
unchanged up to rounding (translation by 10 moves them by < 1e-11 of each
column's largest entry): no cancellation of nearly equal positions.
"""
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

import lbinputs as I
from oracle.geometry import Geometry
from oracle.quad import self_integrals
from oracle.refelem import nodes


def _collapsed_rule(n):
    x, w = leggauss(n)
    a = 0.5 * (x + 1.0)
    wa = 0.5 * w
    A, B = np.meshgrid(a, a, indexing="ij")
    WA, WB = np.meshgrid(wa, wa, indexing="ij")
    u = A.ravel()
    v = ((1.0 - A) * B).ravel()
    return np.stack([u, v], 1), (WA * WB * (1.0 - A)).ravel()


def _lattice(m):
    pts = [(i / m, j / m) for i in range(m + 1) for j in range(m + 1 - i)]
    return np.array(pts)


def _surface(name):
    if name == "sphere":
        return (lambda uv: I.sphere_patches(1, uv)), 4
    if name == "ellipsoid":
        return (lambda uv: I.ellipsoid_patches(1, uv, (1.0, 1.5, 2.0))), 6
    return (lambda uv: I.torus_patches(2.0, 0.7, 6, 16, uv)), 4


@pytest.mark.parametrize("name", ["sphere", "ellipsoid", "torus"])
def test_near_lists_and_radii_against_dense_charts(name):
    chart, k = _surface(name)
    g = Geometry(*chart(nodes(k)), k)
    quv, qw = _collapsed_rule(24)
    Xq, Xuq, Xvq = chart(quv)
    J = np.linalg.norm(np.cross(Xuq, Xvq), axis=-1)
    c_ref = (Xq * (J * qw)[..., None]).sum(1) / (J * qw).sum(1)[:, None]
    Xl = chart(_lattice(40))[0]                              # (NP, m, 3) dense points of each patch
    R_ref = np.linalg.norm(Xl - c_ref[:, None, :], axis=-1).max(1)
    size = R_ref.max()
    ec = np.abs(g.c - c_ref).max() / size
    eR = np.abs(g.R - R_ref).max() / size
    print(f"{name}: centroid {ec:.1e}, radius {eR:.1e} of the largest radius")
    assert ec < 1e-4 and eR < 1e-3
    eta = g.eta
    near = g.near_lists()
    d_ref = np.linalg.norm(g.x[:, None, :] - c_ref[None, :, :], axis=-1)      # (N, NP)
    in_ref = d_ref < eta * R_ref[None, :]
    in_ref[np.arange(g.N), g.patch_of] = True
    in_orc = np.zeros_like(in_ref)
    for i, a in enumerate(near):
        in_orc[i, a] = True
    diff = np.argwhere(in_ref != in_orc)
    margin = np.abs(d_ref - eta * R_ref[None, :]) / (eta * R_ref[None, :])
    print(f"{name}: {in_orc.sum()} near pairs, {len(diff)} differ from the dense construction")
    assert in_orc.sum() > 3 * g.N
    assert all(margin[i, l] < 2e-3 for i, l in diff)
    # far patches: every dense point at distance >= (eta - 1) R from the node
    rows = np.arange(0, g.N, max(1, g.N // 150))
    for i in rows:
        far = np.flatnonzero(~in_orc[i])
        dmin = np.linalg.norm(Xl[far] - g.x[i], axis=-1).min(1)
        assert np.all(dmin >= (eta - 1.0) * R_ref[far] * (1.0 - 2e-3))


def _flat():
    T = np.array([[0.0, 0.0, 0.0], [1.0, 0.2, 0.1], [0.3, 0.9, -0.2]])
    uv = nodes(6)
    X = T[0] + uv[:, 0:1] * (T[1] - T[0]) + uv[:, 1:2] * (T[2] - T[0])
    return Geometry(X[None], np.tile(T[1] - T[0], (len(uv), 1))[None], np.tile(T[2] - T[0], (len(uv), 1))[None], 6)


@pytest.mark.parametrize("name", ["flat", "sphere", "ellipsoid"])
def test_self_rule_converged(name):
    """Default self rule (16 x 12) against 24 x 20 on sampled targets, column
    by column (S, dS/dx1..3, S', S''+D', D), relative to each column's
    largest entry; on the flat triangle S', S''+D' and D vanish and are held
    absolutely."""
    if name == "flat":
        g = _flat()
    else:
        chart, k = _surface(name)
        g = Geometry(*chart(nodes(k)), k)
    t = np.arange(0, min(g.N, 240), 4)
    a = self_integrals(g, t)
    b = self_integrals(g, t, ns=24, nt=20)
    sc = np.abs(b).max(axis=(0, 1))
    d = np.abs(a - b).max(axis=(0, 1))
    print(name, " ".join(f"{x:.1e}" for x in d / sc))
    assert np.all(d[0] < 1e-10 * sc[0])
    assert np.all(d[1:4] < 1e-10 * sc[1:4])
    if name == "flat":
        assert np.all(d[4:] < 1e-11)
    else:
        assert d[4] < 2e-10 * sc[4]
        assert d[5] < 3e-9 * sc[5]
        assert d[6] < 2e-10 * sc[6]


@pytest.mark.parametrize("name", ["sphere", "ellipsoid"])
def test_self_rule_translation_invariant(name):
    """The self integrals of a surface and of its translate by (10, 10, 10)
    agree to rounding: the displacement from the node to a quadrature point
    is not the difference of two positions of size |X|."""
    chart, k = _surface(name)
    X, Xu, Xv = chart(nodes(k))
    t = np.arange(0, 240, 7)
    a = self_integrals(Geometry(X, Xu, Xv, k), t)
    b = self_integrals(Geometry(X + 10.0, Xu, Xv, k), t)
    sc = np.abs(a).max(axis=(0, 1))
    d = np.abs(a - b).max(axis=(0, 1)) / sc
    print(name, " ".join(f"{x:.1e}" for x in d))
    assert np.all(d[:5] < 2e-11) and d[5] < 1e-10 and d[6] < 2e-11
