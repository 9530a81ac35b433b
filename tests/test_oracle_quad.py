"""Pins of the oracle's locally corrected quadrature (Section 4, eqs. nys-lcq,
nys-lcq2): the self-patch Duffy/sinh rule and the principal-value gradient
against closed forms for a flat triangle, and the adaptive near rule against a
uniform-subdivision brute force."""
import numpy as np
import pytest

from oracle.geometry import Geometry
from oracle.quad import self_integrals, near_integrals, far_rule, FOUR_PI
from oracle.refelem import nodes, conical_rule


def flat_geom(k, A, B, C):
    uv = nodes(k)
    X = A + uv[:, 0:1] * (B - A) + uv[:, 1:2] * (C - A)
    Xu = np.tile(B - A, (len(uv), 1))
    Xv = np.tile(C - A, (len(uv), 1))
    return Geometry(X[None], Xu[None], Xv[None], k)


def triangle_potential(x0, V):
    """int_T dA / |y - x0| for x0 in the plane of T (closed form, polar sum over edges)."""
    n = np.cross(V[1] - V[0], V[2] - V[0])
    n /= np.linalg.norm(n)
    tot = 0.0
    for e in range(3):
        a, b = V[e], V[(e + 1) % 3]
        t = (b - a) / np.linalg.norm(b - a)
        # inward edge normal (in plane)
        m = np.cross(n, t)
        h = np.dot(a - x0, m)          # signed distance, >0 when x0 is inside
        la, lb = np.dot(a - x0, t), np.dot(b - x0, t)
        ah = abs(h)
        tot += -np.sign(h) * ah * (np.arcsinh(lb / ah) - np.arcsinh(la / ah)) if ah > 0 else 0.0
    return tot


TRI = np.array([[0.0, 0.0, 0.0], [1.0, 0.2, 0.1], [0.3, 0.9, -0.2]])


@pytest.mark.parametrize("k", [3, 6])
def test_self_flat_potential_closed_form(k):
    g = flat_geom(k, *TRI)
    A = self_integrals(g, np.arange(g.N))
    for a in range(g.N):
        ex = triangle_potential(g.x[a], TRI) / FOUR_PI
        assert abs(A[a, :, 0].sum() - ex) < 1e-11 * abs(ex)


@pytest.mark.parametrize("k", [3, 6])
def test_self_flat_pv_gradient(k):
    """PV gradient = in-plane derivative of the closed-form potential (fourth-
    order central differences); its normal part and S''+D' vanish on a plane."""
    g = flat_geom(k, *TRI)
    A = self_integrals(g, np.arange(g.N))
    n = g.n[0]
    e1 = (TRI[1] - TRI[0]) / np.linalg.norm(TRI[1] - TRI[0])
    e2 = np.cross(n, e1)
    h = 2e-4
    for a in range(g.N):
        grad = A[a, :, 1:4].sum(0)
        for e in (e1, e2):
            f = [triangle_potential(g.x[a] + j * h * e, TRI) for j in (-2, -1, 1, 2)]
            fd = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h) / FOUR_PI
            assert abs(grad @ e - fd) < 3e-9
        assert abs(grad @ n) < 1e-12
        assert abs(A[a, :, 4].sum()) < 1e-12        # S' = n . grad
        assert np.abs(A[a, :, 5]).max() < 1e-10     # S''+D' kernel vanishes on a plane (rounding only)


def _brute_near(g, t, p, level, q=6):
    """Uniform 4^level subdivision of T0 with a q x q conical rule per leaf."""
    ru, rw = conical_rule(q)
    tris = [np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])]
    for _ in range(level):
        nt = []
        for T in tris:
            m01, m12, m20 = (T[0] + T[1]) / 2, (T[1] + T[2]) / 2, (T[2] + T[0]) / 2
            nt += [np.array([T[0], m01, m20]), np.array([m01, T[1], m12]), np.array([m20, m12, T[2]]),
                   np.array([m12, m20, m01])]
        tris = nt
    T = np.array(tris)
    uv = T[:, None, 0, :] + ru[None, :, 0:1] * (T[:, None, 1] - T[:, None, 0]) + ru[None, :, 1:2] * (T[:, None, 2] - T[:, None, 0])
    area2 = np.abs(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]))
    wq = (area2[:, None] * rw[None, :]).reshape(-1)
    uv = uv.reshape(-1, 2)
    L = g.re.interp(uv)
    X = L @ g.Xp[p]
    cr = np.cross(L @ g.Xup[p], L @ g.Xvp[p])
    J = np.linalg.norm(cr, axis=1)
    d = g.x[t] - X
    r = np.linalg.norm(d, axis=1)
    f = wq * J / (FOUR_PI * r)
    grad = -(d * (wq * J / (FOUR_PI * r ** 3))[:, None])
    return L.T @ f, L.T @ grad


def test_near_adaptive_vs_uniform_brute_force():
    import lbinputs as I
    k = 4
    X, Xu, Xv = I.sphere_patches(1, nodes(k))
    g = Geometry(X, Xu, Xv, k)
    nl = g.near_lists(np.arange(0, g.N, 97))
    pairs = [(t, p) for t, l in zip(np.arange(0, g.N, 97), nl) for p in l if p != g.patch_of[t]][:6]
    T = np.array([a for a, _ in pairs])
    Pp = np.array([b for _, b in pairs])
    A = near_integrals(g, T, Pp)
    for j, (t, p) in enumerate(pairs):
        s, gr = _brute_near(g, t, p, 6)
        assert np.abs(A[j, :, 0] - s).max() < 1e-11
        assert np.abs(A[j, :, 1:4] - gr).max() < 1e-9


def test_far_rule_matches_accurate_rule_away_from_patch():
    """B (the oversampled rule) equals A for a patch well outside Near."""
    import lbinputs as I
    k = 4
    X, Xu, Xv = I.sphere_patches(1, nodes(k))
    g = Geometry(X, Xu, Xv, k)
    t = np.array([0])
    d = np.linalg.norm(g.x[0] - g.c, axis=1)
    p = np.array([np.argmin(np.where(d > 3 * g.R, d, np.inf))])
    A = near_integrals(g, t, p)
    B = far_rule(g, t, p)
    assert np.abs(A - B).max() < 1e-12
