"""Pins of the oracle's surface calculus and Hodge decomposition.

* Section 2 operators on the unit sphere: grad_Gamma Y_lm against the
  tangential gradient of the degree-0 extension, and
  div_Gamma grad_Gamma Y_lm = -l(l+1) Y_lm, errors falling under refinement;
  on the torus the divergence theorem (sum_i w_i div F_i = 0) and
  div(n x grad f) = 0.
* Harmonic vector fields (genus 1): on the torus R = 2, r = 0.7 the
  harmonic fields are e_phi / rho and n x e_phi / rho = e_theta / rho
  (rho = R + r cos theta; both are divergence free), so for
  F = grad z + n x grad x + c1 e_phi / rho + c2 e_theta / rho the
  decomposition must return alpha = z - mean, beta = x - mean and exactly
  that harmonic part; the harmonic parts of random fields (the paper's
  tensor-Legendre recipe) must lie in that two-dimensional space: the
  2g-dimensional count with g = 1.  On the sphere (g = 0) they vanish.
"""
import numpy as np
import pytest

import lbinputs as I
from oracle.geometry import Geometry
from oracle.hodge import hodge, surface_divergence, surface_gradient
from oracle.ops import Oracle
from oracle.refelem import nodes

R_T, r_T = 2.0, 0.7


def wnorm(g, v):
    return float(np.sqrt((g.w[:, None] * np.asarray(v).reshape(g.N, -1) ** 2).sum()))


def mean_free(g, f):
    return f - (g.w * f).sum() / g.w.sum()


def tangential(g, v):
    return v - g.n * (g.n * v).sum(1, keepdims=True)


def test_surface_calculus_sphere():
    errs = []
    for nsub in (1, 2):
        X, Xu, Xv = I.sphere_patches(nsub, nodes(6))
        g = Geometry(X, Xu, Xv, 6)
        Y = I.real_sph_harm(3, 1, g.x)
        gY = surface_gradient(g, Y)
        gex = I.sh_gradient_on_sphere(3, 1, g.x)
        lap = surface_divergence(g, gY)
        errs.append((wnorm(g, gY - gex) / wnorm(g, gex), wnorm(g, lap + 12 * Y) / wnorm(g, 12 * Y)))
    assert errs[1][0] < 1e-4 and errs[1][1] < 1e-3
    assert errs[1][0] < errs[0][0] / 8 and errs[1][1] < errs[0][1] / 4


def test_divergence_identities_torus():
    X, Xu, Xv = I.torus_patches(R_T, r_T, 12, 24, nodes(5))
    g = Geometry(X, Xu, Xv, 5)
    F = tangential(g, I.legendre_field(g.x, 5, 2, 2.7))
    d = surface_divergence(g, F)
    assert abs((g.w * d).sum()) < 1e-6 * (g.w * np.abs(d)).sum()
    f = np.sin(g.x[:, 0]) * g.x[:, 2] + g.x[:, 1] ** 2
    c = surface_divergence(g, np.cross(g.n, surface_gradient(g, f)))
    lap = surface_divergence(g, surface_gradient(g, f))
    assert wnorm(g, c) < 1e-3 * wnorm(g, lap)


@pytest.fixture(scope="module")
def torus_oracle():
    """Torus, 6 x 12 cells split in two (144 order-3 patches, N = 1440)."""
    X, Xu, Xv = I.torus_patches(R_T, r_T, 6, 12, nodes(3))
    g = Geometry(X, Xu, Xv, 3)
    return Oracle(g, dense_limit=4e7)


def test_hodge_torus_exact(torus_oracle):
    o = torus_oracle
    g = o.g
    e_ph, e_th, rho = I.torus_frame(g.x, R_T, r_T)
    Hx = tangential(g, 0.7 * e_ph / rho[:, None] - 1.3 * e_th / rho[:, None])
    ez = np.tile([0.0, 0.0, 1.0], (g.N, 1))
    ex = np.tile([1.0, 0.0, 0.0], (g.N, 1))
    F = tangential(g, ez) + np.cross(g.n, tangential(g, ex)) + Hx
    a, b, H = hodge(g, lambda f: o.solve(f, tol=1e-11)[0], F)
    assert wnorm(g, H - Hx) < 3e-2 * wnorm(g, Hx)
    za, xb = mean_free(g, g.x[:, 2]), mean_free(g, g.x[:, 0])
    assert wnorm(g, a - za) < 1e-2 * wnorm(g, za)
    assert wnorm(g, b - xb) < 2e-2 * wnorm(g, xb)


def test_harmonic_space_dimension_torus(torus_oracle):
    o = torus_oracle
    g = o.g
    e_ph, e_th, rho = I.torus_frame(g.x, R_T, r_T)
    basis = [tangential(g, e_ph / rho[:, None]), tangential(g, e_th / rho[:, None])]
    W = np.sqrt(g.w)[:, None]
    B = np.stack([(b * W).ravel() for b in basis], 1)
    Hs = []
    for s in range(4):
        F = tangential(g, I.legendre_field(g.x, 40 + s, 2, 2.7))
        _, _, H = hodge(g, lambda f: o.solve(f, tol=1e-11)[0], F)
        h = (H * W).ravel()
        res = h - B @ np.linalg.lstsq(B, h, rcond=None)[0]
        # outside the exact harmonic space only the discretization error of
        # the chain (~1% of |F| at this resolution); H itself is 5-25% of |F|
        fn = np.linalg.norm((F * W).ravel())
        assert np.linalg.norm(res) < 2e-2 * fn and np.linalg.norm(h) > 3e-2 * fn
        Hs.append(h)
    # the four harmonic parts span both directions (rank 2 = 2g)
    sv = np.linalg.svd(np.stack(Hs, 1), compute_uv=False)
    assert sv[1] > 0.05 * sv[0]


def test_harmonic_parts_vanish_sphere(c1_oracle):
    o = c1_oracle
    g = o.g
    for s in range(2):
        F = tangential(g, I.legendre_field(g.x, 50 + s, 2, 1.1))
        _, _, H = hodge(g, lambda f: o.solve(f, tol=1e-11)[0], F)
        assert wnorm(g, H) < 1e-2 * wnorm(g, F)


def test_twisted_torus_charts():
    """The twisted torus of the harmonic-fields section: chart derivatives
    against central differences, a closed surface (sum of w n = 0), normals
    outward (enclosed volume (1/3) sum w x.n > 0), and the current element
    at (0.2, 0.2, 0.2) outside the solid (in the hole)."""
    u = np.array([0.3, 1.7, 4.0])
    v = np.array([2.1, 5.0, 0.4])
    h = 1e-6
    X, Xu, Xv = I.twisted_torus_point(u, v)
    fu = (I.twisted_torus_point(u + h, v)[0] - I.twisted_torus_point(u - h, v)[0]) / (2 * h)
    fv = (I.twisted_torus_point(u, v + h)[0] - I.twisted_torus_point(u, v - h)[0]) / (2 * h)
    assert np.abs(fu - Xu).max() < 1e-8 and np.abs(fv - Xv).max() < 1e-8
    Xp, Xa, Xb = I.twisted_torus_patches(4, 16, nodes(5))
    g = Geometry(Xp, Xa, Xb, 5)
    # (the quadrature error of this coarse mesh: 1.3e-5 of the area)
    assert np.abs((g.w[:, None] * g.n).sum(0)).max() < 1e-4 * g.w.sum()
    vol = (g.w * (g.x * g.n).sum(1)).sum() / 3
    assert vol > 0
    # solid angle of the surface seen from x0: 0 outside the solid
    d = g.x - 0.2
    omega = (g.w * (d * g.n).sum(1) / np.linalg.norm(d, axis=1) ** 3).sum()
    assert abs(omega) < 1e-3 * 4 * np.pi


def test_current_source_field():
    """V = l x (x - x0)/|x - x0|^3 (the field of a current element): divergence
    free away from x0 (div(l x r/r^3) = -l . curl(r/r^3) = 0; central
    differences), and orthogonal to l and to x - x0."""
    rng = np.random.default_rng(5)
    x = rng.uniform(-3, 3, (20, 3)) + np.array([4.0, 0.0, 0.0])
    h = 1e-5
    V = I.current_source_field(x)
    J = np.zeros((20, 3, 3))   # J[:, i, j] = d V_i / d x_j
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        J[:, :, j] = (I.current_source_field(x + e) - I.current_source_field(x - e)) / (2 * h)
    scale = np.abs(J).max()
    assert np.abs(np.trace(J, axis1=1, axis2=2)).max() < 1e-7 * scale
    assert np.abs(V @ np.array([0.0, 1.0, 1.0])).max() < 1e-14
    assert np.abs((V * (x - 0.2)).sum(1)).max() < 1e-14
