"""Pins of the oracle's discrete operators and solver against closed forms.

* unit sphere (Appendix-style eigen-relations of the Section 3 operators):
  S Y_l = Y_l/(2l+1), S' Y_l = -Y_l/(2(2l+1)), PV grad S Y_l =
  grad_G Y_l/(2l+1) - n Y_l/(2(2l+1)), (S''+D') Y_l = Y_l/(2l+1),
  A3 Y_l = -l(l+1)/(2l+1)^2 Y_l (l >= 1), A3 1 = 1 (eq. ie-dis2); errors fall
  under refinement;
* ellipsoid conductor: S[sigma_eq] constant, grad S[sigma_eq] = -sigma_eq n/2;
* Gauss: sum_i w_i S'[sigma]_i = -1/2 sum_j w_j sigma_j;
* GMRES (Section 6) against numpy.linalg.solve, and the A3 spectrum
  clustering at -1/4 (Section 6.2);
* the Laplace-Beltrami solve (Lemma 1) against u = -f/6 for f = x z.
"""
import numpy as np
import pytest
from scipy.integrate import quad

import lbinputs as I
from conftest import rel_l2
from oracle.geometry import Geometry
from oracle.ops import Oracle, gmres
from oracle.refelem import nodes


def sphere(k, nsub, targets=None):
    X, Xu, Xv = I.sphere_patches(nsub, nodes(k))
    g = Geometry(X, Xu, Xv, k)
    if isinstance(targets, int):
        targets = np.arange(0, g.N, max(1, g.N // targets))
    return g, Oracle(g, targets)


def sphere_errors(g, o, l, m):
    t = o.targets
    Y = I.real_sph_harm(l, m, g.x)
    L = o.layer(Y)
    Yt = Y[t]
    gY = I.sh_gradient_on_sphere(l, m, g.x[t]) if l > 0 else 0 * g.x[t]
    grad_ex = gY / (2 * l + 1) - g.n[t] * Yt[:, None] / (2 * (2 * l + 1))
    return (np.abs(L[:, 0] - Yt / (2 * l + 1)).max(),
            np.abs(L[:, 4] + Yt / (2 * (2 * l + 1))).max(),
            np.abs(L[:, 1:4] - grad_ex).max(),
            np.abs(L[:, 5] - Yt / (2 * l + 1)).max())


def test_sphere_eigenrelations_converge():
    k = 4
    g1, o1 = sphere(k, 1, 60)
    g2, o2 = sphere(k, 2, 60)
    for l, m in [(0, 0), (1, 0), (2, 1), (3, -2)]:
        e1 = sphere_errors(g1, o1, l, m)
        e2 = sphere_errors(g2, o2, l, m)
        assert max(e1) < 1e-3, (l, m, e1)
        # S, S', S''+D' converge at ~h^(k+1); the PV gradient more slowly
        for j in (0, 1, 3):
            assert e2[j] < e1[j] / 10, (l, m, j, e1, e2)
        assert e2[2] < e1[2] / 2.5, (l, m, e1, e2)


def test_sphere_A3_eigenvalues(c1_oracle):
    o = c1_oracle
    g = o.g
    # limited by the mean curvature from spectral differentiation (~2e-2 max at this size)
    assert rel_l2(o.A3(np.ones(g.N)), np.ones(g.N), g.w) < 1e-2
    for l, m in [(1, 1), (2, 0), (3, 2)]:
        Y = I.real_sph_harm(l, m, g.x)
        lam = -l * (l + 1) / (2 * l + 1) ** 2
        assert rel_l2(o.A3(Y), lam * Y, g.w) < 6e-3


def test_gauss_identity(c1_oracle):
    o = c1_oracle
    g = o.g
    sig = 1.0 + I.real_sph_harm(2, 1, g.x) + 0.3 * g.x[:, 0] * g.x[:, 1] ** 2
    sp = o.layer(sig)[:, 4]
    assert abs(g.w @ sp + 0.5 * g.w @ sig) < 1e-4 * abs(g.w @ sig)


def test_ellipsoid_conductor():
    a, b, c = 1.0, 1.5, 2.0
    k = 4
    X, Xu, Xv = I.ellipsoid_patches(2, nodes(k), (a, b, c))
    g = Geometry(X, Xu, Xv, k)
    o = Oracle(g, np.arange(0, g.N, 97))
    x = g.x
    sig = 1.0 / (4 * np.pi * a * b * c) / np.sqrt(x[:, 0] ** 2 / a ** 4 + x[:, 1] ** 2 / b ** 4 + x[:, 2] ** 2 / c ** 4)
    phi0 = quad(lambda s: 1.0 / np.sqrt((a * a + s) * (b * b + s) * (c * c + s)), 0, np.inf, epsabs=1e-14, epsrel=1e-13)[0] / (8 * np.pi)
    assert abs(phi0 - 0.0534509843807422) < 1e-13
    L = o.layer(sig)
    t = o.targets
    assert np.abs(L[:, 0] - phi0).max() < 2e-6
    assert np.abs(L[:, 1:4] + 0.5 * sig[t, None] * g.n[t]).max() < 2e-4 * sig.max()


def test_gmres_matches_dense_solve_and_happy_breakdown():
    rng = np.random.default_rng(0)
    n = 60
    A = np.eye(n) * 2 + rng.standard_normal((n, n)) / np.sqrt(n) * 0.5
    b = rng.standard_normal(n)
    x, info = gmres(lambda v: A @ v, b, tol=1e-14, max_iter=n)
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-11
    # an operator with 3 distinct eigenvalues converges in 3 steps
    d = np.repeat([1.0, -0.25, 3.0], 20)
    x, info = gmres(lambda v: d * v, b, tol=1e-13, max_iter=n)
    assert info["iters"] == 3 and np.abs(x - b / d).max() < 1e-12


def test_dense_A3_spectrum_and_solve():
    k = 2
    g, o = sphere(k, 1)
    N = g.N
    K = o.operator_matrices()
    S, Sp, SDD = K[0], K[4], K[5]
    Wm = np.ones((N, 1)) @ (g.w[None, :] / g.w.sum())
    M = -0.25 * np.eye(N) + Sp @ Sp - (SDD + 2 * g.H[:, None] * Sp) @ S + Wm @ S @ S
    e0 = np.zeros(N)
    e0[7] = 1.0
    assert np.abs(M @ e0 - o.A3(e0)).max() < 1e-12     # the matrix is the operator
    ev = np.linalg.eigvals(M)
    # second kind: spectrum clusters at -1/4, one eigenvalue near 1 (constants)
    near = np.abs(ev + 0.25) < 0.06
    assert near.mean() > 0.9
    assert np.abs(ev - 1.0).min() < 0.05
    f = g.x[:, 0] * g.x[:, 2]
    f = f - o.W(f)
    x, info = gmres(o.A3, f, tol=1e-13, max_iter=100)
    assert np.abs(x - np.linalg.solve(M, f)).max() < 1e-9 * np.abs(x).max()


def test_solve_sphere_closed_form(c1_oracle):
    o = c1_oracle
    g = o.g
    f = g.x[:, 0] * g.x[:, 2]                 # proportional to a real Y_2^1
    u, info = o.solve(f, tol=1e-12)
    assert info["iters"] <= 8
    assert rel_l2(u, -f / 6.0, g.w) < 1e-3
    assert abs(g.w @ u) < 1e-10              # mean-zero solution


def test_table3_iteration_counts_range(c1_oracle):
    rows = np.loadtxt(__file__.replace("test_oracle_ops.py", "golden/paper_table3_a3.txt"))
    lo, hi = rows[:, 2].min(), rows[:, 2].max()
    o = c1_oracle
    g = o.g
    coef = I.random_sh_coeffs(3, seed=11, decay=0.0)
    f = I.sh_series(coef, g.x)
    u, info = o.solve(f, tol=5e-7)
    assert lo - 2 <= info["iters"] <= hi + 2


def test_adjoint_dot_product_identity(c1_oracle):
    """Transposed apply (dense operator matrices, transposed) against the
    forward apply (kernel table times strengths plus corrections): for any
    cotangents g and density sigma, <g, A sigma> = <A^T g, sigma> with A the
    map sigma -> (S, grad S, S' as n . grad S, grad_Gamma S)."""
    o = c1_oracle
    g = o.g
    rng = np.random.default_rng(21)
    sig = rng.standard_normal(g.N)
    gp, gd = rng.standard_normal(g.N), rng.standard_normal(g.N)
    gg, gs = rng.standard_normal((g.N, 3)), rng.standard_normal((g.N, 3))
    L = o.layer(sig)
    pot, grad = L[:, 0], L[:, 1:4]
    dn = (grad * g.n).sum(-1)
    surf = grad - g.n * dn[:, None]
    lhs = gp @ pot + (gg * grad).sum() + gd @ dn + (gs * surf).sum()
    rhs = o.adjoint_gradS(gp, gg, gd, gs) @ sig
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + np.abs(sig).sum())
    # each cotangent alone
    for kw in ({"gpot": gp}, {"ggrad": gg}, {"gdSdn": gd}, {"gsurf": gs}):
        r = o.adjoint_gradS(**kw) @ sig
        l = {"gpot": gp @ pot, "ggrad": (gg * grad).sum(), "gdSdn": gd @ dn, "gsurf": (gs * surf).sum()}[next(iter(kw))]
        assert abs(l - r) < 1e-12 * (abs(l) + np.abs(sig).sum())


def test_A3_matrix_and_solve_adjoint(c1_oracle):
    """Dense A3 against the layer-by-layer apply of Section 4.3, and the
    transposed solve map against the forward solve by the dot-product
    identity <ubar, u(f)> = <fbar(ubar), f> (u(f) by GMRES, fbar by a dense
    solve with A3^T)."""
    o = c1_oracle
    g = o.g
    rng = np.random.default_rng(23)
    A = o.A3_matrix()
    for _ in range(2):
        v = rng.standard_normal(g.N)
        assert np.linalg.norm(A @ v - o.A3(v)) < 1e-12 * np.linalg.norm(A @ v)
    f = rng.standard_normal(g.N)
    ub = rng.standard_normal(g.N)
    u, info = o.solve(f, tol=1e-14)
    fb = o.solve_adjoint(ub)
    lhs, rhs = ub @ u, fb @ f
    assert abs(lhs - rhs) < 1e-10 * np.linalg.norm(ub) * np.linalg.norm(u) * 10
    # the transposed projection removes exactly the weighted constant direction
    assert abs(np.ones(g.N) @ fb) < 1e-9 * np.abs(fb).sum()


def test_position_vjp_S(c1_oracle):
    """Kernel-position derivative of <gbar, S sigma> (nodes and far-rule points
    moving with X, weights, oversampled density and corrections fixed):
    central differences of the far sum written out here, invariance of that
    sum under translations (sum_j X_bar_j = 0; the interpolation reproduces
    constants, so s = P X translates with X) and rotations
    (sum_j x_j x X_bar_j = 0), and the per-patch evaluation."""
    o = c1_oracle
    g = o.g
    rng = np.random.default_rng(31)
    sig = rng.standard_normal((2, g.N))
    gb = rng.standard_normal((2, g.N))
    Xb = o.position_vjp_S(sig, gb)
    assert Xb.shape == (g.N, 3)
    scale = np.abs(Xb).sum()
    assert np.abs(Xb.sum(0)).max() < 1e-11 * scale
    assert np.abs(np.cross(g.x, Xb).sum(0)).max() < 1e-11 * scale
    c = np.stack([o.oversample(t) for t in sig])

    def far(Xp):
        x = Xp.reshape(-1, 3)
        s = np.einsum('mb,pbc->pmc', g.re.P, Xp).reshape(-1, 3)
        r = np.linalg.norm(x[:, None, :] - s[None, :, :], axis=-1)
        return float((gb * (c @ (1.0 / (4.0 * np.pi * r)).T)).sum())
    for sel in (None, 7):
        dX = rng.standard_normal(g.Xp.shape)
        if sel is not None:  # one patch moving alone
            keep = np.zeros(g.NP, bool)
            keep[sel] = True
            dX[~keep] = 0.0
        h = 1e-6
        fd = (far(g.Xp + h * dX) - far(g.Xp - h * dX)) / (2 * h)
        an = float((Xb * dX.reshape(-1, 3)).sum())
        assert abs(fd - an) < 1e-6 * abs(an), (fd, an)
    sub = o.position_vjp_S(sig, gb, patches=[3, 17])
    rows = np.concatenate([np.arange(3 * g.n_p, 4 * g.n_p), np.arange(17 * g.n_p, 18 * g.n_p)])
    assert np.allclose(sub, Xb[rows], rtol=0, atol=1e-13 * np.abs(Xb).max())


def test_sphere_A1_eigenvalues(c1_oracle):
    """A1 = S (Delta + W) S (Section 4.1) on the unit sphere: S Y_l = Y_l /
    (2l+1) and Delta Y_l = -l(l+1) Y_l give A1 Y_l = -l(l+1)/(2l+1)^2 Y_l,
    the eigenvalue of A3 as well; S[1] = 1 and W[1] = 1 give A1[1] = 1.  The
    dense assembly equals the apply."""
    o = c1_oracle
    g = o.g
    assert np.abs(o.A1(np.ones(g.N)) - 1.0).max() < 1e-3
    for l, m in [(1, 0), (2, 1), (3, -2)]:
        Y = I.real_sph_harm(l, m, g.x)
        lam = -l * (l + 1) / (2 * l + 1) ** 2
        assert rel_l2(o.A1(Y), lam * Y, g.w) < 3e-3
    tau = np.cos(2 * g.x[:, 0]) + g.x[:, 1] * g.x[:, 2]
    assert rel_l2(o.A1_matrix() @ tau, o.A1(tau)) < 1e-13


def test_numerical_second_kindness(c1_oracle):
    """Section 5 (numerical second-kindness): on the sphere with order-4
    patches, the smallest singular value of A1 (no explicit identity term)
    falls under refinement while that of A3 stays put, and GMRES on A1 needs
    many more iterations, reaching the cap at the finer mesh, while A3
    converges in a handful (data: random degree <= 4 harmonics, coefficients
    U(-0.5, 0.5))."""
    from oracle.ops import gmres
    res = []
    for nsub in (0, 1):
        g, o = sphere(4, 0) if nsub == 0 else (c1_oracle.g, c1_oracle)
        A1, A3 = o.A1_matrix(), o.A3_matrix()
        s1 = np.linalg.svd(A1, compute_uv=False)
        s3 = np.linalg.svd(A3, compute_uv=False)
        rng = np.random.default_rng(3)
        f = sum(rng.uniform(-0.5, 0.5) * I.real_sph_harm(l, m, g.x) for l in range(1, 5) for m in range(-l, l + 1))
        f = f - o.W(f)
        _, i1 = gmres(lambda v: A1 @ v, o._M[0] @ f, tol=1e-14, max_iter=100)
        _, i3 = gmres(lambda v: A3 @ v, f, tol=1e-14, max_iter=100)
        res.append((s1[-1], s3[-1], i1["iters"], i3["iters"]))
    (a0, b0, n10, n30), (a1, b1, n11, n31) = res
    assert a1 < a0 / 2 and abs(b1 - b0) < 0.05 * b0
    assert a1 < 1e-2 * b1
    assert n30 <= 12 and n31 <= 12 and n10 > 3 * n30 and n11 == 100
