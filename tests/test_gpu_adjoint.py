"""GPU parity of the adjoint (transposed) applies through the C ABI.

Cases: the c1 sphere (80 order-4 patches, N = 1200), direct far sums and
FMM, FP64 and FP32, against the oracle's transpose of its dense operator;
a mid-size sphere through the FMM on the dot-product identity
<g, A sigma> = <A^T g, sigma> with the library's own forward apply (FP64:
the two FMMs differ at their truncation level, ~1e-10); the torch.autograd
wrappers against the adjoint and against central differences.
"""
import sys

import numpy as np
import pytest

import lbinputs as I
from conftest import rel_l2

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def cotangents(N, seed, nd=None):
    rng = np.random.default_rng(seed)
    sh = (N,) if nd is None else (nd, N)
    return (rng.standard_normal(sh), rng.standard_normal(sh + (3,)), rng.standard_normal(sh),
            rng.standard_normal(sh + (3,)))


@pytest.mark.parametrize("direct", [True, False])
@pytest.mark.parametrize("prec", [64, 32])
def test_c1_adjoint_vs_oracle(torch_dev, c1_oracle, direct, prec):
    torch = torch_dev
    import paper_2111_10743_amd as P
    o = c1_oracle
    g = o.g
    note(f"c1 adjoint direct={direct} prec={prec} setup")
    s = P.Surface(g.Xp, g.Xup, g.Xvp, 4, direct=direct)
    dt = torch.float64 if prec == 64 else torch.float32
    gp, gg, gd, gs = cotangents(g.N, 31, nd=2)
    T = [torch.tensor(a, dtype=dt, device="cuda") for a in (gp, gg, gd, gs)]
    note(f"c1 adjoint direct={direct} prec={prec} launch")
    sb = s.apply_gradS_adj(*T).double().cpu().numpy()
    sS = s.apply_S_adj(T[0]).double().cpu().numpy()
    torch.cuda.synchronize()
    tol = 1e-9 if prec == 64 else 2e-6
    for d in range(2):
        ref = o.adjoint_gradS(gp[d], gg[d], gd[d], gs[d])
        refS = o.adjoint_gradS(gpot=gp[d])
        e, eS = rel_l2(sb[d], ref), rel_l2(sS[d], refS)
        note(f"density {d}: full adjoint {e:.2e}  S^T {eS:.2e}")
        assert e < tol and eS < tol
    s.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_fmm_adjoint_dot_product(torch_dev, prec):
    """Transposed tree with several levels: <g, A sigma> against <A^T g, sigma>."""
    torch = torch_dev
    import paper_2111_10743_amd as P
    from oracle.refelem import nodes
    X, Xu, Xv = I.sphere_patches(3, nodes(4))
    note(f"fmm adjoint prec={prec} setup")
    s = P.Surface(X, Xu, Xv, 4)
    note(f"fmm adjoint sizes {s.sizes}")
    N = s.N
    dt = torch.float64 if prec == 64 else torch.float32
    rng = np.random.default_rng(41)
    sig = torch.tensor(rng.standard_normal((3, N)), dtype=dt, device="cuda")
    gp, gg, gd, gs = [torch.tensor(a, dtype=dt, device="cuda") for a in cotangents(N, 42, nd=3)]
    out = s.apply_gradS(sig)
    sb = s.apply_gradS_adj(gp, gg, gd, gs)
    torch.cuda.synchronize()
    for d in range(3):
        lhs = float((gp[d].double() * out["pot"][d].double()).sum() + (gg[d].double() * out["grad"][d].double()).sum()
                    + (gd[d].double() * out["dSdn"][d].double()).sum()
                    + (gs[d].double() * out["surf_grad"][d].double()).sum())
        rhs = float((sb[d].double() * sig[d].double()).sum())
        scale = float(sb[d].double().norm() * sig[d].double().norm())
        note(f"density {d}: <g,A s> {lhs:.12e} <A^T g,s> {rhs:.12e} rel {abs(lhs - rhs) / scale:.2e}")
        assert abs(lhs - rhs) < (1e-10 if prec == 64 else 2e-6) * scale
    s.close()


def test_autograd_apply(torch_dev, c1_oracle):
    """torch.autograd through apply_S / apply_gradS: gradients equal the
    adjoint applies and central differences of the (linear) maps."""
    torch = torch_dev
    import paper_2111_10743_amd as P
    g = c1_oracle.g
    note("autograd setup")
    s = P.Surface(g.Xp, g.Xup, g.Xvp, 4)
    rng = np.random.default_rng(51)
    sig = torch.tensor(rng.standard_normal(g.N), dtype=torch.float64, device="cuda", requires_grad=True)
    tgt = torch.tensor(rng.standard_normal(g.N), dtype=torch.float64, device="cuda")
    w = torch.tensor(g.w, dtype=torch.float64, device="cuda")
    note("autograd apply_S")
    u = P.apply_S(s, sig)
    J = 0.5 * (w * (u - tgt) ** 2).sum()
    J.backward()
    grad = sig.grad.clone()
    ref = s.apply_S_adj((w * (u.detach() - tgt)).contiguous())
    assert float((grad - ref).norm() / ref.norm()) < 1e-14
    v = torch.tensor(rng.standard_normal(g.N), dtype=torch.float64, device="cuda")
    h = 1e-3  # J is quadratic in sigma: central differences are exact up to rounding
    with torch.no_grad():
        Jp = 0.5 * (w * (s.apply_S(sig + h * v) - tgt) ** 2).sum()
        Jm = 0.5 * (w * (s.apply_S(sig - h * v) - tgt) ** 2).sum()
    fd = float((Jp - Jm) / (2 * h))
    an = float((grad * v).sum())
    note(f"apply_S: directional derivative fd {fd:.12e} adjoint {an:.12e}")
    assert abs(fd - an) < 1e-9 * abs(an)
    note("autograd apply_gradS")
    sig.grad = None
    pot, gr, dn, sg = P.apply_gradS(s, sig)
    J2 = (pot * tgt).sum() + (gr ** 2).sum() + (dn * w).sum() + (sg[:, 0] * tgt).sum()
    J2.backward()
    with torch.no_grad():
        o = s.apply_gradS(sig + h * v)
        Jp = (o["pot"] * tgt).sum() + (o["grad"] ** 2).sum() + (o["dSdn"] * w).sum() + (o["surf_grad"][:, 0] * tgt).sum()
        o = s.apply_gradS(sig - h * v)
        Jm = (o["pot"] * tgt).sum() + (o["grad"] ** 2).sum() + (o["dSdn"] * w).sum() + (o["surf_grad"][:, 0] * tgt).sum()
    fd = float((Jp - Jm) / (2 * h))
    an = float((sig.grad * v).sum())
    note(f"apply_gradS: directional derivative fd {fd:.12e} adjoint {an:.12e}")
    assert abs(fd - an) < 1e-8 * abs(an)
    s.close()


@pytest.mark.parametrize("direct", [True, False])
@pytest.mark.parametrize("prec", [64, 32])
def test_c1_A3_adj_vs_oracle(torch_dev, c1_oracle, direct, prec):
    torch = torch_dev
    import paper_2111_10743_amd as P
    o = c1_oracle
    g = o.g
    note(f"c1 A3^T direct={direct} prec={prec}")
    s = P.Surface(g.Xp, g.Xup, g.Xvp, 4, direct=direct)
    dt = torch.float64 if prec == 64 else torch.float32
    rng = np.random.default_rng(61)
    v = np.stack([rng.standard_normal(g.N), I.real_sph_harm(2, 1, g.x) + 0.2])
    out = s.apply_A3_adj(torch.tensor(v, dtype=dt, device="cuda")).double().cpu().numpy()
    AT = o.A3_matrix().T
    for d in range(2):
        e = rel_l2(out[d], AT @ v[d])
        note(f"density {d}: A3^T error {e:.2e}")
        assert e < (1e-9 if prec == 64 else 1e-5)
    s.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_fmm_A3_adj_dot_product(torch_dev, prec):
    torch = torch_dev
    import paper_2111_10743_amd as P
    from oracle.refelem import nodes
    X, Xu, Xv = I.ellipsoid_patches(2, nodes(6), (1.0, 1.5, 2.0))
    note(f"fmm A3^T prec={prec} setup")
    s = P.Surface(X, Xu, Xv, 6)
    dt = torch.float64 if prec == 64 else torch.float32
    rng = np.random.default_rng(62)
    x = torch.tensor(rng.standard_normal((3, s.N)), dtype=dt, device="cuda")
    y = torch.tensor(rng.standard_normal((3, s.N)), dtype=dt, device="cuda")
    Ax = s.apply_A3(x).double()
    ATy = s.apply_A3_adj(y).double()
    for d in range(3):
        lhs = float((y[d].double() * Ax[d]).sum())
        rhs = float((ATy[d] * x[d].double()).sum())
        scale = float(y[d].double().norm() * Ax[d].norm())
        note(f"density {d}: <y, A3 x> {lhs:.12e} <A3^T y, x> {rhs:.12e} rel {abs(lhs - rhs) / scale:.2e}")
        assert abs(lhs - rhs) < (1e-9 if prec == 64 else 1e-5) * scale
    s.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_c1_solve_adj_vs_oracle(torch_dev, c1_oracle, mode):
    torch = torch_dev
    import paper_2111_10743_amd as P
    o = c1_oracle
    g = o.g
    note(f"c1 adjoint solve mode={mode}")
    s = P.Surface(g.Xp, g.Xup, g.Xvp, 4)
    rng = np.random.default_rng(63)
    ub = np.stack([rng.standard_normal(g.N), g.w * I.real_sph_harm(3, 2, g.x)])
    fb, info, code = s.solve_adj(torch.tensor(ub, dtype=torch.float64, device="cuda"), tol=1e-12, mode=mode)
    note(f"info {info}")
    assert code == 0
    fb = fb.cpu().numpy()
    for d in range(2):
        e = rel_l2(fb[d], o.solve_adjoint(ub[d]))
        note(f"rhs {d}: adjoint solve error vs oracle {e:.2e}")
        assert e < 1e-9
    s.close()


def test_autograd_solve_fd(torch_dev):
    """dJ/df through lb_solve_adj against central differences of the solve
    (J = 1/2 sum w (u - u_t)^2 is quadratic in f), FMM path, FP32+refine."""
    torch = torch_dev
    import paper_2111_10743_amd as P
    from oracle.refelem import nodes
    X, Xu, Xv = I.ellipsoid_patches(2, nodes(6), (1.0, 1.5, 2.0))
    note("autograd solve setup")
    s = P.Surface(X, Xu, Xv, 6)
    w = torch.tensor(s.geometry()[0], device="cuda")
    rng = np.random.default_rng(64)
    xi = I.sphere_preimage(X.reshape(-1, 3), (1.0, 1.5, 2.0))
    f = torch.tensor(I.sh_series(I.random_sh_coeffs(4, seed=2, decay=2.0), xi), device="cuda", requires_grad=True)
    ut = torch.tensor(rng.standard_normal(s.N) * 0.01, device="cuda")
    mode = P.LB_SOLVE_FP32_REFINE
    u = P.solve(s, f, 1e-12, mode)
    J = 0.5 * (w * (u - ut) ** 2).sum()
    J.backward()
    v = torch.tensor(I.sh_series(I.random_sh_coeffs(4, seed=3, decay=2.0), xi), device="cuda")
    h = 1e-2
    with torch.no_grad():
        up, _, _ = s.solve(f + h * v, tol=1e-12, mode=mode)
        um, _, _ = s.solve(f - h * v, tol=1e-12, mode=mode)
        fd = float((0.5 * (w * (up - ut) ** 2).sum() - 0.5 * (w * (um - ut) ** 2).sum()) / (2 * h))
    an = float((f.grad * v).sum())
    note(f"directional derivative fd {fd:.12e} adjoint {an:.12e} rel {abs(fd - an) / abs(an):.2e}")
    assert abs(fd - an) < 1e-6 * abs(an)
    s.close()


@pytest.mark.parametrize("direct", [True, False])
@pytest.mark.parametrize("prec", [64, 32])
def test_c1_position_vjp_vs_oracle(torch_dev, c1_oracle, direct, prec):
    """Kernel-position derivative of S (lb_apply_S_adj_X) against the
    oracle's, two densities summed.  The derivative moves the far rule's
    points with the nodes, unmasked, so it is that of each precision's own
    rule: the FP32 path's (max(k+2, 6) = 6 points per direction) is compared
    with the oracle on that rule.  FP32 sums every pair without the near
    mask, so terms up to 1/r^2 of the closest node/point pairs enter the
    FP32 sums (the coarser FP32 rule has pairs closer than the FP64 one):
    1e-4 relative L2 (measured 2e-5)."""
    torch = torch_dev
    import paper_2111_10743_amd as P
    o = c1_oracle
    g = o.g
    if prec == 32:
        from oracle.geometry import Geometry
        from oracle.ops import Oracle
        o = Oracle(Geometry(g.Xp, g.Xup, g.Xvp, 4, q=6))
        g = o.g
    note(f"c1 position vjp direct={direct} prec={prec} setup")
    s = P.Surface(g.Xp, g.Xup, g.Xvp, 4, direct=direct)
    dt = torch.float64 if prec == 64 else torch.float32
    rng = np.random.default_rng(61)
    sig, gb = rng.standard_normal((2, g.N)), rng.standard_normal((2, g.N))
    note(f"c1 position vjp direct={direct} prec={prec} launch")
    xb = s.apply_S_adj_X(torch.tensor(sig, dtype=dt, device="cuda"), torch.tensor(gb, dtype=dt, device="cuda"))
    torch.cuda.synchronize()
    ref = o.position_vjp_S(sig, gb)
    e = rel_l2(xb.double().cpu().numpy(), ref)
    note(f"c1 position vjp error {e:.2e}")
    assert e < (1e-9 if prec == 64 else 1e-4)
    s.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_fmm_position_vjp_sampled(torch_dev, prec):
    """Several FMM levels (sphere, 1280 order-4 patches, N = 19,200): the
    position derivative on the nodes of 24 sampled patches against the
    oracle's, which sums over every node and oversampled point of the
    precision's far rule (FP32: 6 x 6 points per patch; unmasked FP32 sums,
    1e-4 relative L2, measured 6e-5)."""
    torch = torch_dev
    import paper_2111_10743_amd as P
    from oracle.geometry import Geometry
    from oracle.ops import Oracle
    from oracle.refelem import nodes
    X, Xu, Xv = I.sphere_patches(3, nodes(4))
    g = Geometry(X, Xu, Xv, 4, q=None if prec == 64 else 6)
    note(f"fmm position vjp prec={prec} setup")
    s = P.Surface(X, Xu, Xv, 4)
    note(f"fmm position vjp sizes {s.sizes}")
    dt = torch.float64 if prec == 64 else torch.float32
    rng = np.random.default_rng(62)
    xi = g.x / np.linalg.norm(g.x, axis=1, keepdims=True)
    sig = I.real_sph_harm(3, 2, xi) + 0.2 * rng.standard_normal(g.N)
    gb = rng.standard_normal(g.N)
    note(f"fmm position vjp prec={prec} launch")
    xb = s.apply_S_adj_X(torch.tensor(sig, dtype=dt, device="cuda"), torch.tensor(gb, dtype=dt, device="cuda"))
    torch.cuda.synchronize()
    pts = np.arange(0, g.NP, g.NP // 24)[:24]
    o = Oracle(g, np.arange(1))  # rows unused: the position derivative needs no corrections
    ref = o.position_vjp_S(sig, gb, patches=pts)
    rows = (pts[:, None] * g.n_p + np.arange(g.n_p)[None, :]).reshape(-1)
    e = rel_l2(xb.double().cpu().numpy()[rows], ref)
    note(f"fmm position vjp prec={prec} error {e:.2e}")
    assert e < (1e-9 if prec == 64 else 1e-4)
    s.close()


def test_autograd_positions(torch_dev):
    """torch.autograd through apply_S with the node positions as an input:
    the gradients are the library's density and position derivatives."""
    torch = torch_dev
    import paper_2111_10743_amd as P
    X, Xu, Xv = I.sphere_patches(1, __import__("oracle.refelem", fromlist=["nodes"]).nodes(4))
    note("autograd positions setup")
    s = P.Surface(X, Xu, Xv, 4)
    rng = np.random.default_rng(63)
    sig = torch.tensor(rng.standard_normal(s.N), dtype=torch.float64, device="cuda", requires_grad=True)
    Xt = torch.tensor(X.reshape(-1, 3), dtype=torch.float64, device="cuda", requires_grad=True)
    tgt = torch.tensor(rng.standard_normal(s.N), dtype=torch.float64, device="cuda")
    u = P.apply_S(s, sig, Xt)
    J = 0.5 * ((u - tgt) ** 2).sum()
    J.backward()
    gbar = (u.detach() - tgt).contiguous()
    xb = s.apply_S_adj_X(sig.detach().contiguous(), gbar)
    sb = s.apply_S_adj(gbar)
    assert torch.equal(Xt.grad, xb) and torch.equal(sig.grad, sb)
    with pytest.raises(ValueError):
        P.apply_S(s, sig, Xt[:10])
    s.close()
