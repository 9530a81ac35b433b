"""Harmonic vector fields on a torus through the HIP solver (genus 1).

Torus R = 2, r = 0.7 on a 15 x 42 grid of cells split in two (1260 order-6
patches, N = 35,280 nodes).  One batched FP32 + FP64-refinement solve takes
16 right-hand sides (every (right-hand side) pair its own GMRES system
sharing each apply): the two Hodge equations of the harmonic-vector-field
section for an exactly known field and for four random fields (tensor
Legendre components of degree ceil(2^(1/3)) + 3 = 5 on x / 2L, L = 2.7),
and six more band-limited data.  Checks:
* F = grad z + n x grad x + c1 e_phi / rho + c2 e_theta / rho returns
  alpha = z - mean, beta = x - mean and H = c1 e_phi / rho + c2 e_theta / rho
  (the torus's harmonic fields, both divergence free);
* the harmonic parts of the random fields lie in that two-dimensional space
  and span it (the 2g count);
* every solution agrees with the plain FP64 solve to 1e-9.
Surface gradients and divergences of node values come from the order-6
interpolant on each patch (oracle.hodge), applied to the library's solves.
"""
import sys

import numpy as np
import pytest

import lbinputs as I

pytestmark = pytest.mark.gpu

R_T, r_T = 2.0, 0.7


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_torus_harmonic_fields_batched_solve():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_10743_amd as P
    from oracle.geometry import Geometry
    from oracle.hodge import surface_divergence, surface_gradient
    from oracle.refelem import nodes
    X, Xu, Xv = I.torus_patches(R_T, r_T, 15, 42, nodes(6))
    g = Geometry(X, Xu, Xv, 6)
    note(f"torus setup N={g.N}")
    s = P.Surface(X, Xu, Xv, 6)
    note(f"torus sizes {s.sizes}")
    W = np.sqrt(g.w)[:, None]
    T = lambda v: v - g.n * (g.n * v).sum(1, keepdims=True)
    e_ph, e_th, rho = I.torus_frame(g.x, R_T, r_T)
    Hx = T(0.7 * e_ph / rho[:, None] - 1.3 * e_th / rho[:, None])
    ez = np.tile([0.0, 0.0, 1.0], (g.N, 1))
    ex = np.tile([1.0, 0.0, 0.0], (g.N, 1))
    fields = [T(ez) + np.cross(g.n, T(ex)) + Hx]
    fields += [T(I.legendre_field(g.x, 60 + k, 5, 2.7)) for k in range(4)]
    rhs = []
    for F in fields:
        rhs.append(surface_divergence(g, F))
        rhs.append(-surface_divergence(g, np.cross(g.n, F)))
    xi = g.x / np.linalg.norm(g.x, axis=1, keepdims=True)
    for k in range(6):
        rhs.append(I.sh_series(I.random_sh_coeffs(6, seed=70 + k, decay=1.0), xi))
    f = torch.tensor(np.stack(rhs), device="cuda")
    note("torus solve: 16 right-hand sides, FP32 + refinement")
    u, info, code = s.solve(f, tol=1e-11, mode=P.LB_SOLVE_FP32_REFINE)
    note(f"torus solve iterations {[i['iters'] for i in info]}")
    assert code == 0
    note("torus solve: 16 right-hand sides, FP64")
    u64, info64, code64 = s.solve(f, tol=1e-11, mode=P.LB_SOLVE_FP64)
    assert code64 == 0
    e = float((u - u64).norm() / u64.norm())
    note(f"torus FP32+refine vs FP64 {e:.2e}")
    assert e < 1e-9
    u = u.cpu().numpy()
    wn = lambda v: float(np.sqrt((g.w[:, None] * np.asarray(v).reshape(g.N, -1) ** 2).sum()))
    mf = lambda q: q - (g.w * q).sum() / g.w.sum()
    Hs = []
    for k, F in enumerate(fields):
        a, b = u[2 * k], u[2 * k + 1]
        H = F - surface_gradient(g, a) - np.cross(g.n, surface_gradient(g, b))
        if k == 0:
            eh, ea, eb = wn(H - Hx) / wn(Hx), wn(a - mf(g.x[:, 2])) / wn(mf(g.x[:, 2])), \
                wn(b - mf(g.x[:, 0])) / wn(mf(g.x[:, 0]))
            note(f"torus exact field: H {eh:.2e} alpha {ea:.2e} beta {eb:.2e}")
            assert eh < 1e-5 and ea < 1e-6 and eb < 1e-6
        else:
            Hs.append((H * W).ravel())
    B = np.stack([(T(e_ph / rho[:, None]) * W).ravel(), (T(e_th / rho[:, None]) * W).ravel()], 1)
    for k, h in enumerate(Hs):
        fn = np.linalg.norm((fields[k + 1] * W).ravel())
        res = np.linalg.norm(h - B @ np.linalg.lstsq(B, h, rcond=None)[0])
        note(f"torus random field {k}: |H|/|F| {np.linalg.norm(h) / fn:.3f}, outside the harmonic space {res / fn:.2e}")
        assert res < 1e-5 * fn
    sv = np.linalg.svd(np.stack(Hs, 1), compute_uv=False)
    note(f"torus harmonic parts: singular values {sv}")
    assert sv[1] > 0.05 * sv[0] and sv[2] < 1e-4 * sv[0]
    s.close()
