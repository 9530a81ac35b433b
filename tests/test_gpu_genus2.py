"""The 2g count on a genus-2 surface (Section 5: the harmonic vector fields
of a closed surface of genus g form a 2g-dimensional space).

The surface is the smoothed union of two overlapping solid tori with eight
seeded normal bumps (lbinputs.genus2: marching tetrahedra, mesh improvement,
charts projected onto the implicit surface), 6,686 order-6 patches,
N = 187,208.  The Hodge
split of 2g + 2 = 6 random tangential fields (tensor-Legendre components of
degree ceil((2g)^(1/3)) + 3 = 5 on x / 2L, the paper's recipe) by lb_hodge
(two batched FP32 + refinement Laplace-Beltrami solves per field): their
harmonic parts span a space of dimension 4 = 2g (four singular values of
order one, the others at the discretization level), and each harmonic part
is divergence free and co-divergence free to the discretization error.
The gradient of J = 1/2 |u - u_t|^2_w in f by the adjoint solve against
central finite differences (the c5 check in f)."""
import numpy as np
import pytest

import lbinputs as I
from lbinputs import genus2 as G2

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)


def test_genus2_harmonic_count():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_10743_amd as P
    S = G2.FusedTori()
    V, T = G2.mesh(S, 0.16)
    assert G2.euler_characteristic(T) == -2
    uv = P.ref_nodes(6)[0]
    X, Xu, Xv = G2.patches(S, V, T, uv)
    note(f"genus 2: {len(T)} patches, N = {len(T) * uv.shape[0]}")
    s = P.Surface(X, Xu, Xv, 6)
    w, nrm, _ = s.geometry()
    x = X.reshape(-1, 3)
    fields = []
    for k in range(6):
        Vf = I.legendre_field(x, seed=80 + k, deg=5, L=2.6)
        fields.append(Vf - nrm * (nrm * Vf).sum(1, keepdims=True))
    F = torch.tensor(np.stack(fields), device="cuda")
    note("genus 2: Hodge split of 6 fields, FP32 + refinement")
    _, _, H, info, code = s.hodge(F, tol=1e-10, mode=P.LB_SOLVE_FP32_REFINE)
    note(f"genus 2: status {code}, iterations {[i['iters'] for i in info]}")
    assert code == 0
    sw = np.sqrt(w)[:, None]
    wn = lambda v: float(np.sqrt((w[:, None] * np.asarray(v).reshape(len(w), -1) ** 2).sum()))
    Hn = H.cpu().numpy()
    for k in range(6):
        dH = s.surface_div(H[k].contiguous()).cpu().numpy()
        dnH = s.surface_div(H[k].contiguous(), cross_n=True).cpu().numpy()
        note(f"genus 2 field {k}: |H|/|F| {wn(Hn[k]) / wn(fields[k]):.3f}, |div H| {wn(dH):.1e}, "
             f"|div n x H| {wn(dnH):.1e} (|F| {wn(fields[k]):.2f})")
        assert wn(dH) < 1e-3 * wn(fields[k]) and wn(dnH) < 1e-3 * wn(fields[k])
    sv = np.linalg.svd(np.stack([(sw * Hn[k]).ravel() for k in range(6)], 1), compute_uv=False)
    note(f"genus 2 harmonic parts: singular values {sv}")
    assert sv[3] > 0.05 * sv[0] and sv[4] < 1e-4 * sv[0]
    s.close()


def test_genus2_adjoint_gradient_fd():
    """The gradient of J(f) = 1/2 sum_i w_i (u_i - u_t,i)^2, u = solve(f),
    with respect to f by the adjoint solve (torch.autograd over lb_solve /
    lb_solve_adj, FP32 + refinement) against central finite differences of
    J along 8 seeded random directions (FP64 solves, step 1e-6), to 1e-5
    relative, on a coarse mesh of the genus-2 surface (order 4); u_t is
    random band-limited (seed 6)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_10743_amd as P
    S = G2.FusedTori()
    V, T = G2.mesh(S, 0.26)
    uv = P.ref_nodes(4)[0]
    X, Xu, Xv = G2.patches(S, V, T, uv)
    s = P.Surface(X, Xu, Xv, 4)
    w, _, _ = s.geometry()
    x = X.reshape(-1, 3)
    wt = torch.tensor(w, device="cuda")
    ut = torch.tensor(I.legendre_field(x, seed=6, deg=4, L=2.6)[:, 0], device="cuda")
    f0 = torch.tensor(I.legendre_field(x, seed=7, deg=4, L=2.6)[:, 1], device="cuda")

    def J(f, mode):
        u = P.solve(s, f, tol=1e-12, mode=mode)
        return 0.5 * (wt * (u - ut) ** 2).sum()

    f = f0.clone().requires_grad_(True)
    J(f, P.LB_SOLVE_FP32_REFINE).backward()
    g = f.grad.detach()
    rng = np.random.default_rng(8)
    worst = 0.0
    for _ in range(8):
        d = torch.tensor(rng.standard_normal(s.N), device="cuda")
        h = 1e-6
        with torch.no_grad():
            fd = (J(f0 + h * d, P.LB_SOLVE_FP64) - J(f0 - h * d, P.LB_SOLVE_FP64)) / (2 * h)
        ad = float((g * d).sum())
        worst = max(worst, abs(ad - float(fd)) / abs(float(fd)))
    note(f"genus 2 adjoint gradient (N = {s.N}): worst relative difference to central differences {worst:.2e}")
    assert worst < 1e-5
    s.close()
