"""A2 (Section 4.2, eq. ie-dis1) through the C ABI on the unit sphere
(80 order-4 patches, N = 1200) against the oracle's A2 at every row: FP64
with direct far sums (LB_DIRECT) to 1e-11, through the FMM to 3e-9 (the
truncation of the Hessian of the first pass's expansions, as for A3), FP32
to 1e-5; the eigen-relation A2 Y_l = -l(l+1)/(2l+1)^2 Y_l that A2 shares with
A1 and A3 (S (Delta + W) S on the sphere) to the discretization error; a
batch of densities equals the densities applied one at a time; and the A2
solve of the library's operator (u = S sigma with A2 sigma = S f, by GMRES
in NumPy over the FP64 apply) returns u = -f/6 for f = x z, and lb_solve with
LB_SOLVE_A2 (device GMRES, both modes) returns the same solution."""
import numpy as np
import pytest

import lbinputs as I
from conftest import max_row, rel_l2

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def sphere_ctx(torch_dev):
    import paper_2111_10743_amd as P
    from oracle.refelem import nodes
    X, Xu, Xv = I.sphere_patches(1, nodes(4))
    fmm = P.Surface(X, Xu, Xv, 4, leaf_src=64)
    direct = P.Surface(X, Xu, Xv, 4, direct=True)
    assert fmm.sizes["fmm_levels"] >= 3
    yield fmm, direct, X
    fmm.close()
    direct.close()


def test_A2_sphere_vs_oracle(torch_dev, sphere_ctx, c1_oracle):
    torch = torch_dev
    fmm, direct, X = sphere_ctx
    o = c1_oracle
    g = o.g
    tau = I.sh_series(I.random_sh_coeffs(6, seed=31), g.x) + 0.1 * np.random.default_rng(32).standard_normal(g.N)
    ref = o.A2(tau)
    for name, s, prec, bar in (("direct", direct, 64, 1e-11), ("fmm", fmm, 64, 3e-9), ("direct", direct, 32, 1e-5),
                               ("fmm", fmm, 32, 1e-5)):
        dt = torch.float64 if prec == 64 else torch.float32
        out = s.apply_A2(torch.tensor(tau, dtype=dt, device="cuda")).double().cpu().numpy()
        e, m = rel_l2(out, ref), max_row(out, ref)
        note(f"A2 sphere {name} prec={prec}: {e:.2e} (max row {m:.2e})")
        assert e < bar and m < 10 * bar


def test_A2_eigen_batch_and_solve(torch_dev, sphere_ctx):
    torch = torch_dev
    from oracle.ops import gmres
    fmm, _, X = sphere_ctx
    x = X.reshape(-1, 3)
    w = fmm.geometry()[0]
    Ys = []
    for l, m in [(1, 1), (2, 0), (3, -2)]:
        Y = I.real_sph_harm(l, m, x)
        Ys.append(Y)
        out = fmm.apply_A2(torch.tensor(Y, device="cuda")).cpu().numpy()
        lam = -l * (l + 1) / (2 * l + 1) ** 2
        e = rel_l2(out, lam * Y, w)
        note(f"A2 Y_{l}^{m}: {e:.2e}")
        assert e < 6e-3
    one = fmm.apply_A2(torch.ones(len(x), dtype=torch.float64, device="cuda")).cpu().numpy()
    assert rel_l2(one, np.ones(len(x)), w) < 1e-2
    # a batch equals the single applies (the first pass carries 3 expansions
    # per density, the FP64 traversal at most 2 densities)
    B = torch.tensor(np.stack(Ys + [np.ones(len(x))]), device="cuda")
    ob = fmm.apply_A2(B).cpu().numpy()
    for r in range(B.shape[0]):
        single = fmm.apply_A2(B[r].contiguous()).cpu().numpy()
        assert np.abs(ob[r] - single).max() <= 1e-14 * np.abs(single).max()
    f = x[:, 0] * x[:, 2]
    fz = f - (w * f).sum() / w.sum()
    Sf = fmm.apply_S(torch.tensor(fz, device="cuda")).cpu().numpy()
    A = lambda v: fmm.apply_A2(torch.tensor(v, device="cuda")).cpu().numpy()
    sig, info = gmres(A, Sf, tol=1e-12, max_iter=100)
    u = fmm.apply_S(torch.tensor(sig, device="cuda")).cpu().numpy()
    note(f"A2 solve: {info['iters']} iterations, u vs -f/6 {rel_l2(u, -f / 6.0, w):.2e}")
    assert info["iters"] <= 12 and rel_l2(u, -f / 6.0, w) < 1e-3
    # the library's A2 solve (LB_SOLVE_A2) in both modes: the same solution
    import paper_2111_10743_amd as P
    for mode in (P.LB_SOLVE_FP64, P.LB_SOLVE_FP32_REFINE):
        ul, info_l, code = fmm.solve(torch.tensor(f, device="cuda"), tol=1e-12, mode=mode | P.LB_SOLVE_A2)
        ul = ul.cpu().numpy()
        note(f"lb_solve A2 mode {mode}: {info_l[0]['iters']} iterations, against the NumPy GMRES {rel_l2(ul, u, w):.2e}")
        assert code == 0 and rel_l2(ul, u, w) < 1e-9
