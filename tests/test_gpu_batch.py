"""Several independent surfaces in one context (lb_setup_batch) against one
context per surface: the forest of octrees, the per-surface W terms and
mean projections and the per-(right-hand side, surface) GMRES systems must
reproduce the separate results.  Cases: three star-shaped surfaces of
different sizes (icosahedral faces split 2, 3 and 4 ways, order 4, seeds
4, 5, 6) -- every apply and its transpose in FP64 and FP32, the solve in
both modes with two right-hand sides, the adjoint solve -- and the batch
against the oracle on the smallest surface.
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


@pytest.fixture(scope="module")
def stars():
    from oracle.refelem import nodes
    uv = nodes(4)
    return [I.star_patches(n_s, uv, I.star_coeffs(4 + q)) for q, n_s in enumerate((2, 3, 4))]


def seg(t, offs, q):
    return t[..., offs[q]:offs[q + 1]]


def test_batch_matches_separate(torch_dev, stars):
    torch = torch_dev
    import paper_2111_10743_amd as P
    X = np.concatenate([s[0] for s in stars])
    Xu = np.concatenate([s[1] for s in stars])
    Xv = np.concatenate([s[2] for s in stars])
    pps = [s[0].shape[0] for s in stars]
    note(f"batch setup patches {pps}")
    b = P.Surface(X, Xu, Xv, 4, patches_per_surf=pps)
    assert b.n_surf == 3
    singles = [P.Surface(*s, 4) for s in stars]
    offs = np.cumsum([0] + [s.N for s in singles])
    assert b.N == offs[-1]
    rng = np.random.default_rng(71)
    sig = rng.standard_normal((2, b.N))
    for prec, tol in ((64, 1e-13), (32, 1e-6)):
        dt = torch.float64 if prec == 64 else torch.float32
        tb = torch.tensor(sig, dtype=dt, device="cuda")
        ob = b.apply_gradS(tb)
        ab = b.apply_A3(tb)
        sb = b.apply_S(tb)
        gb = b.apply_gradS_adj(gpot=tb, gdSdn=tb)
        atb = b.apply_A3_adj(tb)
        torch.cuda.synchronize()
        exact = True
        for q, s in enumerate(singles):
            tq = seg(tb, offs, q).contiguous()
            oq = s.apply_gradS(tq)
            pairs = [(seg(ob["pot"], offs, q), oq["pot"]), (ob["grad"][:, offs[q]:offs[q + 1]], oq["grad"]),
                     (seg(ab, offs, q), s.apply_A3(tq)), (seg(sb, offs, q), s.apply_S(tq)),
                     (seg(gb, offs, q), s.apply_gradS_adj(gpot=tq, gdSdn=tq)),
                     (seg(atb, offs, q), s.apply_A3_adj(tq))]
            for k, (x, y) in enumerate(pairs):
                e = float((x.double() - y.double()).norm() / y.double().norm())
                exact &= bool(torch.equal(x, y))
                assert e < tol, (prec, q, k, e)
        note(f"prec {prec}: batch applies match the separate contexts (bit-identical: {exact})")
    # solves: two right-hand sides, both modes
    f = np.stack([I.sh_series(I.random_sh_coeffs(3, seed=8), X.reshape(-1, 3)),
                  X.reshape(-1, 3)[:, 0] * X.reshape(-1, 3)[:, 1]])
    fb = torch.tensor(f, device="cuda")
    for mode in (P.LB_SOLVE_FP64, P.LB_SOLVE_FP32_REFINE):
        ub, info, code = b.solve(fb, tol=1e-11, mode=mode)
        assert code == 0 and len(info) == 2 * 3
        for q, s in enumerate(singles):
            uq, iq, cq = s.solve(seg(fb, offs, q).contiguous(), tol=1e-11, mode=mode)
            e = rel_l2(seg(ub, offs, q).cpu().numpy().T, uq.cpu().numpy().T)
            note(f"mode {mode} surface {q}: solve vs separate {e:.2e}; iters {[info[r * 3 + q]['iters'] for r in range(2)]}"
                 f" vs {[i['iters'] for i in iq]}")
            assert e < 1e-9
            for r in range(2):
                assert abs(info[r * 3 + q]["removed_mean"] - iq[r]["removed_mean"]) < 1e-12 * (1 + abs(iq[r]["removed_mean"]))
        fbar, info, code = b.solve_adj(fb, tol=1e-11, mode=mode)
        assert code == 0
        for q, s in enumerate(singles):
            fq, _, _ = s.solve_adj(seg(fb, offs, q).contiguous(), tol=1e-11, mode=mode)
            e = rel_l2(seg(fbar, offs, q).cpu().numpy().T, fq.cpu().numpy().T)
            note(f"mode {mode} surface {q}: adjoint solve vs separate {e:.2e}")
            assert e < 1e-9
    b.close()
    for s in singles:
        s.close()


def test_batch_vs_oracle(torch_dev, stars):
    """The smallest star surface inside the batch against the oracle."""
    torch = torch_dev
    import paper_2111_10743_amd as P
    from oracle.geometry import Geometry
    from oracle.ops import Oracle
    X = np.concatenate([s[0] for s in stars])
    Xu = np.concatenate([s[1] for s in stars])
    Xv = np.concatenate([s[2] for s in stars])
    b = P.Surface(X, Xu, Xv, 4, patches_per_surf=[s[0].shape[0] for s in stars])
    g = Geometry(*stars[0], 4)
    o = Oracle(g)
    rng = np.random.default_rng(72)
    sig = rng.standard_normal(b.N)
    out = b.apply_gradS(torch.tensor(sig, device="cuda"))
    L = o.layer(sig[:g.N])
    e1 = rel_l2(out["pot"][:g.N].cpu().numpy(), L[:, 0])
    e2 = rel_l2(out["grad"][:g.N].cpu().numpy(), L[:, 1:4])
    a3 = b.apply_A3(torch.tensor(sig, device="cuda"))[:g.N].cpu().numpy()
    e3 = rel_l2(a3, o.A3(sig[:g.N]))
    note(f"batch surface 0 vs oracle: pot {e1:.2e} grad {e2:.2e} A3 {e3:.2e}")
    assert e1 < 1e-9 and e2 < 1e-9 and e3 < 1e-9
    b.close()
