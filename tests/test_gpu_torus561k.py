"""The torus at its full size (R = 2, r = 0.7, 60 x 167 cells split in two:
20,040 order-6 patches, N = 561,120) with sixteen densities in one FMM
traversal, through the C ABI.

* FP64 and FP32 gradient applies of 16 densities (trigonometric series) in
  one call against the oracle on 32 sampled rows for three of them (S to
  1e-9 / 1e-6, grad S to 1e-8 / 4e-6: the FMM's gradient error on tori,
  2e-9 .. 5e-9 / 1.5e-6 here, see the N ~ 1M test), and density 7 of the batch against its own
  single-density apply (the traversal's M2L columns are independent: 1e-14
  FP64, 1e-6 FP32).
* The 2g count of the harmonic-vector-field section at this size: the
  Hodge-harmonic parts of four random tangential fields (lb_hodge, FP32 +
  refinement, tol 1e-9) span a space of dimension 2 = 2g.
"""
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
def torus(torch_dev):
    import paper_2111_10743_amd as P
    from oracle.refelem import nodes
    X, Xu, Xv = I.torus_patches(2.0, 0.7, 60, 167, nodes(6))
    note("torus561k setup")
    s = P.Surface(X, Xu, Xv, 6)
    note(f"torus561k sizes {s.sizes}")
    assert s.N == 561120
    yield s, X, Xu, Xv
    s.close()


def test_sixteen_densities_one_traversal(torch_dev, torus):
    torch = torch_dev
    from oracle.geometry import Geometry
    from oracle.ops import Oracle
    s, X, Xu, Xv = torus
    th, ph = I.torus_angles(X.reshape(-1, 3), 2.0)
    sig = np.stack([I.trig_series(th, ph, seed=sd) for sd in range(4, 20)])
    outs = {}
    for prec, dt in ((64, torch.float64), (32, torch.float32)):
        note(f"torus561k 16 densities prec={prec}")
        t = torch.tensor(sig, dtype=dt, device="cuda")
        o = s.apply_gradS(t)
        one = s.apply_gradS(t[7:8].contiguous())
        torch.cuda.synchronize()
        outs[prec] = {k: o[k].double().cpu().numpy() for k in ("pot", "grad")}
        e = max(float((o[k][7] - one[k][0]).double().norm() / one[k][0].double().norm()) for k in ("pot", "grad"))
        note(f"torus561k prec={prec}: density 7 batched vs alone {e:.2e}")
        assert e < (1e-14 if prec == 64 else 1e-6)
    g = Geometry(X, Xu, Xv, 6)
    rows = np.linspace(0, g.N - 1, 32).astype(np.int64)
    o = Oracle(g, rows, dense_limit=0)
    for d in (0, 7, 15):
        note(f"torus561k oracle density {d}")
        L = o.layer(sig[d])
        for prec, bar, gbar in ((64, 1e-9, 1e-8), (32, 1e-6, 4e-6)):
            pot, grad = outs[prec]["pot"][d][rows], outs[prec]["grad"][d][rows]
            e1, e2 = rel_l2(pot, L[:, 0]), rel_l2(grad, L[:, 1:4])
            m1, m2 = max_row(pot, L[:, 0]), max_row(grad, L[:, 1:4])
            note(f"density {d} prec={prec}: S {e1:.2e} (max row {m1:.2e}) grad S {e2:.2e} (max row {m2:.2e})")
            assert e1 < bar and e2 < gbar and m1 < 10 * bar and m2 < 10 * gbar


def test_harmonic_count_at_size(torch_dev, torus):
    torch = torch_dev
    import paper_2111_10743_amd as P
    s, X, Xu, Xv = torus
    x = X.reshape(-1, 3)
    w, nrm, _ = s.geometry()
    Fs = []
    for sd in range(3, 7):
        V = I.legendre_field(x, seed=sd, deg=5, L=2.7)
        Fs.append(V - nrm * (nrm * V).sum(1, keepdims=True))
    F = torch.tensor(np.stack(Fs), device="cuda")
    note("torus561k Hodge of four fields (8 right-hand sides, FP32 + refine)")
    _, _, H, info, code = s.hodge(F, tol=1e-9, mode=P.LB_SOLVE_FP32_REFINE)
    note(f"torus561k Hodge: iterations {[i['iters'] for i in info]}, code {code}")
    assert code == 0
    Hn = H.cpu().numpy().reshape(4, -1) * np.repeat(np.sqrt(w), 3)[None, :]
    sv = np.linalg.svd(Hn, compute_uv=False)
    note(f"torus561k harmonic parts: singular values {sv}")
    assert sv[1] > 1e-2 * sv[0] and sv[2] < 1e-5 * sv[0]
