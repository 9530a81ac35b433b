"""Device generation of the quadrature corrections (Section 4, eqs. nys-lcq
and nys-lcq2: C = A - B for every (target, near patch) pair; the self rule
with its principal value, the adaptive near rule and the far rule with and
without the FP32 mask, all on the device).

* Against the oracle's corrections on sampled rows, at the bar of the host
  rule (2e-10 of the largest entry), for a sphere (k = 4) and an ellipsoid
  (k = 6).
* Against the host rules (LB_HOST_QUAD) on every block: the same rules, so
  the two differ by rounding order unless a leaf test of the near rule lands
  on the other side of its threshold, where both are within the rule's
  accuracy (2e-10 of the largest entry).  Every order 1..7 (each its own
  kernel instantiation), leaves of 25 points (near_q = 5: lanes left idle)
  and of 81 points (near_q = 9: two passes of the wavefront).
* FP64 applies of the two contexts agree to 1e-12 and FP32 applies to 1e-7:
  the FP32 corrections leave out exactly the far-rule points that the
  float32 near-field kernel skips, decided by the same float test on both
  sides (one point decided differently would show as an error of the order
  of its kernel value, far above float rounding).
"""
import sys
import time

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


def _self_mask(ptr, patch, n_p):
    N = len(ptr) - 1
    rows = np.repeat(np.arange(N), np.diff(ptr))
    return patch == rows // n_p


def _compare_to_host(P, X, Xu, Xv, k, label, **kw):
    t0 = time.perf_counter()
    d = P.Surface(X, Xu, Xv, k, **kw)
    t1 = time.perf_counter()
    h = P.Surface(X, Xu, Xv, k, host_quad=True, **kw)
    t2 = time.perf_counter()
    pd, cd, vd = d.corrections()
    ph, ch, vh = h.corrections()
    assert np.array_equal(pd, ph) and np.array_equal(cd, ch)
    selfb = _self_mask(pd, cd, d.sizes["n_p"])
    assert selfb.sum() == d.N
    scale = np.abs(vh).max()
    diff = np.abs(vd - vh).max(axis=(1, 2)) / scale
    ds, dn = diff[selfb], diff[~selfb]
    note(f"{label}: setup device rules {t1 - t0:.2f} s, host rules {t2 - t1:.2f} s; "
         f"self blocks {len(ds)}: max diff {ds.max():.1e}, median {np.median(ds):.1e}; "
         f"other blocks {len(dn)}: max {dn.max() if len(dn) else 0:.1e}, median {np.median(dn) if len(dn) else 0:.1e}")
    assert diff.max() < 2e-10
    return d, h


def test_corrections_against_oracle(torch_dev):
    import paper_2111_10743_amd as P
    from oracle.geometry import Geometry
    from oracle.quad import Corrections
    from oracle.refelem import nodes
    for label, k, (X, Xu, Xv) in (("sphere k=4", 4, I.sphere_patches(1, nodes(4))),
                                  ("ellipsoid k=6", 6, I.ellipsoid_patches(1, nodes(6), (1.0, 1.5, 2.0)))):
        note(f"{label}: device corrections vs oracle")
        s = P.Surface(X, Xu, Xv, k)
        g = Geometry(X, Xu, Xv, k)
        ptr, patch, vals = s.corrections()
        rows = np.arange(0, g.N, 11)
        c = Corrections(g, rows)
        scale = np.abs(c.C).max()
        worst = 0.0
        for r, i in enumerate(rows):
            assert np.array_equal(patch[ptr[i]:ptr[i + 1]], c.patch[c.ptr[r]:c.ptr[r + 1]])
            worst = max(worst, np.abs(vals[ptr[i]:ptr[i + 1]] - c.C[c.ptr[r]:c.ptr[r + 1]]).max() / scale)
        note(f"{label}: {len(rows)} rows, worst {worst:.1e} of the largest entry")
        assert worst < 2e-10
        s.close()


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
def test_every_order_against_host_rule(torch_dev, k):
    import paper_2111_10743_amd as P
    from oracle.refelem import nodes
    X, Xu, Xv = I.ellipsoid_patches(0, nodes(k), (1.0, 1.3, 0.8))
    d, h = _compare_to_host(P, X, Xu, Xv, k, f"ellipsoid order {k}")
    d.close()
    h.close()


@pytest.mark.parametrize("near_q", [5, 9])
def test_leaf_rule_sizes_and_applies(torch_dev, near_q):
    torch = torch_dev
    import paper_2111_10743_amd as P
    from oracle.refelem import nodes
    X, Xu, Xv = I.star_patches(2, nodes(5), I.star_coeffs(7))
    d, h = _compare_to_host(P, X, Xu, Xv, 5, f"star order 5 near_q={near_q}", near_q=near_q)
    x = torch.tensor(np.random.default_rng(5).standard_normal((2, d.N)), device="cuda")
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-7)):
        xd = x.to(dt)
        a, b = d.apply_gradS(xd), h.apply_gradS(xd)
        e = max(rel_l2(a[key].double().cpu().numpy(), b[key].double().cpu().numpy()) for key in ("pot", "grad"))
        e3 = rel_l2(d.apply_A3(xd).double().cpu().numpy(), h.apply_A3(xd).double().cpu().numpy())
        note(f"star near_q={near_q} {dt}: gradS applies differ {e:.1e}, A3 {e3:.1e}")
        assert e < tol and e3 < tol
    d.close()
    h.close()
