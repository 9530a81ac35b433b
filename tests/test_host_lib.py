"""Host-side checks of liblb.so (no GPU): the C ABI loads and exports every
symbol of include/lb.h, argument errors come back as status codes, and the
library's host setup (nodes, geometry, near lists, corrections) agrees with
the oracle's independent implementation."""
import os
import re

import numpy as np
import pytest

import lbinputs as I
from oracle.geometry import Geometry
from oracle.quad import Corrections
from oracle.refelem import nodes, RefElem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2111_10743_amd import lb
    return lb


def test_exports_every_declared_symbol():
    lb = _lib()
    L = lb.lib()
    hdr = open(os.path.join(ROOT, "include", "lb.h")).read()
    names = set(re.findall(r"\b(lb_[A-Za-z_0-9]+)\s*\(", hdr))
    assert names == set(lb.EXPORTED)
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("k", [1, 4, 6, 7])
def test_ref_nodes_match_oracle(k):
    uv, w = _lib().ref_nodes(k)
    assert np.abs(uv - nodes(k)).max() < 1e-15
    assert np.abs(w - RefElem(k, k + 2).w_ref).max() < 1e-14


def test_error_codes():
    lb = _lib()
    uv, _ = lb.ref_nodes(4)
    X, Xu, Xv = I.sphere_patches(0, uv)
    with pytest.raises(lb.LBError) as e:
        lb.Surface(X, Xu, Xv, 9, host_only=True)
    assert e.value.code == lb.LB_EINVAL
    Xn = X.copy()
    Xn[3, 2, 1] = np.nan
    with pytest.raises(lb.LBError) as e:
        lb.Surface(Xn, Xu, Xv, 4, host_only=True)
    assert e.value.code == lb.LB_EINVAL
    Xz = Xu.copy()
    Xz[5] = 0.0
    with pytest.raises(lb.LBError) as e:
        lb.Surface(X, Xz, Xv, 4, host_only=True)
    assert e.value.code == lb.LB_EGEOM
    for bad in (-1.0, float("nan")):
        with pytest.raises(lb.LBError) as e:
            lb.Surface(X, Xu, Xv, 4, host_only=True, m2l_trunc64=bad)
        assert e.value.code == lb.LB_EINVAL
    s = lb.Surface(X, Xu, Xv, 4, host_only=True)
    import ctypes
    code = lb.lib().lb_apply_S(s._ctx, 1, 32, ctypes.c_void_p(16), ctypes.c_void_p(16), None)
    assert code == lb.LB_EINVAL          # host-only context: no device state


@pytest.mark.parametrize("case", ["sphere_k4", "ellipsoid_k6"])
def test_host_corrections_match_oracle(case):
    lb = _lib()
    if case == "sphere_k4":
        k = 4
        X, Xu, Xv = I.sphere_patches(1, nodes(k))
    else:
        k = 6
        X, Xu, Xv = I.ellipsoid_patches(1, nodes(k), (1.0, 1.5, 2.0))
    s = lb.Surface(X, Xu, Xv, k, host_only=True)
    g = Geometry(X, Xu, Xv, k)
    w, n, H = s.geometry()
    assert np.abs(w - g.w).max() < 1e-15
    assert np.abs(n - g.n).max() < 1e-14
    assert np.abs(H - g.H).max() < 1e-11
    ptr, patch, vals = s.corrections()
    rows = np.arange(0, g.N, 11)
    c = Corrections(g, rows)
    scale = np.abs(c.C).max()
    for r, i in enumerate(rows):
        assert np.array_equal(patch[ptr[i]:ptr[i + 1]], c.patch[c.ptr[r]:c.ptr[r + 1]])
        d = np.abs(vals[ptr[i]:ptr[i + 1]] - c.C[c.ptr[r]:c.ptr[r + 1]]).max()
        assert d < 2e-10 * scale, (i, d)


def test_host_only_rejects_device_entry_points():
    """A LB_HOST_ONLY context has no device state: every entry point that
    needs it returns LB_EINVAL without touching the (bogus) pointers, and
    lb_get_corrections still returns the host-rule corrections."""
    import ctypes
    lb = _lib()
    uv, _ = lb.ref_nodes(3)
    X, Xu, Xv = I.sphere_patches(0, uv)
    s = lb.Surface(X, Xu, Xv, 3, host_only=True)
    L = lb.lib()
    p = ctypes.c_void_p(16)
    info = lb.SolveInfo()
    cfg = lb.TuneInfo()
    cfg.leaf_src, cfg.leaf_fmax = 1024, 64
    assert L.lb_apply_A1(s._ctx, 1, 64, p, p, None) == lb.LB_EINVAL
    assert L.lb_surface_grad(s._ctx, 1, p, p, None) == lb.LB_EINVAL
    assert L.lb_surface_div(s._ctx, 1, p, 0, p, None) == lb.LB_EINVAL
    assert L.lb_hodge(s._ctx, 1, p, None, None, p, 1e-10, 0, ctypes.byref(info), None) == lb.LB_EINVAL
    assert L.lb_set_tuning(s._ctx, 32, ctypes.byref(cfg)) == lb.LB_EINVAL
    ptr, patch, vals = s.corrections()
    assert ptr[-1] == len(patch) and np.isfinite(vals).all() and np.abs(vals).max() > 0


def test_saved_setup_errors_on_host(tmp_path):
    """lb_export_setup refuses a host-only context and lb_import_setup a file
    that is not a saved setup, before any device call."""
    import ctypes
    import paper_2111_10743_amd as P
    from oracle.refelem import nodes
    import lbinputs as I
    s = P.Surface(*I.sphere_patches(0, nodes(2)), 2, host_only=True)
    with pytest.raises(P.LBError) as e:
        s.save(str(tmp_path / "x.lbsetup"))
    assert e.value.code == P.LB_EINVAL and "LB_HOST_ONLY" in str(e.value)
    bad = tmp_path / "bad.lbsetup"
    bad.write_bytes(b"not a setup at all")
    ctx = ctypes.c_void_p()
    code = P.lib().lb_import_setup(ctypes.byref(ctx), str(bad).encode(), None)
    assert code == P.LB_EINVAL and not ctx
    s.close()
