"""lb_export_setup / lb_import_setup through the C ABI: a context loaded from
a saved setup (corrections of eq. nys-lcq2 not regenerated, the saved
tuning re-applied) gives the same applies, A3 and solves bit for bit as the
context that was saved, for one surface and for a batch; damaged files are
rejected with LB_EINVAL."""
import os

import numpy as np
import pytest

import lbinputs as I

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _same(a, b):
    return all(__import__("torch").equal(a[k], b[k]) for k in a)


def test_saved_setup_bit_identical(torch_dev, tmp_path):
    torch = torch_dev
    import paper_2111_10743_amd as P
    from oracle.refelem import nodes
    X, Xu, Xv = I.ellipsoid_patches(3, nodes(4), (1.0, 1.5, 2.0))
    note("saved setup: ellipsoid 1280 order-4 patches, tuned")
    a = P.Surface(X, Xu, Xv, 4)
    a.set_tuning(32, 512, 32, 1, 1, 300, 1)
    a.set_tuning(64, 512, 64, 2, 0, 0, 0)
    path = str(tmp_path / "ellipsoid1280.lbsetup")
    a.save(path)
    note(f"saved {os.path.getsize(path) / 1e6:.1f} MB")
    b = P.Surface.load(path)
    assert b.sizes == a.sizes
    rng = np.random.default_rng(101)
    x = rng.standard_normal((2, a.N))
    for dt in (torch.float32, torch.float64):
        xs = torch.tensor(x, dtype=dt, device="cuda")
        ga, gb = a.apply_gradS(xs), b.apply_gradS(xs)
        same = _same(ga, gb) and torch.equal(a.apply_A3(xs), b.apply_A3(xs)) and \
            torch.equal(a.apply_S_adj(xs), b.apply_S_adj(xs))
        note(f"{dt}: applies bit-identical {same}")
        assert same
    f = torch.tensor(x, device="cuda")
    for mode in (P.LB_SOLVE_FP64, P.LB_SOLVE_FP32_REFINE):
        ua, ia, ca = a.solve(f, tol=1e-11, mode=mode)
        ub, ib, cb = b.solve(f, tol=1e-11, mode=mode)
        note(f"mode {mode}: iters {[i['iters'] for i in ia]} / {[i['iters'] for i in ib]}, setup "
             f"{ia[0]['t_setup']:.2f} s / imported {ib[0]['t_setup']:.2f} s")
        assert ca == cb == 0 and torch.equal(ua, ub)
        assert [i["iters"] for i in ia] == [i["iters"] for i in ib]
    a.close()
    b.close()


def test_saved_batch_setup(torch_dev, tmp_path):
    torch = torch_dev
    import paper_2111_10743_amd as P
    from oracle.refelem import nodes
    uv = nodes(4)
    parts = [I.star_patches(n, uv, I.star_coeffs(4 + q)) for q, n in enumerate((1, 2, 1))]
    X = np.concatenate([p[0] for p in parts])
    Xu = np.concatenate([p[1] for p in parts])
    Xv = np.concatenate([p[2] for p in parts])
    note("saved setup: batch of 3 star surfaces")
    a = P.Surface(X, Xu, Xv, 4, patches_per_surf=[p[0].shape[0] for p in parts])
    path = str(tmp_path / "batch.lbsetup")
    a.save(path)
    b = P.Surface.load(path)
    assert b.n_surf == 3 and b.N == a.N
    f = torch.tensor(np.random.default_rng(102).standard_normal(a.N), device="cuda")
    ua, _, ca = a.solve(f, tol=1e-11, mode=P.LB_SOLVE_FP32_REFINE)
    ub, _, cb = b.solve(f, tol=1e-11, mode=P.LB_SOLVE_FP32_REFINE)
    note(f"batch solve bit-identical {torch.equal(ua, ub)}")
    assert ca == cb == 0 and torch.equal(ua, ub)
    a.close()
    b.close()


def test_damaged_saved_setup_rejected(torch_dev, tmp_path):
    import paper_2111_10743_amd as P
    from oracle.refelem import nodes
    a = P.Surface(*I.sphere_patches(1, nodes(3)), 3)
    path = str(tmp_path / "s.lbsetup")
    a.save(path)
    data = bytearray(open(path, "rb").read())
    cases = {"missing": None, "truncated": data[: len(data) // 2], "flipped": None, "magic": b"XXXX" + data[4:]}
    flipped = bytearray(data)
    flipped[len(flipped) // 3] ^= 0x40
    cases["flipped"] = flipped
    for name, content in cases.items():
        p = str(tmp_path / f"{name}.lbsetup")
        if content is not None:
            open(p, "wb").write(bytes(content))
        with pytest.raises(P.LBError) as e:
            P.Surface.load(p)
        note(f"{name}: {e.value}")
        assert e.value.code == P.LB_EINVAL
    a.close()
