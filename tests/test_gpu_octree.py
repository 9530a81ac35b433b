"""The device octree build (HIP kernels) against the oracle and the host
build: bit-exact integer results (orders, ranges, boxes, U- and V-lists).

Cases: the oracle's edge cases (depth 0 and 1, one target, grid-aligned and
coincident points); an ellipsoid-like cloud of 150,000 points (radix sort
tiles of 4096 with a ragged tail, automatic depth) against the host build;
the trees of a surface context (FP32, FP64 and the transposed trees of the
adjoint applies) against a context built with LB_HOST_OCTREE, whose applies
must then agree bit for bit.
"""
import sys

import numpy as np
import pytest

from test_oracle_octree import KEYS, surface_points, tree_cases

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


def same(a, b):
    return all(np.array_equal(np.asarray(a[k]), np.asarray(b[k])) for k in KEYS) and a["depth"] == b["depth"]


@pytest.mark.parametrize("name,tgt,src,depth", list(tree_cases()), ids=lambda v: v if isinstance(v, str) else "")
def test_device_tree_matches_oracle(torch_dev, name, tgt, src, depth):
    import paper_2111_10743_amd as P
    from oracle.octree import Tree
    note(f"device tree {name} nt={len(tgt)} ns={len(src)} depth={depth}")
    d = P.build_tree(tgt, src, leaf_src=64, depth=depth, device=True)
    o = Tree(tgt, src, d["depth"])
    h = P.build_tree(tgt, src, leaf_src=64, depth=depth, device=False)
    assert d["depth"] == h["depth"]
    for k in KEYS:
        assert np.array_equal(np.asarray(d[k]), np.asarray(getattr(o, k))), k


@pytest.mark.parametrize("leaf_src", [64, 1024])
def test_device_tree_large(torch_dev, leaf_src):
    import paper_2111_10743_amd as P
    rng = np.random.default_rng(17)
    tgt, src = surface_points(rng, 50_001), surface_points(rng, 150_003)
    note(f"device tree large leaf_src={leaf_src}")
    d = P.build_tree(tgt, src, leaf_src=leaf_src, device=True)
    h = P.build_tree(tgt, src, leaf_src=leaf_src, device=False)
    note(f"depth {d['depth']} boxes {len(d['boxes'])} vlist {len(d['vlist_src'])}")
    assert same(d, h)


def test_context_trees_and_applies(torch_dev):
    torch = torch_dev
    import paper_2111_10743_amd as P
    import lbinputs as I
    X, Xu, Xv = I.ellipsoid_patches(2, P.ref_nodes(6)[0], (1.0, 1.5, 2.0))
    note("context trees: device build")
    a = P.Surface(X, Xu, Xv, 6)
    note("context trees: host build")
    b = P.Surface(X, Xu, Xv, 6, host_octree=True)
    rng = np.random.default_rng(3)
    for prec in (32, 64):
        dt = torch.float32 if prec == 32 else torch.float64
        sig = torch.tensor(rng.standard_normal(a.N), dtype=dt, device="cuda")
        a.apply_S_adj(sig)
        b.apply_S_adj(sig)
        for tr in (False, True):
            assert same(a.tree(prec, tr), b.tree(prec, tr)), (prec, tr)
        oa, ob = a.apply_gradS(sig), b.apply_gradS(sig)
        torch.cuda.synchronize()
        assert torch.equal(oa["pot"], ob["pot"]) and torch.equal(oa["grad"], ob["grad"])
        assert torch.equal(a.apply_S_adj(sig), b.apply_S_adj(sig))
        note(f"prec {prec}: trees equal, applies bit-identical")
    a.close()
    b.close()
