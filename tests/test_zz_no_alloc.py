"""lb_apply_gradS_noalloc (the gradient apply whose workspace lives in a
static device array, for callers that cannot allocate) against
lb_apply_gradS through the C ABI: two calls in a row, the second on a
smaller surface with fewer densities, in both precisions; the same kernels
in the same order, so the outputs must be bit-identical.  A request whose
workspace does not fit the static array is rejected with LB_ENOMEM."""
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


def _outputs(torch, sigma):
    shp = sigma.shape
    return {"pot": torch.empty_like(sigma), "grad": torch.empty(shp + (3,), dtype=sigma.dtype, device=sigma.device),
            "dSdn": torch.empty_like(sigma),
            "surf_grad": torch.empty(shp + (3,), dtype=sigma.dtype, device=sigma.device)}


def test_noalloc_matches_apply_gradS(torch_dev):
    torch = torch_dev
    import paper_2111_10743_amd as P
    from oracle.refelem import nodes
    big = P.Surface(*I.ellipsoid_patches(3, nodes(4), (1.0, 1.5, 2.0)), 4)
    small = P.Surface(*I.sphere_patches(1, nodes(4)), 4)
    rng = np.random.default_rng(91)
    for surf, nd, name in ((big, 3, "ellipsoid 1280 patches, nd=3"), (small, 1, "sphere 80 patches, nd=1")):
        for dt in (torch.float32, torch.float64):
            note(f"noalloc {name} {dt}")
            sig = torch.tensor(rng.standard_normal((nd, surf.N)), dtype=dt, device="cuda")
            ref = surf.apply_gradS(sig)
            out = surf.apply_gradS_noalloc(sig, _outputs(torch, sig))
            torch.cuda.synchronize()
            for k in ("pot", "grad", "dSdn", "surf_grad"):
                same = torch.equal(out[k], ref[k])
                note(f"noalloc {name} {dt} {k}: bit-identical {same}")
                assert same, k
    # FP64 workspace of 8 densities on 1280 order-6 patches exceeds the static array
    huge = P.Surface(*I.ellipsoid_patches(3, nodes(6), (1.0, 1.5, 2.0)), 6)
    sig = torch.zeros((8, huge.N), dtype=torch.float64, device="cuda")
    note("noalloc oversized request")
    with pytest.raises(P.LBError) as e:
        huge.apply_gradS_noalloc(sig, _outputs(torch, sig))
    assert e.value.code == P.LB_ENOMEM and "static scratch" in str(e.value)
    for s in (big, small, huge):
        s.close()
