"""Many uneven surfaces in one context: 64 star-shaped surfaces
r(xi) = 1 + 0.25 sum_{l<=4} a_lm Y_lm(xi), a_lm ~ U(-1, 1)/(l+1) (seed 4 + s),
on icosahedra whose faces are split n_s x n_s with n_s drawn from {2, 3, 4}
(seed 99), order 4: 80 to 320 patches (1,200 to 4,800 nodes) per surface.

* lb_autotune on the forest of 64 octrees;
* one right-hand side over all surfaces (64 GMRES systems sharing every
  apply, the operator replayed from a captured graph): FP32 + FP64
  refinement against the FP64 solve, <= 1e-9 on every surface;
* the manufactured solution of each surface: for phi = x1 x2 + x3 the
  surface Laplacian is Delta phi - n.(grad grad phi) n - 2 H dphi/dn =
  -2 n1 n2 - 2 H (n . grad phi) (Section 2), so u = phi - mean on each
  surface to discretization accuracy (below 1e-2, and falling from the
  n_s = 2 to the n_s = 4 surfaces);
* surfaces 0 and 63 against contexts of their own.
"""
import sys

import numpy as np
import pytest

import lbinputs as I
from conftest import rel_l2

pytestmark = pytest.mark.gpu

NSURF = 64


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_64_surfaces():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_10743_amd as P
    from oracle.geometry import Geometry
    from oracle.refelem import nodes
    uv = nodes(4)
    ns = np.random.default_rng(99).integers(2, 5, NSURF)
    surfs = [I.star_patches(int(n), uv, I.star_coeffs(4 + q)) for q, n in enumerate(ns)]
    geoms = [Geometry(*s, 4) for s in surfs]
    X = np.concatenate([s[0] for s in surfs])
    Xu = np.concatenate([s[1] for s in surfs])
    Xv = np.concatenate([s[2] for s in surfs])
    pps = [s[0].shape[0] for s in surfs]
    note(f"64 surfaces: patches {min(pps)}..{max(pps)}, total {sum(pps)}")
    b = P.Surface(X, Xu, Xv, 4, patches_per_surf=pps)
    assert b.n_surf == NSURF
    offs = np.cumsum([0] + [g.N for g in geoms])
    assert b.N == offs[-1]
    t = b.autotune(32, 1)
    note(f"64 surfaces: autotune fp32 leaf_src {t['leaf_src']} leaf_fmax {t['leaf_fmax']} "
         f"split {t['leaf_split']}: {t['ms_best']:.3f} ms (start {t['ms_default']:.3f} ms)")
    f, uex = [], []
    for g in geoms:
        x, n = g.x, g.n
        grad = np.stack([x[:, 1], x[:, 0], np.ones(g.N)], 1)
        f.append(-2.0 * n[:, 0] * n[:, 1] - 2.0 * g.H * (n * grad).sum(1))
        phi = x[:, 0] * x[:, 1] + x[:, 2]
        uex.append(phi - (g.w * phi).sum() / g.w.sum())
    fb = torch.tensor(np.concatenate(f), device="cuda")
    note("64 surfaces: FP64 solve")
    u64, i64, c64 = b.solve(fb, tol=1e-11, mode=P.LB_SOLVE_FP64)
    note("64 surfaces: FP32 + refinement solve")
    u32, i32, c32 = b.solve(fb, tol=1e-11, mode=P.LB_SOLVE_FP32_REFINE)
    assert c64 == 0 and c32 == 0 and len(i32) == NSURF
    u64, u32 = u64.cpu().numpy(), u32.cpu().numpy()
    worst_mode = 0.0
    ex = {2: [], 3: [], 4: []}
    for q, g in enumerate(geoms):
        a, z = offs[q], offs[q + 1]
        worst_mode = max(worst_mode, rel_l2(u32[a:z], u64[a:z], g.w))
        ex[int(ns[q])].append(rel_l2(u64[a:z], uex[q], g.w))
    note(f"64 surfaces: worst FP32+refine vs FP64 {worst_mode:.2e}, "
         f"iterations {min(i['iters'] for i in i32)}..{max(i['iters'] for i in i32)}")
    for k, v in ex.items():
        note(f"64 surfaces: n_s = {k}: {len(v)} surfaces, manufactured error mean {np.mean(v):.2e} max {np.max(v):.2e}")
    assert worst_mode < 1e-9
    # discretization error of the order-4 charts: small, and falling as the
    # faces are split finer
    assert max(max(v) for v in ex.values()) < 1e-2
    assert np.mean(ex[4]) < 0.5 * np.mean(ex[2])
    for q in (0, NSURF - 1):
        s = P.Surface(*surfs[q], 4)
        uq, iq, cq = s.solve(torch.tensor(f[q], device="cuda"), tol=1e-11, mode=P.LB_SOLVE_FP64)
        e = rel_l2(u64[offs[q]:offs[q + 1]], uq.cpu().numpy(), geoms[q].w)
        note(f"64 surfaces: surface {q} batched vs alone {e:.2e}")
        assert cq == 0 and e < 1e-9
        s.close()
    b.close()
