"""The genus-2 input generator (lbinputs.genus2): a closed, outward-oriented
triangulation of the implicit surface with Euler characteristic -2 (genus 2),
chart samples on the surface to rounding, chart derivatives consistent with
the charts (finite differences at two step sizes agree), and the surface
area and enclosed volume converging under mesh refinement (the charts tile
the same smooth surface), with sum w n = 0 (a closed surface)."""
import numpy as np

from lbinputs import genus2 as G2
from oracle.geometry import Geometry
from oracle.refelem import nodes


def test_genus2_generator():
    S = G2.FusedTori()
    res = []
    for h in (0.26, 0.2):
        V, T = G2.mesh(S, h)
        assert G2.euler_characteristic(T) == -2
        amin, ratio = G2.quality(V, T)
        assert amin > 20.0 and ratio < 6.0, (amin, ratio)
        X, Xu, Xv = G2.patches(S, V, T, nodes(4))
        assert np.abs(S.F(X.reshape(-1, 3))).max() < 1e-13
        _, Xu2, Xv2 = G2.patches(S, V, T[:50], nodes(4), h=2e-4)
        assert np.abs(Xu2 - Xu[:50]).max() < 1e-9 and np.abs(Xv2 - Xv[:50]).max() < 1e-9
        g = Geometry(X, Xu, Xv, 4)
        assert np.all((S.grad(g.x) * g.n).sum(1) > 0)                     # outward
        assert np.abs((g.w[:, None] * g.n).sum(0)).max() < 1e-4 * g.w.sum()
        res.append((g.w.sum(), (g.w * (g.x * g.n).sum(1)).sum() / 3.0))
    (a1, v1), (a2, v2) = res
    assert abs(a1 - a2) < 1e-5 * a2 and abs(v1 - v2) < 1e-5 * v2, res
