"""Discrete surface quantities from chart samples (FP64).

Section 2 (surface calculus in chart coordinates) and Section 4:
* smooth weights w_i = |X_u x X_v|_i w_ref,i and normals n = X_u x X_v / |.|;
* mean curvature H from second derivatives obtained by spectral
  differentiation of the stored first derivatives (Section 4, the paragraph on
  normals at oversampled nodes), with the sign that gives H = +1 on the unit
  sphere with the outward normal;
* the oversampled far rule: positions from the interpolated chart, normals
  and weights from the interpolated X_u, X_v (same paragraph);
* Near(x_i): patches with |x_i - c_l| < eta R_l (Section 4, the Near/Far split;
  the paper leaves the criterion open, eta = 2 by default).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import numpy as np
from scipy.spatial import cKDTree

from .refelem import RefElem


def _cross(a, b):
    return np.cross(a, b)


class Geometry:
    """All node/oversampled/near-list data of one surface."""

    def __init__(self, X, Xu, Xv, k, q=None, eta=2.0):
        X = np.asarray(X, dtype=float)
        Xu = np.asarray(Xu, dtype=float)
        Xv = np.asarray(Xv, dtype=float)
        if q is None:
            q = default_q(k)
        re = RefElem(k, q)
        self.re = re
        self.k = k
        self.NP = X.shape[0]
        self.n_p = re.n_p
        self.N = self.NP * self.n_p
        assert X.shape == (self.NP, self.n_p, 3)
        self.Xp, self.Xup, self.Xvp = X, Xu, Xv
        cr = _cross(Xu, Xv)
        J = np.linalg.norm(cr, axis=-1)
        self.J = J.reshape(-1)
        self.x = X.reshape(-1, 3)
        self.n = (cr / J[..., None]).reshape(-1, 3)
        self.w = (J * re.w_ref[None, :]).reshape(-1)
        self.area = self.w.sum()
        # spectral second derivatives of the chart
        Xuu = np.einsum('ab,pbc->pac', re.Du, Xu)
        Xvv = np.einsum('ab,pbc->pac', re.Dv, Xv)
        Xuv = 0.5 * (np.einsum('ab,pbc->pac', re.Dv, Xu) + np.einsum('ab,pbc->pac', re.Du, Xv))
        nn = cr / J[..., None]
        E = (Xu * Xu).sum(-1)
        F = (Xu * Xv).sum(-1)
        G = (Xv * Xv).sum(-1)
        L2 = (Xuu * nn).sum(-1)
        M2 = (Xuv * nn).sum(-1)
        N2 = (Xvv * nn).sum(-1)
        self.H = (-(E * N2 - 2.0 * F * M2 + G * L2) / (2.0 * (E * G - F * F))).reshape(-1)
        # tangential derivative of the interpolated X at the nodes (used by the
        # principal-value subtraction on the self patch)
        self.dXu = np.einsum('ab,pbc->pac', re.Du, X)
        self.dXv = np.einsum('ab,pbc->pac', re.Dv, X)
        # oversampled far rule
        P = re.P
        s = np.einsum('mb,pbc->pmc', P, X)
        su = np.einsum('mb,pbc->pmc', P, Xu)
        sv = np.einsum('mb,pbc->pmc', P, Xv)
        crs = _cross(su, sv)
        Js = np.linalg.norm(crs, axis=-1)
        self.n_o = re.n_o
        self.No = self.NP * self.n_o
        self.s = s.reshape(-1, 3)
        self.nu = (crs / Js[..., None]).reshape(-1, 3)
        self.wo = (Js * re.over_w[None, :]).reshape(-1)
        # patch centres and radii (nodes, oversampled points and mapped vertices)
        wp = self.w.reshape(self.NP, self.n_p)
        self.c = (wp[..., None] * X).sum(1) / wp.sum(1)[:, None]
        Lv = re.interp(np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]))
        verts = np.einsum('mb,pbc->pmc', Lv, X)
        d1 = np.linalg.norm(X - self.c[:, None, :], axis=-1).max(1)
        d2 = np.linalg.norm(s - self.c[:, None, :], axis=-1).max(1)
        d3 = np.linalg.norm(verts - self.c[:, None, :], axis=-1).max(1)
        self.R = np.maximum(np.maximum(d1, d2), d3)
        self.eta = eta
        self.patch_of = np.repeat(np.arange(self.NP), self.n_p)
        self.local_of = np.tile(np.arange(self.n_p), self.NP)
        self._near = None

    # ------------------------------------------------------------------
    def near_lists(self, targets=None):
        """Near(i) for the given target node indices: list of sorted patch arrays."""
        if targets is None:
            targets = np.arange(self.N)
        tree = cKDTree(self.c)
        rmax = self.eta * self.R.max()
        cand = tree.query_ball_point(self.x[targets], rmax)
        out = []
        for t, cl in zip(targets, cand):
            cl = np.asarray(cl, dtype=np.int64)
            d = np.linalg.norm(self.x[t] - self.c[cl], axis=-1)
            sel = cl[d < self.eta * self.R[cl]]
            sel = np.union1d(sel, [self.patch_of[t]])
            out.append(np.sort(sel))
        return out

    def coef(self, A):
        """Basis coefficients (n_p x 3) of per-patch node samples A (NP, n_p, 3)."""
        return np.einsum('ab,pbc->pac', self.re.Vinv, A)


def default_q(k):
    """Oversampling order of the far rule for order k (q x q conical points)."""
    return k + 6
