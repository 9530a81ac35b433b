"""Locally corrected quadrature: near/self integrals and corrections (FP64).

Section 4, eqs. (nys-lcq) and (nys-lcq2): for target x_i and each patch l in
Near(x_i) the correction is

    C^K_{i,lk} = A^K_{i,lk} - B^K_{i,lk},
    A^K_{i,lk} = int_{T0} K(x_i, X_l(u,v)) L_k(u,v) J_l(u,v) du dv   (accurate)
    B^K_{i,lk} = sum_m K(x_i, s_lm) w^over_lm P_mk                     (far rule)

so that  K[tau]_i = sum_m w^over_m K(x_i, s_m) tau~_m + sum_l sum_k C_{i,lk} tau_lk.
The paper uses generalized Gaussian quadrature and adaptive integration from a
third-party package that is not reproduced; this module computes A with
(reading recorded in the design notes):

* self patch: T0 split at the target node into three triangles, each mapped
  from [0,1]^2 by the Duffy map (radial variable s, edge variable along the
  opposite edge); the edge variable is graded with the sinh map about the foot
  of the perpendicular, measured in the chart's metric at the node, so that
  nodes close to an edge cost no more than central ones.  The displacement
  from the node to a point of the ray is formed without cancellation: the
  chart is a polynomial of degree k, so X(u0 + s e) - X(u0) =
  s int_0^1 X'(u0 + t s e) e dt exactly, with X' the derivative of the
  interpolated chart (degree k - 1) and ceil(k/2) Gauss points in t; the
  difference of two nearly equal positions would carry a rounding error
  proportional to |X| / |x - y| into the 1/r^2 kernels.  The gradient kernel is a Cauchy principal value with a ball of R^3
  as exclusion set: its 1/s part is subtracted and integrated analytically
  (Guiggiani-Gigante singularity subtraction), which adds f_{-1} ln|B| with
  B the chart's tangent along the ray.
  The double layer D has the same 1/s^2 term as S' with the opposite sign
  (non-zero on the interpolated chart only through the interpolation error),
  and takes the same subtraction.
* other near patches: level-by-level 4-way subdivision of T0 with a conical
  Gauss rule on each leaf; a leaf is accepted once its distance to the target
  is at least ``adm`` times its diameter.

Kernels (x target with normal n, y source with normal nu, d = x - y, r = |d|):
  S    : 1/(4 pi r)
  G_l  : d/dx_l of 1/(4 pi r) = -d_l/(4 pi r^3)            (l = 1, 2, 3)
  S'   : n . grad_x G
  SDD  : n . grad grad G . (n - nu)   (S'' + D', Section 3)
  D    : grad_y G . nu = (nu . d)/(4 pi r^3)   (the double layer, Section 3;
         weakly singular on a smooth surface, nu . d = O(r^2), so its
         on-surface principal value is the improper integral)
TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import numpy as np

from .refelem import basis, gauss01, conical_rule

FOUR_PI = 4.0 * np.pi
NK = 7  # S, Gx, Gy, Gz, S', SDD, D
KNAMES = ("S", "Gx", "Gy", "Gz", "Sp", "SDD", "D")


def kernels(x, n, y, nu):
    """Pointwise kernel values, shape (..., 6): S, Gx, Gy, Gz, SDD, D."""
    return kernels_d(x - y, n, nu)


def kernels_d(d, n, nu):
    """The same from the displacement d = x - y."""
    r2 = (d * d).sum(-1)
    r = np.sqrt(r2)
    inv_r = 1.0 / r
    inv_r3 = inv_r / r2
    out = np.empty(d.shape[:-1] + (6,))
    out[..., 0] = inv_r / FOUR_PI
    out[..., 1:4] = -d * inv_r3[..., None] / FOUR_PI
    m = n - nu
    nd = (n * d).sum(-1)
    md = (m * d).sum(-1)
    nm = (n * m).sum(-1)
    out[..., 4] = (3.0 * nd * md * inv_r3 / r2 - nm * inv_r3) / FOUR_PI
    out[..., 5] = (nu * d).sum(-1) * inv_r3 / FOUR_PI
    return out


def _chart(geom, patch, uv):
    """Interpolated X, X_u, X_v at param points uv (M,2) of patches patch (M,)."""
    L = basis(geom.k, uv[:, 0], uv[:, 1]) @ geom.re.Vinv            # (M, n_p)
    X = np.einsum('mb,mbc->mc', L, geom.Xp[patch])
    Xu = np.einsum('mb,mbc->mc', L, geom.Xup[patch])
    Xv = np.einsum('mb,mbc->mc', L, geom.Xvp[patch])
    return L, X, Xu, Xv


def _full(vals, n):
    """Expand (…,6) kernel values to the NK columns S, Gx, Gy, Gz, S', SDD, D
    with S' = n . G."""
    out = np.empty(vals.shape[:-1] + (NK,))
    out[..., 0:4] = vals[..., 0:4]
    out[..., 4] = (vals[..., 1:4] * n).sum(-1)
    out[..., 5] = vals[..., 4]
    out[..., 6] = vals[..., 5]
    return out


# ----------------------------------------------------------------------
# self patch: Duffy + sinh + principal-value subtraction
# ----------------------------------------------------------------------
def self_integrals(geom, targets, ns=16, nt=12, panel=2.0):
    """A^K_{i, p(i), k} for the given target nodes: array (T, n_p, NK).

    ns Gauss points along the ray; the sinh-graded edge variable is split into
    ceil(length / panel) equal panels of nt Gauss points each.
    """
    targets = np.asarray(targets)
    re = geom.re
    n_p = geom.n_p
    sg, sw = gauss01(ns)
    tg, tw = gauss01(nt)
    mg, mw = gauss01((geom.k + 1) // 2)      # exact for the degree k - 1 of X'
    verts = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    out = np.zeros((len(targets), n_p, NK))
    for ti, i in enumerate(targets):
        pch = geom.patch_of[i]
        a = geom.local_of[i]
        x0 = re.uv[a]
        xi = geom.x[i]
        ni = geom.n[i]
        Ji = geom.J[i]
        dXu = geom.dXu[pch, a]
        dXv = geom.dXv[pch, a]
        acc = np.zeros((n_p, NK))
        # metric of the interpolated chart at the node: the edge coordinate is
        # graded with sinh in the metric arclength, so that |X(y) - x_i| is
        # exactly s * h cosh(t) for an affine chart
        Gm = np.array([[dXu @ dXu, dXu @ dXv], [dXu @ dXv, dXv @ dXv]])
        for e in range(3):
            pa, pb = verts[e], verts[(e + 1) % 3]
            ed = pb - pa
            eG = np.sqrt(ed @ Gm @ ed)
            tstar = -((pa - x0) @ Gm @ ed) / (ed @ Gm @ ed)
            foot = pa + tstar * ed
            h = np.sqrt((foot - x0) @ Gm @ (foot - x0))
            c0 = abs((pa - x0)[0] * ed[1] - (pa - x0)[1] * ed[0])
            ta = np.arcsinh((0.0 - tstar) * eG / h)
            tb = np.arcsinh((1.0 - tstar) * eG / h)
            npan = max(1, int(np.ceil((tb - ta) / panel)))
            dl = (tb - ta) / npan
            tau = (ta + dl * (np.arange(npan)[:, None] + tg[None, :])).reshape(-1)
            wtau = np.tile(dl * tw, npan)
            E = foot[None, :] + (h * np.sinh(tau) / eG)[:, None] * ed[None, :]   # (nt,2)
            dvec = E - x0[None, :]                                           # (nt,2)
            jac_t = c0 * h * np.cosh(tau) / eG                               # area factor / s
            # points (nt, ns)
            uv = x0[None, None, :] + sg[None, :, None] * dvec[:, None, :]
            uvf = uv.reshape(-1, 2)
            L, X, Xu, Xv = _chart(geom, np.full(len(uvf), pch), uvf)
            cr = np.cross(Xu, Xv)
            J = np.linalg.norm(cr, axis=-1)
            nu = cr / J[:, None]
            # d = x_i - X(u0 + s e) = -s sum_j mw_j X'(u0 + mg_j s e) e,  e = dvec
            um = (x0[None, None, None, :] + (sg[None, :, None] * mg[None, None, :])[..., None]
                  * dvec[:, None, None, :])                                    # (nt, ns, m, 2)
            Lm = basis(geom.k, um[..., 0].ravel(), um[..., 1].ravel()) @ re.Vinv
            Lm = Lm.reshape(um.shape[:-1] + (n_p,))
            Xd = (np.einsum('tsmb,bc->tsmc', Lm, geom.dXu[pch]) * dvec[:, None, None, 0:1]
                  + np.einsum('tsmb,bc->tsmc', Lm, geom.dXv[pch]) * dvec[:, None, None, 1:2])
            d = -(sg[None, :, None] * np.einsum('m,tsmc->tsc', mw, Xd)).reshape(-1, 3)
            kv = _full(kernels_d(d, ni[None, :], nu), ni[None, :])              # (nt*ns, NK)
            wgt = (jac_t[:, None] * sg[None, :] * wtau[:, None] * sw[None, :]).reshape(-1)
            f = kv * (J * wgt)[:, None]                                     # (M, NK)
            acc += L.T @ f
            # principal-value subtraction for the gradient kernels (cols 1..4)
            B = dvec[:, 0:1] * dXu[None, :] + dvec[:, 1:2] * dXv[None, :]     # (nt,3)
            Bn = np.linalg.norm(B, axis=-1)
            fm1 = B / (FOUR_PI * Bn[:, None] ** 3) * (Ji * jac_t)[:, None]   # (nt,3)
            fm1_full = np.concatenate([fm1, (fm1 * ni).sum(-1, keepdims=True)], axis=1)  # Gx,Gy,Gz,S'
            # subtract sum_s ws fm1/s and add fm1 ln|B| (per tau), weights wtau
            sub = (sw / sg).sum()
            corr = (wtau[:, None] * fm1_full * (np.log(Bn)[:, None] - sub)).sum(0)
            acc[a, 1:5] += corr
            # D has the 1/s^2 part of S' with the opposite sign (nu . d = -n . d
            # to first order along the ray): the same principal value
            acc[a, 6] -= corr[3]
        out[ti] = acc
    return out


# ----------------------------------------------------------------------
# other near patches: adaptive subdivision
# ----------------------------------------------------------------------
def near_integrals(geom, tgt, pch, qa=8, adm=2.0, max_depth=16):
    """A^K_{i,l,k} for pairs (tgt[j], pch[j]) with pch not the target's patch."""
    tgt = np.asarray(tgt)
    pch = np.asarray(pch)
    M = len(tgt)
    n_p = geom.n_p
    out = np.zeros((M, n_p, NK))
    ru, rw = conical_rule(qa)
    tri = np.array([[[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]])
    pair = np.arange(M)
    tris = np.repeat(tri, M, axis=0)                 # (T,3,2)
    for depth in range(max_depth + 1):
        if len(pair) == 0:
            break
        # admissibility from mapped vertices and centroid
        pts = np.concatenate([tris, tris.mean(1, keepdims=True)], axis=1)   # (T,4,2)
        _, Xc, _, _ = _chart(geom, np.repeat(pch[pair], 4), pts.reshape(-1, 2))
        Xc = Xc.reshape(-1, 4, 3)
        diam = np.max(np.stack([np.linalg.norm(Xc[:, 0] - Xc[:, 1], axis=-1),
                                np.linalg.norm(Xc[:, 1] - Xc[:, 2], axis=-1),
                                np.linalg.norm(Xc[:, 2] - Xc[:, 0], axis=-1)]), axis=0)
        dist = np.linalg.norm(geom.x[tgt[pair]] - Xc[:, 3], axis=-1)
        acc = (dist >= adm * diam) | (depth == max_depth)
        if acc.any():
            ap = pair[acc]
            at = tris[acc]
            # map leaf rule
            p0 = at[:, 0]
            e1 = at[:, 1] - p0
            e2 = at[:, 2] - p0
            area2 = np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
            uv = p0[:, None, :] + ru[None, :, 0:1] * e1[:, None, :] + ru[None, :, 1:2] * e2[:, None, :]
            nq = len(ru)
            # chunk to bound memory
            CH = max(1, 20000 // nq)
            for c0 in range(0, len(ap), CH):
                sl = slice(c0, c0 + CH)
                apc = ap[sl]
                uvf = uv[sl].reshape(-1, 2)
                pp = np.repeat(pch[apc], nq)
                L, X, Xu, Xv = _chart(geom, pp, uvf)
                cr = np.cross(Xu, Xv)
                J = np.linalg.norm(cr, axis=-1)
                nu = cr / J[:, None]
                tt = np.repeat(tgt[apc], nq)
                kv = _full(kernels(geom.x[tt], geom.n[tt], X, nu), geom.n[tt])
                wq = (area2[sl][:, None] * rw[None, :]).reshape(-1) * J
                f = kv * wq[:, None]                                    # (m, NK)
                contrib = np.einsum('mb,mk->mbk', L, f).reshape(len(apc), nq, n_p, NK).sum(1)
                np.add.at(out, apc, contrib)
        rej = ~acc
        if not rej.any():
            break
        rp = pair[rej]
        rt = tris[rej]
        m01 = 0.5 * (rt[:, 0] + rt[:, 1])
        m12 = 0.5 * (rt[:, 1] + rt[:, 2])
        m20 = 0.5 * (rt[:, 2] + rt[:, 0])
        kids = np.stack([
            np.stack([rt[:, 0], m01, m20], 1),
            np.stack([m01, rt[:, 1], m12], 1),
            np.stack([m20, m12, rt[:, 2]], 1),
            np.stack([m12, m20, m01], 1)], 1)                         # (R,4,3,2)
        tris = kids.reshape(-1, 3, 2)
        pair = np.repeat(rp, 4)
    return out


def far_rule(geom, tgt, pch):
    """B^K_{i,l,k}: the oversampled rule restricted to patch l, (M, n_p, NK)."""
    tgt = np.asarray(tgt)
    pch = np.asarray(pch)
    n_o = geom.n_o
    P = geom.re.P
    out = np.empty((len(tgt), geom.n_p, NK))
    CH = 2048
    for c0 in range(0, len(tgt), CH):
        t = tgt[c0:c0 + CH]
        p = pch[c0:c0 + CH]
        idx = p[:, None] * n_o + np.arange(n_o)[None, :]
        y = geom.s[idx]
        nu = geom.nu[idx]
        kv = _full(kernels(geom.x[t][:, None, :], geom.n[t][:, None, :], y, nu), geom.n[t][:, None, :])
        kv = kv * geom.wo[idx][..., None]
        out[c0:c0 + CH] = np.einsum('mok,ob->mbk', kv, P)
    return out


class Corrections:
    """Block-sparse corrections C = A - B for a set of target rows."""

    def __init__(self, geom, targets=None, ns=16, nt=12, qa=8, adm=2.0):
        if targets is None:
            targets = np.arange(geom.N)
        targets = np.asarray(targets)
        self.targets = targets
        near = geom.near_lists(targets)
        self.ptr = np.zeros(len(targets) + 1, dtype=np.int64)
        self.ptr[1:] = np.cumsum([len(a) for a in near])
        self.patch = np.concatenate(near).astype(np.int64)
        rows = np.repeat(np.arange(len(targets)), np.diff(self.ptr))
        tg = targets[rows]
        A = np.zeros((len(self.patch), geom.n_p, NK))
        is_self = self.patch == geom.patch_of[tg]
        A[is_self] = self_integrals(geom, tg[is_self], ns=ns, nt=nt)
        A[~is_self] = near_integrals(geom, tg[~is_self], self.patch[~is_self], qa=qa, adm=adm)
        self.A = A
        self.B = far_rule(geom, tg, self.patch)
        self.C = A - self.B
        self.rows = rows

    def apply(self, geom, tau):
        """Near-correction part sum_l sum_k C_{i,lk} tau_lk for each row, (T, NK)."""
        tau_p = np.asarray(tau).reshape(geom.NP, geom.n_p)
        contrib = np.einsum('jbk,jb->jk', self.C, tau_p[self.patch])
        out = np.zeros((len(self.targets), NK))
        np.add.at(out, self.rows, contrib)
        return out
