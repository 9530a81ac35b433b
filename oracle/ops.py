"""Discrete layer potentials, the A3 operator and GMRES (FP64, plain definitions).

* Section 4, eq. (nys-lcq2): K[tau]_i = sum over ALL oversampled sources of
  w^over_m K(x_i, s_m) tau~_m  +  sum over Near(i) of C_{i,lk} tau_lk.
  The far sum is evaluated directly (no FMM): the FMM only replaces this sum.
  The 1/(4 pi) of the Green's function (Section 3) is part of every kernel.
* Section 4.1 (the gradient part of the A1 apply): grad S, and the surface
  gradient grad_Gamma S = grad S - n (n . grad S), which equals the g^{ij}
  form of that section.
* Section 4.1 / eq. (ie-dis0): A1[tau] = div S[mu] + W(S tau) S[1] with
  mu = grad_Gamma S tau, div S[mu] = sum_l d_l S[mu_l] (each Cartesian
  component of mu a density of the single layer, its x_l derivative taken),
  applied right to left.
* Section 4.2 / eq. (ie-dis1): A2[tau] = -tau/4 + D[D tau]
  - S[(S''+D') tau + 2 H S' tau] + S W S tau, applied right to left: mu1 = D tau,
  mu2 = -(S''+D') tau - 2 H S' tau + W(S tau), A2 tau = -tau/4 + S mu2 + D mu1
  (the double layer D of Section 3 with the source normal: grad_y G . nu).
  Its right-hand side is S[f] and the solution u = S sigma (eq. ie-dis1).
* Section 4.3 / eq. (ie-dis2): A3[tau] = -tau/4 + S'[S' tau]
  - (S''+D')[S tau] - 2 H S'[S tau] + W S[S tau], applied right to left, with
  W[phi] = sum_j w_j phi_j / sum_j w_j (the averaging operator of Section 3).
* Section 6: GMRES, x0 = 0, no restart, at most 100 iterations, stop when
  the relative Euclidean residual drops below tol.  Arnoldi by modified
  Gram-Schmidt, Givens rotations.
* Lemma 1 / Section 3: f is projected onto mean zero, u = S[S[sigma]].
TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import numpy as np

from .quad import Corrections, FOUR_PI, NK


def direct(x, n, s, nu, c, chunk=None):
    """Direct sums over all sources for targets x (T,3) with normals n (T,3).

    c: strengths (No,) or (nd, No).  Returns pot (nd,T), grad (nd,T,3),
    sdd (nd,T) = sum c n.gradgrad G.(n - nu) and dbl (nd,T) = sum c grad_y G . nu
    (the double layer); every term includes 1/(4 pi).
    """
    c = np.atleast_2d(c)
    nd = c.shape[0]
    T = x.shape[0]
    pot = np.zeros((nd, T))
    grad = np.zeros((nd, T, 3))
    sdd = np.zeros((nd, T))
    dbl = np.zeros((nd, T))
    if chunk is None:
        chunk = max(1, int(4e6 // max(1, s.shape[0])))
    for t0 in range(0, T, chunk):
        xt = x[t0:t0 + chunk]
        nt = n[t0:t0 + chunk]
        d = xt[:, None, :] - s[None, :, :]                     # (t, No, 3)
        r2 = (d * d).sum(-1)
        inv_r = 1.0 / np.sqrt(r2)
        inv_r3 = inv_r / r2
        G = inv_r / FOUR_PI
        Gd = -d * (inv_r3 / FOUR_PI)[..., None]
        m = nt[:, None, :] - nu[None, :, :]
        ndt = (nt[:, None, :] * d).sum(-1)
        md = (m * d).sum(-1)
        nm = (nt[:, None, :] * m).sum(-1)
        H = (3.0 * ndt * md * inv_r3 / r2 - nm * inv_r3) / FOUR_PI
        pot[:, t0:t0 + chunk] = c @ G.T
        grad[:, t0:t0 + chunk, :] = np.einsum('dm,tmc->dtc', c, Gd)
        sdd[:, t0:t0 + chunk] = c @ H.T
        Dk = (nu[None, :, :] * d).sum(-1) * inv_r3 / FOUR_PI
        dbl[:, t0:t0 + chunk] = c @ Dk.T
    return pot, grad, sdd, dbl


class Oracle:
    """Discrete operators on one surface; ``targets`` restricts the rows.

    For small problems (rows x oversampled sources <= dense_limit) the kernel
    values of the far sum are tabulated once as dense matrices; the sums are
    the same, only evaluated as matrix-vector products.
    """

    def __init__(self, geom, targets=None, corr=None, dense_limit=2e7, **quad_opts):
        self.g = geom
        self.corr = corr if corr is not None else Corrections(geom, targets, **quad_opts)
        self.targets = self.corr.targets
        self._K = None
        if len(self.targets) * geom.No <= dense_limit:
            t = self.targets
            d = geom.x[t][:, None, :] - geom.s[None, :, :]
            r2 = (d * d).sum(-1)
            inv_r = 1.0 / np.sqrt(r2)
            inv_r3 = inv_r / r2
            n = geom.n[t][:, None, :]
            m = n - geom.nu[None, :, :]
            ndt = (n * d).sum(-1)
            K = np.empty((NK,) + r2.shape)
            K[0] = inv_r / FOUR_PI
            K[1:4] = np.moveaxis(-d * (inv_r3 / FOUR_PI)[..., None], -1, 0)
            K[4] = -ndt * inv_r3 / FOUR_PI
            K[5] = (3.0 * ndt * (m * d).sum(-1) * inv_r3 / r2 - (n * m).sum(-1) * inv_r3) / FOUR_PI
            K[6] = (geom.nu[None, :, :] * d).sum(-1) * inv_r3 / FOUR_PI
            self._K = K

    # -- pieces ---------------------------------------------------------
    def oversample(self, tau):
        """tau~ = P tau per patch, strengths w^over tau~ (Section 4, eq. nys-lcq)."""
        g = self.g
        tt = np.einsum('mb,pb->pm', g.re.P, np.asarray(tau).reshape(g.NP, g.n_p)).reshape(-1)
        return g.wo * tt

    def layer(self, tau):
        """All seven discrete kernels applied to tau at the target rows: (T, 7).

        Columns: S, dS/dx1, dS/dx2, dS/dx3, S', S''+D', D.
        """
        g = self.g
        t = self.targets
        c = self.oversample(tau)
        if self._K is not None:
            out = (self._K @ c).T
        else:
            pot, grad, sdd, dbl = direct(g.x[t], g.n[t], g.s, g.nu, c)
            out = np.empty((len(t), NK))
            out[:, 0] = pot[0]
            out[:, 1:4] = grad[0]
            out[:, 4] = (grad[0] * g.n[t]).sum(-1)
            out[:, 5] = sdd[0]
            out[:, 6] = dbl[0]
        return out + self.corr.apply(g, tau)

    def operator_matrices(self):
        """Dense matrices (7, rows, N) of the seven discrete kernels (small N only)."""
        g = self.g
        assert self._K is not None
        Pfull = np.zeros((g.No, g.N))
        for p in range(g.NP):
            Pfull[p * g.n_o:(p + 1) * g.n_o, p * g.n_p:(p + 1) * g.n_p] = g.re.P
        Pw = g.wo[:, None] * Pfull
        M = self._K @ Pw
        cr = self.corr
        for j in range(len(cr.patch)):
            r = cr.rows[j]
            p = cr.patch[j]
            M[:, r, p * g.n_p:(p + 1) * g.n_p] += cr.C[j].T
        return M

    # -- public applies ---------------------------------------------------
    def apply_S(self, tau):
        return self.layer(tau)[:, 0]

    def apply_gradS(self, tau):
        """Returns (S, grad S (T,3), S', grad_Gamma S (T,3))."""
        L = self.layer(tau)
        n = self.g.n[self.targets]
        grad = L[:, 1:4]
        sp = L[:, 4]
        surf = grad - n * (grad * n).sum(-1, keepdims=True)
        return L[:, 0], grad, sp, surf

    def adjoint_gradS(self, gpot=None, ggrad=None, gdSdn=None, gsurf=None):
        """Transpose of the discrete apply_gradS operator (all rows, small N).

        sigma_bar = S^T gpot + G^T gg with G = the three gradient rows
        (dS/dx1..3) and gg = ggrad + n gdSdn + (gsurf - n (n . gsurf)): the
        chain rule of S' = n . grad S and grad_Gamma S = grad S - n (n . grad S)
        (Section 4.1).  Each cotangent is optional.
        """
        g = self.g
        assert len(self.targets) == g.N
        if getattr(self, "_M", None) is None:
            self._M = self.operator_matrices()
        M = self._M
        n = g.n
        gg = np.zeros((g.N, 3))
        if ggrad is not None:
            gg += ggrad
        if gdSdn is not None:
            gg += n * gdSdn[:, None]
        if gsurf is not None:
            gg += gsurf - n * (gsurf * n).sum(-1, keepdims=True)
        out = np.einsum('kr,krn->n', gg.T, M[1:4])
        if gpot is not None:
            out += M[0].T @ gpot
        return out

    def position_vjp_S(self, sigma, gbar, patches=None):
        """Derivative of <gbar, S sigma> with respect to the node positions X.

        Reading of the kernel-position derivative: in the discrete S of
        eq. (nys-lcq2) the targets are the nodes x_i = X_i and the far-rule
        points move with the chart, s_m = (P X)_m (Section 4); the weights
        w^over, the oversampled density P sigma and the corrections are held
        fixed.  With c = w^over P sigma, phi(x) = sum_m c_m G(x - s_m) and
        psi(y) = sum_i gbar_i G(x_i - y):
            X_bar_j = gbar_j grad phi(x_j) + sum_{m in patch(j)} P_{m,k(j)} c_m grad psi(s_m).
        sigma, gbar: (N,) or (nd, N), summed over the densities.  Returns
        (len(patches) * n_p, 3) for the nodes of `patches` (default: all).
        """
        g = self.g
        sig = np.atleast_2d(np.asarray(sigma, dtype=float))
        gb = np.atleast_2d(np.asarray(gbar, dtype=float))
        pts = np.arange(g.NP) if patches is None else np.asarray(patches)
        nodes = (pts[:, None] * g.n_p + np.arange(g.n_p)[None, :]).reshape(-1)
        over = (pts[:, None] * g.n_o + np.arange(g.n_o)[None, :]).reshape(-1)
        c = np.stack([self.oversample(t) for t in sig])
        zn = np.zeros((len(nodes), 3))
        zo = np.zeros((len(over), 3))
        # grad phi at the nodes (far sum over every oversampled point)
        _, gphi, _, _ = direct(g.x[nodes], zn, g.s, np.zeros_like(g.s), c)
        # grad psi at the oversampled points (charges gbar on every node)
        _, gpsi, _, _ = direct(g.s[over], zo, g.x, np.zeros_like(g.x), gb)
        out = (gb[:, nodes, None] * gphi).sum(0)
        sbar = (c[:, over, None] * gpsi).sum(0).reshape(len(pts), g.n_o, 3)
        out += np.einsum('mk,pmc->pkc', g.re.P, sbar).reshape(-1, 3)
        return out

    def A3_matrix(self):
        """Dense A3 of Section 4.3 from the operator matrices (all rows, small N):
        -I/4 + S' S' - (S''+D') S - 2 diag(H) S' S + (1/area) 1 w^T S S."""
        g = self.g
        if getattr(self, "_M", None) is None:
            self._M = self.operator_matrices()
        S, Sp, K = self._M[0], self._M[4], self._M[5]
        SS = S @ S
        return (-0.25 * np.eye(g.N) + Sp @ Sp - K @ S - 2.0 * g.H[:, None] * (Sp @ S)
                + np.outer(np.ones(g.N), g.w @ SS) / g.w.sum())

    def A2_matrix(self):
        """Dense A2 of Section 4.2 from the operator matrices (all rows, small N):
        -I/4 + D D - S ((S''+D') + 2 diag(H) S') + (1/area) S 1 w^T S."""
        g = self.g
        if getattr(self, "_M", None) is None:
            self._M = self.operator_matrices()
        S, Sp, K, D = self._M[0], self._M[4], self._M[5], self._M[6]
        return (-0.25 * np.eye(g.N) + D @ D - S @ (K + 2.0 * g.H[:, None] * Sp)
                + np.outer(S @ np.ones(g.N), g.w @ S) / g.w.sum())

    def A1_matrix(self):
        """Dense A1 of Section 4.1 from the operator matrices (all rows, small N):
        sum_l G_l T_l G + (1/area) S 1 w^T S, with G = (G_1, G_2, G_3) the
        gradient matrices and T_l the l-th row of the tangential projector
        I - n n^T at each node."""
        g = self.g
        if getattr(self, "_M", None) is None:
            self._M = self.operator_matrices()
        S = self._M[0]
        G = self._M[1:4]
        A = np.outer(S @ np.ones(g.N), g.w @ S) / g.w.sum()
        for l in range(3):
            Mu = G[l] - g.n[:, l, None] * sum(g.n[:, m, None] * G[m] for m in range(3))
            A += G[l] @ Mu
        return A

    def A1(self, tau):
        """Section 4.1; needs all rows (targets == all nodes)."""
        g = self.g
        assert len(self.targets) == g.N
        L = self.layer(tau)
        grad = L[:, 1:4]
        mu = grad - g.n * (grad * g.n).sum(-1, keepdims=True)
        div = sum(self.layer(mu[:, l])[:, 1 + l] for l in range(3))
        phi0 = self.layer(np.ones(g.N))[:, 0]
        return div + self.W(L[:, 0]) * phi0

    def solve_adjoint(self, ubar):
        """fbar = (I - w 1^T / area) A3^{-T} S^T S^T ubar: the transpose of the
        linear map f -> u of solve() (mean projection, A3^{-1}, u = S S sigma)."""
        g = self.g
        if getattr(self, "_M", None) is None:
            self._M = self.operator_matrices()
        S = self._M[0]
        y = np.linalg.solve(self.A3_matrix().T, S.T @ (S.T @ ubar))
        return y - g.w * y.sum() / g.w.sum()

    def W(self, phi):
        g = self.g
        return (g.w * phi).sum() / g.w.sum()

    def A3(self, tau):
        """Section 4.3; needs all rows (targets == all nodes)."""
        g = self.g
        assert len(self.targets) == g.N
        L1 = self.layer(tau)
        mu1 = L1[:, 4]           # S' tau
        mu2 = L1[:, 0]           # S tau
        La = self.layer(mu1)
        Lb = self.layer(mu2)
        return (-0.25 * tau + La[:, 4] - Lb[:, 5] - 2.0 * g.H * Lb[:, 4]
                + self.W(Lb[:, 0]))

    def A2(self, tau):
        """Section 4.2; needs all rows (targets == all nodes)."""
        g = self.g
        assert len(self.targets) == g.N
        L1 = self.layer(tau)
        mu1 = L1[:, 6]                                              # D tau
        mu2 = -L1[:, 5] - 2.0 * g.H * L1[:, 4] + self.W(L1[:, 0])   # -(S''+D'+2HS') tau + W S tau
        return -0.25 * tau + self.layer(mu2)[:, 0] + self.layer(mu1)[:, 6]

    def solve_A2(self, f, tol=1e-12, max_iter=100):
        """u = S sigma with A2 sigma = S[f - mean] (eq. ie-dis1), plus info."""
        f = np.asarray(f, dtype=float)
        fz = f - self.W(f)
        sigma, info = gmres(self.A2, self.apply_S(fz), tol=tol, max_iter=max_iter)
        info["sigma"] = sigma
        return self.apply_S(sigma), info

    def solve(self, f, tol=1e-12, max_iter=100):
        """u solving Delta_Gamma u = f (mean-projected f), plus info dict."""
        g = self.g
        f = np.asarray(f, dtype=float)
        mean = self.W(f)
        fz = f - mean
        sigma, info = gmres(self.A3, fz, tol=tol, max_iter=max_iter)
        u = self.apply_S(self.apply_S(sigma))
        info["removed_mean"] = mean
        info["sigma"] = sigma
        return u, info


def gmres(A, b, tol=1e-12, max_iter=100):
    """Un-restarted GMRES, x0 = 0, MGS Arnoldi, Givens rotations (Section 6)."""
    b = np.asarray(b, dtype=float)
    n = b.shape[0]
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros(n), {"iters": 0, "rel_resid": 0.0, "history": []}
    m = max_iter
    V = np.zeros((m + 1, n))
    Hs = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    gvec = np.zeros(m + 1)
    gvec[0] = beta
    V[0] = b / beta
    hist = []
    k_done = 0
    for j in range(m):
        w = A(V[j])
        for i in range(j + 1):
            Hs[i, j] = np.dot(V[i], w)
            w = w - Hs[i, j] * V[i]
        Hs[j + 1, j] = np.linalg.norm(w)
        for i in range(j):
            t = cs[i] * Hs[i, j] + sn[i] * Hs[i + 1, j]
            Hs[i + 1, j] = -sn[i] * Hs[i, j] + cs[i] * Hs[i + 1, j]
            Hs[i, j] = t
        den = np.hypot(Hs[j, j], Hs[j + 1, j])
        cs[j] = Hs[j, j] / den
        sn[j] = Hs[j + 1, j] / den
        hnext = Hs[j + 1, j]
        Hs[j, j] = den
        Hs[j + 1, j] = 0.0
        gvec[j + 1] = -sn[j] * gvec[j]
        gvec[j] = cs[j] * gvec[j]
        k_done = j + 1
        rel = abs(gvec[j + 1]) / beta
        hist.append(rel)
        if rel < tol or hnext == 0.0:
            break
        V[j + 1] = w / hnext
    y = np.linalg.solve(np.triu(Hs[:k_done, :k_done]), gvec[:k_done])
    x = V[:k_done].T @ y
    return x, {"iters": k_done, "rel_resid": hist[-1], "history": hist}
