"""Reference element on the standard simplex T0 = {u >= 0, v >= 0, u + v <= 1}.

Section 4 (discretization): each patch is a chart X: T0 -> Gamma whose
components, and those of dX/du and dX/dv, are polynomials represented by their
samples at stable interpolation nodes for the orthogonal (Koornwinder) basis on
T0.  The paper samples at Vioreanu-Rokhlin nodes, whose tables are not
reproduced here; this oracle uses the node family below (a reading recorded in
the design notes), with the order convention "total degree <= k",
n_p = (k+1)(k+2)/2 nodes.

Node family: the symmetric Blyth-Pozrikidis construction driven by the k+1
Gauss-Legendre points v_0 < ... < v_k of [0, 1]: for i + j + l = k the
barycentric coordinates are (1 + 2 v_a - v_b - v_c)/3 for (a, b, c) the cyclic
triple of (i, j, l).  All nodes are interior and the interpolatory weights are
positive for k = 1..7.

Plain definitions only: Vandermonde matrix of the orthonormal-up-to-scaling
Dubiner basis, interpolation L(u, v) = K(u, v) V^{-1}, weights
w = V^{-T} (integral of the basis), differentiation D = K_u V^{-1}.  TEST
INFRASTRUCTURE ONLY (see the package docstring).
"""
import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.special import eval_jacobi


def gauss01(n):
    """Gauss-Legendre nodes/weights on [0, 1] (numpy's leggauss, rescaled)."""
    x, w = leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def order_npts(k):
    return (k + 1) * (k + 2) // 2


def nodes(k):
    """Order-k interpolation nodes on T0, shape (n_p, 2), in (i, j) loop order."""
    if k < 1 or k > 7:
        raise ValueError("order must be in 1..7")
    v, _ = gauss01(k + 1)
    pts = []
    for i in range(k + 1):
        for j in range(k + 1 - i):
            l = k - i - j
            pts.append(((1.0 + 2.0 * v[i] - v[j] - v[l]) / 3.0,
                        (1.0 + 2.0 * v[j] - v[i] - v[l]) / 3.0))
    return np.array(pts)


def basis(k, u, v, deriv=False):
    """Dubiner/Koornwinder basis psi_{ij}(u, v), i + j <= k, anywhere on T0.

    psi_ij = (1 - v)^i P_i(xi) P_j^{(2i+1, 0)}(eta), xi = (2u - 1 + v)/(1 - v),
    eta = 2v - 1.  The factor Q_i = (1 - v)^i P_i(xi) is a polynomial in (u, v)
    computed by the Legendre recurrence multiplied through by (1 - v)^(i+1),
    so the vertex v = 1 needs no special case.  Returns K (npts, n_p), and
    K_u, K_v if deriv.
    """
    u = np.asarray(u, dtype=float)
    v = np.asarray(v, dtype=float)
    a = 2.0 * u - 1.0 + v
    b = 1.0 - v
    eta = 2.0 * v - 1.0
    # Q_i and derivatives (da/du = 2, da/dv = 1, db/dv = -1)
    Q = [np.ones_like(u), a]
    Qu = [np.zeros_like(u), 2.0 + 0.0 * u]
    Qv = [np.zeros_like(u), 1.0 + 0.0 * u]
    for i in range(1, k):
        Q.append(((2 * i + 1) * a * Q[i] - i * b * b * Q[i - 1]) / (i + 1))
        Qu.append(((2 * i + 1) * (2.0 * Q[i] + a * Qu[i]) - i * b * b * Qu[i - 1]) / (i + 1))
        Qv.append(((2 * i + 1) * (Q[i] + a * Qv[i])
                   - i * (-2.0 * b * Q[i - 1] + b * b * Qv[i - 1])) / (i + 1))
    cols, cu, cv = [], [], []
    for n in range(k + 1):
        for i in range(n + 1):
            j = n - i
            B = eval_jacobi(j, 2 * i + 1, 0, eta)
            cols.append(Q[i] * B)
            if deriv:
                dB = 0.5 * (j + 2 * i + 2) * eval_jacobi(j - 1, 2 * i + 2, 1, eta) if j > 0 else 0.0 * eta
                cu.append(Qu[i] * B)
                cv.append(Qv[i] * B + Q[i] * 2.0 * dB)
    K = np.stack(cols, axis=-1)
    if not deriv:
        return K
    return K, np.stack(cu, axis=-1), np.stack(cv, axis=-1)


class RefElem:
    """Everything about T0 that depends only on the order k (and q)."""

    def __init__(self, k, q):
        self.k = k
        self.n_p = order_npts(k)
        self.uv = nodes(k)
        V = basis(k, self.uv[:, 0], self.uv[:, 1])
        self.V = V
        self.Vinv = np.linalg.inv(V)
        # integral of each basis function over T0: only psi_00 = 1 survives
        # orthogonality; computed with a conical Gauss rule instead of relying
        # on it, which a test then checks against the exact monomial integrals.
        qu, qw = conical_rule(k + 2)
        integ = basis(k, qu[:, 0], qu[:, 1]).T @ qw
        self.w_ref = np.linalg.solve(V.T, integ)
        _, Ku, Kv = basis(k, self.uv[:, 0], self.uv[:, 1], deriv=True)
        self.Du = Ku @ self.Vinv
        self.Dv = Kv @ self.Vinv
        self.q = q
        self.over_uv, self.over_w = conical_rule(q)
        self.n_o = q * q
        self.P = self.interp(self.over_uv)

    def interp(self, uv):
        """Interpolation matrix from node values to values at the points uv."""
        uv = np.atleast_2d(uv)
        return basis(self.k, uv[:, 0], uv[:, 1]) @ self.Vinv


def conical_rule(q):
    """q x q conical-product Gauss rule on T0 (u = a (1 - b), v = b)."""
    a, wa = gauss01(q)
    U = np.empty((q * q, 2))
    W = np.empty(q * q)
    m = 0
    for jb in range(q):
        for ia in range(q):
            U[m, 0] = a[ia] * (1.0 - a[jb])
            U[m, 1] = a[jb]
            W[m] = wa[ia] * wa[jb] * (1.0 - a[jb])
            m += 1
    return U, W
