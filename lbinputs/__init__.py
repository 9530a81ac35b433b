"""Seeded synthetic inputs: analytic surface charts and right-hand sides.

This module holds no arithmetic of the method: it only samples analytic charts
X(u, v) and their exact derivatives at caller-supplied reference points, and
evaluates analytic test functions.  Both the oracle-side tests and the HIP
side (tests, bench) consume it; it imports neither.

Surfaces (each patch is a chart T0 -> Gamma, T0 = {u, v >= 0, u + v <= 1}):
* ``sphere_patches(nsub)``: icosahedron, ``nsub`` 4-way splits with midpoints
  pushed to the sphere at each level, each flat triangle (A, B, C) radially
  projected: X = P/|P|, P = A + u (B - A) + v (C - A).  80 patches at nsub=1,
  5120 at nsub=4.
* ``ellipsoid_patches(nsub, axes)``: the same charts scaled by diag(axes).
* ``torus_patches(R, r, n_theta, n_phi)``: (theta, phi) grid, each cell split
  along a fixed diagonal.
* ``star_patches(n_s, uv, coeffs)``: r(xi) = 1 + 0.25 sum a_lm Y_lm(xi) on
  the sphere charts of an icosahedron whose faces are split n_s x n_s
  (``star_coeffs(seed)`` draws the a_lm).
"""
import numpy as np
from scipy.special import sph_harm_y


# ----------------------------------------------------------------------
# icosahedral triangulations of the unit sphere
# ----------------------------------------------------------------------
def icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=float)
    V /= np.linalg.norm(V, axis=1)[:, None]
    F = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]])
    return V, F


def icosphere(nsub):
    """Vertices (on the unit sphere) and outward-oriented faces."""
    V, F = icosahedron()
    V = list(V)
    for _ in range(nsub):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]
        nf = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]]
        F = np.array(nf)
    V = np.array(V)
    # orient outward
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    flip = (np.cross(B - A, C - A) * (A + B + C)).sum(1) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def icosphere_ns(n_s):
    """Icosahedron with every face split into n_s^2 triangles (projected)."""
    V0, F0 = icosahedron()
    tris = []
    for a, b, c in F0:
        A, B, C = V0[a], V0[b], V0[c]
        P = {}
        for i in range(n_s + 1):
            for j in range(n_s + 1 - i):
                p = A + (B - A) * i / n_s + (C - A) * j / n_s
                P[(i, j)] = p / np.linalg.norm(p)
        for i in range(n_s):
            for j in range(n_s - i):
                tris.append((P[(i, j)], P[(i + 1, j)], P[(i, j + 1)]))
                if i + j < n_s - 1:
                    tris.append((P[(i + 1, j)], P[(i + 1, j + 1)], P[(i, j + 1)]))
    T = np.array(tris)
    flip = (np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]) * T.sum(1)).sum(1) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return T


def _radial_charts(T, uv):
    """Radial projection of flat triangles T (NP,3,3) sampled at uv (n,2)."""
    A, B, C = T[:, 0], T[:, 1], T[:, 2]
    u = uv[None, :, 0:1]
    v = uv[None, :, 1:2]
    P = A[:, None, :] + u * (B - A)[:, None, :] + v * (C - A)[:, None, :]
    nP = np.linalg.norm(P, axis=-1, keepdims=True)
    X = P / nP

    def d(Dv):
        Dv = Dv[:, None, :]
        return (Dv - X * (X * Dv).sum(-1, keepdims=True)) / nP
    return X, d(B - A), d(C - A)


def sphere_patches(nsub, uv, radius=1.0):
    V, F = icosphere(nsub)
    T = V[F]
    X, Xu, Xv = _radial_charts(T, np.asarray(uv, dtype=float))
    return radius * X, radius * Xu, radius * Xv


def ellipsoid_patches(nsub, uv, axes=(1.0, 1.5, 2.0)):
    X, Xu, Xv = sphere_patches(nsub, uv)
    a = np.asarray(axes, dtype=float)
    return X * a, Xu * a, Xv * a


def sphere_preimage(X, axes):
    """Unit-sphere point xi whose scaled image is X (for ellipsoid data)."""
    return X / np.asarray(axes, dtype=float)


def torus_patches(R, r, n_theta, n_phi, uv):
    """Torus X = ((R + r cos th) cos ph, (R + r cos th) sin ph, r sin th).

    The (ph, th) grid has n_phi x n_theta cells; each cell is split into the
    triangles corner (0,0) + u e_ph + v e_th and corner (1,1) - u e_ph - v e_th,
    so that X_u x X_v points outward.  Patch order: theta-major, phi, triangle.
    """
    uv = np.asarray(uv, dtype=float)
    dth = 2 * np.pi / n_theta
    dph = 2 * np.pi / n_phi
    Xs, Us, Vs = [], [], []
    for it in range(n_theta):
        for ip in range(n_phi):
            for corner, sgn in (((0, 0), 1.0), ((1, 1), -1.0)):
                ph = (ip + corner[0]) * dph + sgn * dph * uv[:, 0]
                th = (it + corner[1]) * dth + sgn * dth * uv[:, 1]
                ct, st, cp, sp = np.cos(th), np.sin(th), np.cos(ph), np.sin(ph)
                rho = R + r * ct
                X = np.stack([rho * cp, rho * sp, r * st], -1)
                Xth = np.stack([-r * st * cp, -r * st * sp, r * ct], -1)
                Xph = np.stack([-rho * sp, rho * cp, 0 * ct], -1)
                Xs.append(X)
                Us.append(sgn * dph * Xph)
                Vs.append(sgn * dth * Xth)
    return np.array(Xs), np.array(Us), np.array(Vs)


# twisted torus: X(u, v) = sum_{i,j} d_ij (cos v cos t, sin v cos t, sin t),
# t = (1 - i) u + j v, with the nonzero d_ij below (harmonic-fields section)
TWISTED_TORUS_COEFFS = {(-1, -1): 0.17, (-1, 0): 0.11, (0, 0): 1.0, (1, 0): 4.5, (2, 0): -0.25,
                        (0, 1): 0.01, (2, 1): -0.45}


def twisted_torus_point(u, v):
    """X, X_u, X_v of the twisted torus at parameters (u, v) (arrays)."""
    u = np.asarray(u, dtype=float)
    v = np.asarray(v, dtype=float)
    X = np.zeros(u.shape + (3,))
    Xu = np.zeros_like(X)
    Xv = np.zeros_like(X)
    cv, sv = np.cos(v), np.sin(v)
    for (i, j), d in TWISTED_TORUS_COEFFS.items():
        t = (1 - i) * u + j * v
        ct, st = np.cos(t), np.sin(t)
        X += d * np.stack([cv * ct, sv * ct, st], -1)
        dt = np.stack([-cv * st, -sv * st, ct], -1)        # d/dt
        Xu += d * (1 - i) * dt
        Xv += d * (np.stack([-sv * ct, cv * ct, 0 * ct], -1) + j * dt)
    return X, Xu, Xv


def twisted_torus_patches(n_u, n_v, uv):
    """The twisted torus on an n_v x n_u grid of (v, u) cells (v the long way
    round), each cell split into the triangles corner (0,0) + a e_v + b e_u
    and corner (1,1) - a e_v - b e_u, so that X_a x X_b points outward."""
    uv = np.asarray(uv, dtype=float)
    du = 2 * np.pi / n_u
    dv = 2 * np.pi / n_v
    Xs, As, Bs = [], [], []
    for iu in range(n_u):
        for iv in range(n_v):
            for corner, sgn in (((0, 0), 1.0), ((1, 1), -1.0)):
                v = (iv + corner[0]) * dv + sgn * dv * uv[:, 0]
                u = (iu + corner[1]) * du + sgn * du * uv[:, 1]
                X, Xu, Xv = twisted_torus_point(u, v)
                Xs.append(X)
                As.append(sgn * dv * Xv)
                Bs.append(sgn * du * Xu)
    return np.array(Xs), np.array(As), np.array(Bs)


def current_source_field(x, x0=(0.2, 0.2, 0.2), ell=(0.0, 1.0, 1.0)):
    """V = ell x (x - x0) / |x - x0|^3 (a line current element at x0)."""
    d = np.asarray(x, dtype=float) - np.asarray(x0, dtype=float)
    r3 = np.linalg.norm(d, axis=-1, keepdims=True) ** 3
    return np.cross(np.asarray(ell, dtype=float), d) / r3


def torus_mean_curvature(X, R, r):
    """H = (R + 2 r cos th) / (2 r (R + r cos th)) with the outward normal."""
    rho = np.linalg.norm(X[..., :2], axis=-1)
    ct = (rho - R) / r
    return (R + 2 * r * ct) / (2 * r * (R + r * ct))


# ----------------------------------------------------------------------
# analytic functions
# ----------------------------------------------------------------------
def real_sph_harm(l, m, x):
    """Real orthonormal spherical harmonic Y_lm at unit vectors x (..., 3)."""
    x = np.asarray(x, dtype=float)
    r = np.linalg.norm(x, axis=-1)
    theta = np.arccos(np.clip(x[..., 2] / r, -1, 1))
    phi = np.arctan2(x[..., 1], x[..., 0])
    Y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return np.sqrt(2.0) * (-1) ** m * Y.real
    if m < 0:
        return np.sqrt(2.0) * (-1) ** m * Y.imag
    return Y.real


def sh_gradient_on_sphere(l, m, x, h=1e-6):
    """Surface gradient of Y_lm on the unit sphere (central differences of the
    degree-0 homogeneous extension, projected on the tangent plane)."""
    x = np.asarray(x, dtype=float)
    g = np.zeros_like(x)
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        g[..., c] = (real_sph_harm(l, m, x + e) - real_sph_harm(l, m, x - e)) / (2 * h)
    n = x / np.linalg.norm(x, axis=-1, keepdims=True)
    return g - n * (g * n).sum(-1, keepdims=True)


def random_sh_coeffs(lmax, seed, decay=2.0, lmin=1):
    """a_lm ~ N(0,1) (l+1)^-decay for lmin <= l <= lmax (seeded)."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(lmin, lmax + 1):
        for m in range(-l, l + 1):
            out.append((l, m, rng.standard_normal() * (l + 1.0) ** (-decay)))
    return out


def sh_series(coeffs, x):
    return sum(a * real_sph_harm(l, m, x) for l, m, a in coeffs)


# ----------------------------------------------------------------------
# star-shaped surfaces r(xi) = 1 + amp * sum_{l <= lmax} a_lm Y_lm(xi)
# ----------------------------------------------------------------------
def star_coeffs(seed, lmax=4, amp=0.25, rmin=0.3):
    """a_lm ~ U(-1, 1) / (l + 1), l = 0..lmax (seeded); redrawn until the
    radius stays >= rmin on a fine sample of the sphere."""
    rng = np.random.default_rng(seed)
    probe = icosphere(4)[0]
    while True:
        c = [(l, m, rng.uniform(-1.0, 1.0) / (l + 1.0)) for l in range(lmax + 1) for m in range(-l, l + 1)]
        if (1.0 + amp * sh_series(c, probe)).min() >= rmin:
            return c


def star_patches(n_s, uv, coeffs, amp=0.25, h=1e-3):
    """Charts X = r(xi) xi over the icosahedron split into n_s^2 triangles per
    face; X_u = r xi_u + (d r / d u) xi with the derivative of r along the
    chart by 4th-order central differences of r(normalize(xi + t xi_u))."""
    T = icosphere_ns(n_s)
    xi, xu, xv = _radial_charts(T, np.asarray(uv, dtype=float))
    r = lambda p: 1.0 + amp * sh_series(coeffs, p / np.linalg.norm(p, axis=-1, keepdims=True))

    def dr(d):
        return (-r(xi + 2 * h * d) + 8 * r(xi + h * d) - 8 * r(xi - h * d) + r(xi - 2 * h * d)) / (12 * h)
    r0 = r(xi)[..., None]
    X = r0 * xi
    Xu = r0 * xu + dr(xu)[..., None] * xi
    Xv = r0 * xv + dr(xv)[..., None] * xi
    return X, Xu, Xv


# ----------------------------------------------------------------------
# random smooth ambient vector fields (harmonic-field experiments)
# ----------------------------------------------------------------------
def legendre_field(x, seed, deg, L):
    """V (n, 3): each component sum_{a,b,c <= deg} C_abc P_a(x/2L) P_b(y/2L) P_c(z/2L)
    with C_abc ~ N(0, 1) (seeded), for points inside (-L, L)^3."""
    from numpy.polynomial import legendre
    x = np.asarray(x, dtype=float)
    rng = np.random.default_rng(seed)
    V = np.zeros_like(x)
    for c in range(3):
        C = rng.standard_normal((deg + 1, deg + 1, deg + 1))
        V[:, c] = legendre.legval3d(x[:, 0] / (2 * L), x[:, 1] / (2 * L), x[:, 2] / (2 * L), C)
    return V


def torus_angles(X, R):
    """(theta, phi) of points X (n, 3) on the torus of torus_patches."""
    X = np.asarray(X, dtype=float)
    ph = np.arctan2(X[:, 1], X[:, 0])
    th = np.arctan2(X[:, 2], np.hypot(X[:, 0], X[:, 1]) - R)
    return th, ph


def trig_series(theta, phi, seed, amax=6):
    """sum over |a|, |b| <= amax of c cos(a theta + b phi) + d sin(a theta + b phi),
    c, d ~ N(0, 1) / (1 + a^2 + b^2) (seeded): a random smooth periodic field."""
    rng = np.random.default_rng(seed)
    out = np.zeros_like(np.asarray(theta, dtype=float))
    for a in range(-amax, amax + 1):
        for b in range(-amax, amax + 1):
            c, d = rng.standard_normal(2) / (1.0 + a * a + b * b)
            t = a * theta + b * phi
            out += c * np.cos(t) + d * np.sin(t)
    return out


def torus_frame(X, R, r):
    """Unit tangents e_phi, e_theta and rho = R + r cos(theta) of the torus of
    torus_patches at the points X (n, 3)."""
    X = np.asarray(X, dtype=float)
    ph = np.arctan2(X[:, 1], X[:, 0])
    rho = np.hypot(X[:, 0], X[:, 1])
    th = np.arctan2(X[:, 2], rho - R)
    e_ph = np.stack([-np.sin(ph), np.cos(ph), 0 * ph], 1)
    e_th = np.stack([-np.sin(th) * np.cos(ph), -np.sin(th) * np.sin(ph), np.cos(th)], 1)
    return e_ph, e_th, R + r * np.cos(th)
