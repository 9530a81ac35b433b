"""A genus-2 test surface: two tori fused where they overlap.

F(x) = T1 + T2 - sqrt(T1^2 + T2^2 + c^2),
T_i(x) = (sqrt((x1 - a_i)^2 + x2^2) - R)^2 + x3^2 - r^2,  a_i = -d, +d.
Inside a torus T_i < 0; F < 0 exactly where x lies in the union of the two
solid tori (a smoothed minimum of T1 and T2: F is close to T1 away from the
second torus), and c rounds off the crease where the two tubes meet (over a
width of order c / (2 r)).  With the rings a little more than a diameter
apart (d slightly above R) the tubes overlap in one lens, and the union has
genus 2.  Seeded bumps displace the surface along its normal by about
amp * a_b * exp(-|x - c_b|^2 / (2 width^2)), a_b ~ U(-1, 1), centres c_b on
the surface: F - 0.8 sum_b amp a_b exp(...) (0.8 ~ |grad F| = 2 r on the
tubes).

Meshing (synthetic input generation, no part of the method): marching
tetrahedra on the six-tetrahedra split of a cubic grid, vertices moved onto
F = 0 by Newton steps along grad F, then short edges collapsed, edges flipped
towards the Delaunay condition and vertices relaxed tangentially, each pass
followed by the projection.  Each final triangle (A, B, C) gets the chart
X(u, v) = proj((1 - u - v) A + u B + v C), the projection of the flat
triangle onto the surface; X_u and X_v by fourth-order central differences
of that map.  Adjacent charts agree on their common edge (the projection
depends on the 3-D point only), so the patches tile the smooth surface.
"""
import numpy as np

# the six tetrahedra of a unit cube sharing its main diagonal (0 -> 7);
# cube corners numbered by bits (x, y, z) = (i & 1, i >> 1 & 1, i >> 2 & 1)
_TETS = np.array([[0, 1, 3, 7], [0, 3, 2, 7], [0, 2, 6, 7], [0, 6, 4, 7], [0, 4, 5, 7], [0, 5, 1, 7]])


class FusedTori:
    def __init__(self, R=1.0, r=0.4, d=1.1, c=0.3, bumps=8, amp=0.05, width=0.25, seed=5):
        self.R, self.r, self.d, self.c = R, r, d, c
        self.amp, self.width = amp, width
        self.bc = np.zeros((0, 3))
        self.ba = np.zeros(0)
        if bumps:
            rng = np.random.default_rng(seed)
            lo, hi = self.bounds()
            p = lo + (hi - lo) * rng.uniform(size=(bumps, 3))
            a = rng.uniform(-1.0, 1.0, bumps)
            self.bc = self.project(p)  # centres on the surface without bumps
            self.ba = a

    def _bump(self, x):
        if len(self.ba) == 0:
            return 0.0, 0.0
        # |x - c|^2 = |x|^2 + |c|^2 - 2 x.c (a product with the few centres)
        d2 = (x * x).sum(-1)[..., None] + (self.bc * self.bc).sum(-1) - 2.0 * (x @ self.bc.T)
        e = np.exp(-np.maximum(d2, 0.0) / (2.0 * self.width ** 2)) * (0.8 * self.amp * self.ba)
        es = e.sum(-1)
        return es, -(es[..., None] * x - e @ self.bc) / self.width ** 2

    def _torus(self, x, a):
        rho = np.sqrt((x[..., 0] - a) ** 2 + x[..., 1] ** 2)
        t = (rho - self.R) ** 2 + x[..., 2] ** 2 - self.r ** 2
        f = 2.0 * (rho - self.R) / np.maximum(rho, 1e-300)
        g = np.stack([f * (x[..., 0] - a), f * x[..., 1], 2.0 * x[..., 2]], axis=-1)
        return t, g

    def F(self, x):
        t1, _ = self._torus(x, -self.d)
        t2, _ = self._torus(x, self.d)
        b, _ = self._bump(x)
        return t1 + t2 - np.sqrt(t1 * t1 + t2 * t2 + self.c * self.c) - b

    def grad(self, x):
        t1, g1 = self._torus(x, -self.d)
        t2, g2 = self._torus(x, self.d)
        q = np.sqrt(t1 * t1 + t2 * t2 + self.c * self.c)
        _, gb = self._bump(x)
        return (1.0 - t1 / q)[..., None] * g1 + (1.0 - t2 / q)[..., None] * g2 - gb

    def bounds(self):
        # F < 0 reaches beyond the tori where both T_i < c / sqrt(2) (the
        # blend), i.e. at most to the tube radius sqrt(r^2 + c / sqrt(2))
        R, d = self.R, self.d
        r = np.sqrt(self.r ** 2 + self.c / np.sqrt(2.0)) + 2.0 * self.amp
        return np.array([-d - R - r, -R - r, -r]), np.array([d + R + r, R + r, r])

    def project(self, p, iters=60):
        """Newton steps along grad F onto F = 0 (to rounding)."""
        x = np.array(p, dtype=float, copy=True)
        for it in range(iters):
            f = self.F(x)
            g = self.grad(x)
            step = f / (g * g).sum(-1)
            x -= step[..., None] * g
            if it > 3 and np.abs(step).max() * np.abs(g).max() < 1e-17:
                break
        # two more steps past convergence: the map is then smooth to rounding
        for _ in range(2):
            f = self.F(x)
            g = self.grad(x)
            x -= (f / (g * g).sum(-1))[..., None] * g
        return x


def _marching_tets(S, h):
    lo, hi = S.bounds()
    lo = lo - 1.5 * h
    hi = hi + 1.5 * h
    n = np.ceil((hi - lo) / h).astype(int) + 1
    gx, gy, gz = (lo[k] + h * np.arange(n[k]) for k in range(3))
    P = np.stack(np.meshgrid(gx, gy, gz, indexing="ij"), axis=-1)
    val = S.F(P)
    # keep lattice values away from zero (no triangle collapses to a point)
    tiny = 1e-6 * np.abs(val).max()
    val = np.where(np.abs(val) < tiny, tiny, val)
    nx, ny, nz = n
    ii, jj, kk = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1), indexing="ij")
    base = (ii * ny + jj) * nz + kk
    off = np.array([((c & 1) * ny + (c >> 1 & 1)) * nz + (c >> 2 & 1) for c in range(8)])
    corner = base.reshape(-1, 1) + off[None, :]                          # (cubes, 8) vertex ids
    flatv = val.reshape(-1)
    flatp = P.reshape(-1, 3)
    tris = []
    for tet in _TETS:
        vid = corner[:, tet]                                              # (cubes, 4)
        s = flatv[vid] < 0
        cnt = s.sum(1)
        for k in (1, 2, 3):
            sel = np.nonzero(cnt == k)[0]
            if len(sel) == 0:
                continue
            v = vid[sel]
            neg = s[sel]
            if k == 3:  # one positive corner: the mirror case of one negative
                neg = ~neg
            if k in (1, 3):
                a = np.argmax(neg, axis=1)                                # the lone corner
                others = np.array([[j for j in range(4) if j != q] for q in range(4)])[a]
                A = v[np.arange(len(v)), a]
                e = [np.stack([A, v[np.arange(len(v)), others[:, j]]], 1) for j in range(3)]
                tris.append(np.stack(e, 1))                               # (m, 3, 2) edges
            else:
                order = np.argsort(~neg, axis=1, kind="stable")          # two negatives first
                a0, a1 = v[np.arange(len(v)), order[:, 0]], v[np.arange(len(v)), order[:, 1]]
                b0, b1 = v[np.arange(len(v)), order[:, 2]], v[np.arange(len(v)), order[:, 3]]
                e00, e01 = np.stack([a0, b0], 1), np.stack([a0, b1], 1)
                e11, e10 = np.stack([a1, b1], 1), np.stack([a1, b0], 1)
                tris.append(np.stack([e00, e01, e11], 1))
                tris.append(np.stack([e00, e11, e10], 1))
    E = np.concatenate(tris)                                             # (t, 3, 2)
    key = np.sort(E, axis=2).reshape(-1, 2)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    fa, fb = flatv[uniq[:, 0]], flatv[uniq[:, 1]]
    t = fa / (fa - fb)
    V = flatp[uniq[:, 0]] + t[:, None] * (flatp[uniq[:, 1]] - flatp[uniq[:, 0]])
    T = inv.reshape(-1, 3)
    return V, T


def _orient(S, V, T):
    nrm = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    g = S.grad(V[T].mean(1))
    flip = (nrm * g).sum(1) < 0
    T = T.copy()
    T[flip] = T[flip][:, [0, 2, 1]]
    return T


def _edges(T):
    """Unique edges (a < b) and, per edge, its two triangles."""
    he = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    tri = np.tile(np.arange(len(T)), 3)
    key = np.sort(he, axis=1)
    order = np.lexsort((key[:, 1], key[:, 0]))
    key, tri = key[order], tri[order]
    assert np.all(key[0::2] == key[1::2]), "mesh is not closed and manifold"
    return key[0::2], np.stack([tri[0::2], tri[1::2]], 1)


def _collapse(S, V, T, lmin):
    E, _ = _edges(T)
    L = np.linalg.norm(V[E[:, 0]] - V[E[:, 1]], axis=1)
    cand = np.argsort(L)
    cand = cand[L[cand] < lmin]
    if len(cand) == 0:
        return V, T, 0
    # midpoints of the candidate edges on the surface, in one call (an edge
    # is collapsed only while both its ends are untouched in this pass, so
    # its midpoint stays the one computed here)
    mids = S.project(0.5 * (V[E[cand, 0]] + V[E[cand, 1]]))
    mid_of = {int(e): mids[i] for i, e in enumerate(cand)}
    vt = [[] for _ in range(len(V))]
    for t, (a, b, c) in enumerate(T):
        vt[a].append(t); vt[b].append(t); vt[c].append(t)
    alive = np.ones(len(T), bool)
    remap = np.arange(len(V))
    touched = np.zeros(len(V), bool)
    V = V.copy()
    done = 0
    for e in cand:
        a, b = E[e]
        if touched[a] or touched[b]:
            continue
        ta = [t for t in vt[a] if alive[t]]
        tb = [t for t in vt[b] if alive[t]]
        na = set(T[ta].ravel()) - {a}
        nb = set(T[tb].ravel()) - {b}
        shared = [t for t in ta if b in T[t]]
        if len(shared) != 2 or len(na & nb) != 2:
            continue                                   # link condition
        m = mid_of[int(e)]
        ok = True
        for t in set(ta) | set(tb):
            if t in shared:
                continue
            p = V[T[t]].copy()
            n0 = np.cross(p[1] - p[0], p[2] - p[0])
            p[(T[t] == a) | (T[t] == b)] = m
            n1 = np.cross(p[1] - p[0], p[2] - p[0])
            if (n0 @ n1) <= 0.2 * np.linalg.norm(n0) * np.linalg.norm(n1):
                ok = False
                break
        if not ok:
            continue
        V[a] = m
        for t in shared:
            alive[t] = False
        for t in tb:
            if alive[t]:
                T[t][T[t] == b] = a
                vt[a].append(t)
        remap[b] = a
        touched[list(na | nb | {a, b})] = True
        done += 1
    T = T[alive]
    used = np.unique(T)
    new = -np.ones(len(V), int)
    new[used] = np.arange(len(used))
    return V[used], new[T], done


def _angles(P):
    """Interior angles (m, 3) of triangles P (m, 3, 3)."""
    out = np.empty(P.shape[:2])
    for k in range(3):
        u = P[:, (k + 1) % 3] - P[:, k]
        w = P[:, (k + 2) % 3] - P[:, k]
        c = (u * w).sum(1) / (np.linalg.norm(u, axis=1) * np.linalg.norm(w, axis=1))
        out[:, k] = np.arccos(np.clip(c, -1.0, 1.0))
    return out


def _flip(S, V, T):
    E, ET = _edges(T)
    T = T.copy()
    touched = np.zeros(len(T), bool)
    eset = set(map(tuple, E))
    done = 0
    for (a, b), (t1, t2) in zip(E, ET):
        if touched[t1] or touched[t2]:
            continue
        c = [v for v in T[t1] if v != a and v != b][0]
        d = [v for v in T[t2] if v != a and v != b][0]
        if (min(c, d), max(c, d)) in eset or c == d:
            continue
        ang = lambda p, q, r: np.arccos(np.clip(((V[q] - p) @ (V[r] - p)) /
                                                (np.linalg.norm(V[q] - p) * np.linalg.norm(V[r] - p)), -1, 1))
        if ang(V[c], a, b) + ang(V[d], a, b) <= np.pi + 1e-9:
            continue
        # new triangles keep the orientation of t1: (a, b, c) order in t1
        i = list(T[t1]).index(c)
        x, y = T[t1][(i + 1) % 3], T[t1][(i + 2) % 3]       # t1 = (c, x, y), {x, y} = {a, b}
        n1 = np.array([c, x, d])
        n2 = np.array([c, d, y])
        g = S.grad(V[[c, d]].mean(0)[None])[0]
        if (np.cross(V[n1[1]] - V[n1[0]], V[n1[2]] - V[n1[0]]) @ g <= 0 or
                np.cross(V[n2[1]] - V[n2[0]], V[n2[2]] - V[n2[0]]) @ g <= 0):
            continue
        old = min(_angles(V[T[[t1, t2]]]).min(1))
        new = min(_angles(V[np.stack([n1, n2])]).min(1))
        if new <= old:
            continue
        T[t1], T[t2] = n1, n2
        touched[t1] = touched[t2] = True
        eset.discard((min(a, b), max(a, b)))
        eset.add((min(c, d), max(c, d)))
        done += 1
    return T, done


def _smooth(S, V, T, lam=0.5):
    E, _ = _edges(T)
    nb = np.zeros_like(V)
    cnt = np.zeros(len(V))
    np.add.at(nb, E[:, 0], V[E[:, 1]])
    np.add.at(nb, E[:, 1], V[E[:, 0]])
    np.add.at(cnt, E[:, 0], 1)
    np.add.at(cnt, E[:, 1], 1)
    c = nb / cnt[:, None]
    g = S.grad(V)
    n = g / np.linalg.norm(g, axis=1, keepdims=True)
    dv = c - V
    dv -= (dv * n).sum(1, keepdims=True) * n
    return S.project(V + lam * dv)


def mesh(S, h, rounds=6):
    """Triangle mesh of F = 0 with edges of about h: vertices on the surface,
    outward orientation (along grad F)."""
    V, T = _marching_tets(S, h)
    V = S.project(V)
    for _ in range(rounds):
        V, T, _ = _collapse(S, V, T, 0.45 * h)
        T = _orient(S, V, T)
        for _ in range(3):
            T, nf = _flip(S, V, T)
            if nf == 0:
                break
        V = _smooth(S, V, T)
    T = _orient(S, V, T)
    return V, T


def euler_characteristic(T):
    E, _ = _edges(T)
    return len(np.unique(T)) - len(E) + len(T)


def patches(S, V, T, uv, h=1e-4):
    """Chart samples X, X_u, X_v [n_tri][n_p][3] at the reference nodes uv:
    the projection of each flat triangle onto F = 0."""
    A, B, C = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    eu, ev = B - A, C - A
    u = uv[None, :, 0:1]
    v = uv[None, :, 1:2]
    flat = A[:, None, :] + u * eu[:, None, :] + v * ev[:, None, :]
    proj = lambda p: S.project(p.reshape(-1, 3)).reshape(p.shape)
    X = proj(flat)

    def d(e):
        s = h * e[:, None, :]
        return (-proj(flat + 2 * s) + 8 * proj(flat + s) - 8 * proj(flat - s) + proj(flat - 2 * s)) / (12 * h)

    return X, d(eu), d(ev)


def quality(V, T):
    """Smallest angle (degrees), and the ratio of the longest to the
    shortest edge."""
    ang = _angles(V[T])
    E, _ = _edges(T)
    L = np.linalg.norm(V[E[:, 0]] - V[E[:, 1]], axis=1)
    return np.degrees(ang.min()), L.max() / L.min()
