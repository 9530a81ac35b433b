"""Uniform-depth octree of the point FMM (TEST INFRASTRUCTURE ONLY).

The paper leaves the tree to the point FMM it calls for the far sums of
Section 4; the tree checked here is the plain uniform one: a root cube
around all points, leaves on one level, points ordered by the Morton (Z)
order of their leaf with ties kept in input order, U-lists (adjacent leaves)
and V-lists (children of the parent's neighbours that are not adjacent).

Everything is written from those definitions with integer cell
coordinates; the Morton key is built bit by bit.  Only tests may import
this module.
"""
import numpy as np

BITS = 21


def frame(points):
    """Root cube (lo, side) from the bounding box, slightly enlarged."""
    mn = points.min(axis=0)
    mx = points.max(axis=0)
    side = float(np.max(mx - mn)) * (1.0 + 1e-6) + 1e-12
    lo = 0.5 * (mn + mx) - 0.5 * side
    return lo, side


def cells(points, lo, side):
    """Integer cell coordinates on the finest (2^21) grid."""
    scale = float(2 ** BITS) / side
    t = np.floor((points - lo[None, :]) * scale)
    return np.clip(t, 0.0, float(2 ** BITS - 1)).astype(np.int64)


def morton(c):
    """Morton key of integer coordinates c (n, 3): bit b of x, y, z goes to
    bits 3b, 3b+1, 3b+2."""
    c = np.asarray(c, dtype=np.int64)
    key = np.zeros(c.shape[0], dtype=np.int64)
    for b in range(BITS):
        for a in range(3):
            key |= ((c[:, a] >> b) & 1) << (3 * b + a)
    return key


def auto_depth(src_cells, leaf_src, min_leaf_side, side):
    """First level >= 2 with (sources / non-empty source leaves) <= leaf_src,
    then coarsened while the leaf side is <= min_leaf_side."""
    ns = src_cells.shape[0]
    depth = 2
    for l in range(2, 21):
        depth = l
        nocc = len(np.unique(morton(src_cells >> (BITS - l))))
        if nocc > 0 and ns / nocc <= leaf_src:
            break
    while depth > 1 and side / 2 ** depth <= min_leaf_side:
        depth -= 1
    return depth


class Tree:
    """Uniform tree of the given depth over targets and sources (n, 3)."""

    def __init__(self, tgt, src, depth):
        self.lo, self.side = frame(np.concatenate([tgt, src]))
        self.depth = depth
        ct = cells(tgt, self.lo, self.side) >> (BITS - depth)
        cs = cells(src, self.lo, self.side) >> (BITS - depth)
        kt, ks = morton(ct), morton(cs)
        self.tgt_perm = np.argsort(kt, kind="stable")
        self.src_perm = np.argsort(ks, kind="stable")
        kt_s, ks_s = kt[self.tgt_perm], ks[self.src_perm]
        # boxes per level, Morton order, numbered level by level
        self.levels = []        # per level: (keys, integer coords)
        occ = np.unique(np.concatenate([ct, cs]), axis=0)
        for l in range(depth, -1, -1):
            c = np.unique(occ >> (depth - l), axis=0)
            k = morton(c)
            o = np.argsort(k)
            self.levels.append((k[o], c[o]))
        self.levels.reverse()
        self.off = np.cumsum([0] + [len(k) for k, _ in self.levels])
        self.index = [{tuple(c): self.off[l] + i for i, c in enumerate(cl)} for l, (_, cl) in enumerate(self.levels)]
        nb = self.off[-1]
        lk = self.levels[depth][0]
        self.leaf_ranges = np.stack([np.searchsorted(kt_s, lk, "left"), np.searchsorted(kt_s, lk, "right"),
                                     np.searchsorted(ks_s, lk, "left"), np.searchsorted(ks_s, lk, "right")], 1)
        # holds targets / sources: a box holds a point iff it contains its leaf
        self.has_t = np.zeros(nb, bool)
        self.has_s = np.zeros(nb, bool)
        for l, (_, cl) in enumerate(self.levels):
            occ_t = {tuple(c) for c in np.unique(ct >> (depth - l), axis=0)}
            occ_s = {tuple(c) for c in np.unique(cs >> (depth - l), axis=0)}
            for i, c in enumerate(cl):
                self.has_t[self.off[l] + i] = tuple(c) in occ_t
                self.has_s[self.off[l] + i] = tuple(c) in occ_s
        self.boxes = np.zeros((nb, 5), np.int32)
        for l, (_, cl) in enumerate(self.levels):
            for i, c in enumerate(cl):
                g = self.off[l] + i
                self.boxes[g] = (l, c[0], c[1], c[2], int(self.has_t[g]) | 2 * int(self.has_s[g]))
        self._lists()

    def box(self, l, c):
        return self.index[l].get(tuple(int(v) for v in c), -1)

    def _lists(self):
        d = self.depth
        nleaf = len(self.levels[d][0])
        steps = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)]
        uptr, ul = [0], []
        for b, c in enumerate(self.levels[d][1]):
            if self.has_t[self.off[d] + b]:
                for s in steps:
                    n = self.box(d, c + np.array(s))
                    if n >= 0 and self.has_s[n]:
                        ul.append(n - self.off[d])
            uptr.append(len(ul))
        self.ulist_ptr, self.ulist = np.array(uptr), np.array(ul, dtype=np.int64)
        vptr, vs, vo = [0], [], []
        for l, (_, cl) in enumerate(self.levels):
            for i, c in enumerate(cl):
                g = self.off[l] + i
                if l >= 2 and self.has_t[g]:
                    pc = c >> 1
                    for s in steps:
                        pn = self.box(l - 1, pc + np.array(s))
                        if pn < 0:
                            continue
                        pcell = self.levels[l - 1][1][pn - self.off[l - 1]]
                        for o in range(8):
                            cc = 2 * pcell + np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1])
                            ch = self.box(l, cc)
                            if ch < 0 or not self.has_s[ch]:
                                continue
                            off = c - cc
                            if np.all(np.abs(off) <= 1):
                                continue
                            vs.append(ch)
                            vo.append(((off[0] + 3) * 7 + (off[1] + 3)) * 7 + (off[2] + 3))
                vptr.append(len(vs))
        self.vlist_ptr = np.array(vptr)
        self.vlist_src = np.array(vs, dtype=np.int64)
        self.vlist_off = np.array(vo, dtype=np.int64)
