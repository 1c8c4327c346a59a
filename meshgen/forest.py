"""Octree forest over a macro-mesh: integer cells, cross-macro neighbours, 2:1 face balance.

Pure topology on integer anchors; no geometry.
"""
import itertools

import numpy as np


def orient_map_int(o, a, b, level):
    """Map integer face-cell coordinates (a, b) at ``level`` through orientation code o."""
    if o & 1:
        s, t = b, a
    else:
        s, t = a, b
    n = 1 << level
    if o & 2:
        s = n - 1 - s
    if o & 4:
        t = n - 1 - t
    return s, t


def _tangential(d):
    return [x for x in range(3) if x != d]


def face_corner_orientation(verts_a, fa, verts_b, fb):
    """Orientation code mapping face fa of hex A to face fb of hex B, from shared vertex ids.

    ``verts_*`` are the 8 vertex ids of a hex in corner order c = i + 2 j + 4 k
    (i, j, k in {0,1} for xi = -1/+1 along axes 0, 1, 2).  Returns None when the
    faces do not share their four vertices.
    """
    def face_vertex(verts, f, ca, cb):
        d, s = divmod(f, 2)
        t0, t1 = _tangential(d)
        c = [0, 0, 0]
        c[d] = s
        c[t0] = ca
        c[t1] = cb
        return verts[c[0] + 2 * c[1] + 4 * c[2]]

    for o in range(8):
        ok = True
        for ca in (0, 1):
            for cb in (0, 1):
                s, t = (cb, ca) if o & 1 else (ca, cb)
                if o & 2:
                    s = 1 - s
                if o & 4:
                    t = 1 - t
                if face_vertex(verts_a, fa, ca, cb) != face_vertex(verts_b, fb, s, t):
                    ok = False
        if ok:
            return o
    return None


def macro_connectivity(hex_vertices):
    """Face connectivity of a macro-mesh given as hexes of vertex ids.

    Returns (nbr, nbr_face, nbr_orient), each int32[M, 6]; nbr = -1 on the boundary.
    """
    M = len(hex_vertices)
    nbr = -np.ones((M, 6), np.int32)
    nface = -np.ones((M, 6), np.int32)
    nor = np.zeros((M, 6), np.int32)
    keyed = {}
    for m, v in enumerate(hex_vertices):
        for f in range(6):
            d, s = divmod(f, 2)
            corners = [v[c] for c in range(8) if ((c >> d) & 1) == s]
            keyed.setdefault(frozenset(corners), []).append((m, f))
    for lst in keyed.values():
        if len(lst) == 1:
            continue
        assert len(lst) == 2, "a face shared by more than two macro-elements"
        (ma, fa), (mb, fb) = lst
        oab = face_corner_orientation(hex_vertices[ma], fa, hex_vertices[mb], fb)
        oba = face_corner_orientation(hex_vertices[mb], fb, hex_vertices[ma], fa)
        assert oab is not None and oba is not None
        nbr[ma, fa], nface[ma, fa], nor[ma, fa] = mb, fb, oab
        nbr[mb, fb], nface[mb, fb], nor[mb, fb] = ma, fa, oba
    return nbr, nface, nor


class Forest:
    """Leaves of an octree forest keyed by (macro, level, i, j, k)."""

    def __init__(self, n_macro, nbr, nbr_face, nbr_orient):
        self.n_macro = n_macro
        self.nbr = np.asarray(nbr)
        self.nbr_face = np.asarray(nbr_face)
        self.nbr_orient = np.asarray(nbr_orient)
        self.leaves = {(m, 0, 0, 0, 0) for m in range(n_macro)}

    # -- topology -----------------------------------------------------------
    def same_level_neighbor(self, m, l, a, f):
        """Cell (m', a') at level l across face f of cell (m, l, a); None on the boundary."""
        d, s = divmod(f, 2)
        n = 1 << l
        b = list(a)
        b[d] += 1 if s else -1
        if 0 <= b[d] < n:
            return m, tuple(b)
        mb = int(self.nbr[m, f])
        if mb < 0:
            return None
        fb = int(self.nbr_face[m, f])
        o = int(self.nbr_orient[m, f])
        t0, t1 = _tangential(d)
        sa, sb = orient_map_int(o, a[t0], a[t1], l)
        db, sidb = divmod(fb, 2)
        u0, u1 = _tangential(db)
        c = [0, 0, 0]
        c[db] = 0 if sidb == 0 else n - 1
        c[u0] = sa
        c[u1] = sb
        return mb, tuple(c)

    def covering_leaf(self, m, l, a):
        """Leaf containing cell (m, l, a) (the cell itself or an ancestor), or None if refined."""
        for lev in range(l, -1, -1):
            sh = l - lev
            key = (m, lev, a[0] >> sh, a[1] >> sh, a[2] >> sh)
            if key in self.leaves:
                return key
        return None

    # -- refinement ---------------------------------------------------------
    def refine(self, key):
        m, l, i, j, k = key
        self.leaves.remove(key)
        for dz, dy, dx in itertools.product((0, 1), repeat=3):
            self.leaves.add((m, l + 1, 2 * i + dx, 2 * j + dy, 2 * k + dz))

    def refine_where(self, pred):
        """Refine every leaf for which pred(key) is true (one level)."""
        for key in [k for k in self.leaves if pred(k)]:
            self.refine(key)

    def balance(self):
        """Refine until no two face-adjacent leaves differ by more than one level."""
        changed = True
        while changed:
            changed = False
            for key in sorted(self.leaves, key=lambda k: -k[1]):
                if key not in self.leaves:
                    continue
                m, l = key[0], key[1]
                a = key[2:]
                for f in range(6):
                    nb = self.same_level_neighbor(m, l, a, f)
                    if nb is None:
                        continue
                    leaf = self.covering_leaf(nb[0], l, nb[1])
                    if leaf is not None and leaf[1] <= l - 2:
                        self.refine(leaf)
                        changed = True

    # -- export ---------------------------------------------------------------
    def element_arrays(self, p_of, order_key=None):
        """Arrays (macro, level, anchor[E,3], p) sorted by (p, macro, Morton)."""
        keys = list(self.leaves)
        lmax = max(k[1] for k in keys)

        def morton(k):
            m, l, i, j, kk = k
            sh = lmax - l
            i, j, kk = i << sh, j << sh, kk << sh
            code = 0
            for bit in range(lmax + 1):
                code |= ((i >> bit) & 1) << (3 * bit)
                code |= ((j >> bit) & 1) << (3 * bit + 1)
                code |= ((kk >> bit) & 1) << (3 * bit + 2)
            return code

        ps = {k: int(p_of(k)) for k in keys}
        if order_key is None:
            keys.sort(key=lambda k: (ps[k], k[0], morton(k)))
        else:
            keys.sort(key=lambda k: order_key(k, ps[k], morton(k)))
        macro = np.array([k[0] for k in keys], np.int32)
        level = np.array([k[1] for k in keys], np.int32)
        anchor = np.array([k[2:] for k in keys], np.int32).reshape(-1, 3)
        p = np.array([ps[k] for k in keys], np.int32)
        return macro, level, anchor, p
