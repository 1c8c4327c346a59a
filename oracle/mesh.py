"""Mortar decomposition of a fine mesh and the multigrid mesh hierarchy.

Sec. II.A.1: the mortar Gamma splits into mortar elements, each touching at most two
elements; at most 2:1 refinement across a face.  Sec. II.D.3 (Multigrid Meshes):
coarse meshes by naive h-coarsening of complete sibling families (the surrogate),
then refinement where the surrogate violates 2:1; coarse degree = min over the
children; an element that is not coarsened keeps its degree.

A "cell mesh" here is a dict with the macro arrays of the neutral mesh format and
element arrays elem_macro, elem_level, elem_anchor, elem_p.
"""
import itertools

import numpy as np

MACRO_KEYS = ("macro_kind", "macro_params", "macro_nbr", "macro_nbr_face",
              "macro_nbr_orient", "macro_bc")


def tangential_axes(d):
    return [a for a in range(3) if a != d]


def neighbor_cell(mesh, m, l, a, f):
    """Same-level cell across face f: (macro, anchor, face seen from it, orientation) or None."""
    d, s = divmod(f, 2)
    n = 1 << l
    b = list(a)
    b[d] += 1 if s else -1
    if 0 <= b[d] < n:
        return m, tuple(b), f ^ 1, 0
    mb = int(mesh["macro_nbr"][m, f])
    if mb < 0:
        return None
    fb = int(mesh["macro_nbr_face"][m, f])
    o = int(mesh["macro_nbr_orient"][m, f])
    t0, t1 = tangential_axes(d)
    s_, t_ = (a[t1], a[t0]) if o & 1 else (a[t0], a[t1])
    if o & 2:
        s_ = n - 1 - s_
    if o & 4:
        t_ = n - 1 - t_
    db, sb = divmod(fb, 2)
    u0, u1 = tangential_axes(db)
    c = [0, 0, 0]
    c[db] = 0 if sb == 0 else n - 1
    c[u0], c[u1] = s_, t_
    return mb, tuple(c), fb, o


def build_mortars(mesh):
    """List the mortar elements of a cell mesh.

    Each mortar is a dict: minus side (em, fm) = the finer element (equal levels: the
    lower index); plus side (ep, fp) with orientation ``o`` from minus to plus face
    coordinates and ``sub`` = (ia, ib) position of the minus face inside the coarser
    plus face (None when both faces coincide); ``bc`` = boundary kind (0 interior).
    """
    macro, level, anchor = mesh["elem_macro"], mesh["elem_level"], mesh["elem_anchor"]
    index = {(int(macro[e]), int(level[e])) + tuple(int(x) for x in anchor[e]): e
             for e in range(len(macro))}
    mortars = []
    for e in range(len(macro)):
        m, l = int(macro[e]), int(level[e])
        a = tuple(int(x) for x in anchor[e])
        for f in range(6):
            nb = neighbor_cell(mesh, m, l, a, f)
            if nb is None:
                mortars.append(dict(em=e, fm=f, ep=-1, fp=-1, o=0, sub=None,
                                    bc=int(mesh["macro_bc"][m, f])))
                continue
            mb, ab, fb, o = nb
            e2 = index.get((mb, l) + ab)
            if e2 is not None:
                if e < e2:
                    mortars.append(dict(em=e, fm=f, ep=e2, fp=fb, o=o, sub=None, bc=0))
                continue
            if l > 0:
                e2 = index.get((mb, l - 1) + tuple(x >> 1 for x in ab))
                if e2 is not None:
                    u0, u1 = tangential_axes(fb // 2)
                    mortars.append(dict(em=e, fm=f, ep=e2, fp=fb, o=o,
                                        sub=(ab[u0] & 1, ab[u1] & 1), bc=0))
                    continue
            # the neighbour cell is refined: its children own these mortars; check 2:1
            db = fb // 2
            kids = 0
            for bits in itertools.product((0, 1), repeat=3):
                c = tuple(2 * ab[i] + bits[i] for i in range(3))
                side = (fb % 2)
                if bits[db] != side:
                    continue
                if (mb, l + 1) + c in index:
                    kids += 1
            if kids != 4:
                raise ValueError("mesh is not 2:1 balanced at element %d face %d" % (e, f))
    return mortars


def minus_to_plus(mt, s, t):
    """Plus-side face coordinates of the mortar point with minus-side face coordinates (s, t)."""
    o = mt["o"]
    a, b = (t, s) if o & 1 else (s, t)
    if o & 2:
        a = -a
    if o & 4:
        b = -b
    if mt["sub"] is not None:
        ia, ib = mt["sub"]
        a = 0.5 * (a + 2 * ia - 1)
        b = 0.5 * (b + 2 * ib - 1)
    return a, b


def face_point(f, a, b):
    """Reference-cube point on face f with face coordinates (a, b)."""
    d, s = divmod(f, 2)
    t0, t1 = tangential_axes(d)
    a = np.asarray(a, float)
    xi = np.zeros(a.shape + (3,))
    xi[..., d] = 1.0 if s else -1.0
    xi[..., t0] = a
    xi[..., t1] = b
    return xi


# -- multigrid hierarchy ---------------------------------------------------------

def _cells(mesh):
    return {(int(mesh["elem_macro"][e]), int(mesh["elem_level"][e]))
            + tuple(int(x) for x in mesh["elem_anchor"][e]): int(mesh["elem_p"][e])
            for e in range(len(mesh["elem_p"]))}


def _leaf_covering(cells, m, l, a):
    for lev in range(l, -1, -1):
        sh = l - lev
        key = (m, lev, a[0] >> sh, a[1] >> sh, a[2] >> sh)
        if key in cells:
            return key
    return None


def coarsen(mesh):
    """One multigrid coarsening step (surrogate + 2:1 restoration); returns a cell mesh or None.

    None means no sibling family could be coarsened (the mesh is the macro-mesh or
    cannot be coarsened further).
    """
    cells = _cells(mesh)
    fam = {}
    for key in cells:
        m, l = key[0], key[1]
        if l == 0:
            continue
        parent = (m, l - 1, key[2] >> 1, key[3] >> 1, key[4] >> 1)
        fam.setdefault(parent, []).append(key)
    new = {}
    coarsened = set()
    for parent, kids in fam.items():
        if len(kids) == 8:
            new[parent] = min(cells[k] for k in kids)
            coarsened.update(kids)
    if not new:
        return None
    for key, p in cells.items():
        if key not in coarsened:
            new[key] = p
    # restore 2:1 face balance by refining too-coarse leaves (children keep the degree)
    changed = True
    while changed:
        changed = False
        for key in sorted(new, key=lambda k: -k[1]):
            if key not in new:
                continue
            m, l = key[0], key[1]
            for f in range(6):
                nb = neighbor_cell(mesh, m, l, key[2:], f)
                if nb is None:
                    continue
                leaf = _leaf_covering(new, nb[0], l, nb[1])
                if leaf is not None and leaf[1] <= l - 2:
                    p = new.pop(leaf)
                    lm, ll, i, j, k = leaf
                    for bz, by, bx in itertools.product((0, 1), repeat=3):
                        new[(lm, ll + 1, 2 * i + bx, 2 * j + by, 2 * k + bz)] = p
                    changed = True
    if set(new) == set(cells):
        return None
    keys = sorted(new, key=lambda k: (new[k], k[0], k[1], k[2:]))
    out = {k: mesh[k] for k in MACRO_KEYS}
    out["elem_macro"] = np.array([k[0] for k in keys], np.int32)
    out["elem_level"] = np.array([k[1] for k in keys], np.int32)
    out["elem_anchor"] = np.array([k[2:] for k in keys], np.int32).reshape(-1, 3)
    out["elem_p"] = np.array([new[k] for k in keys], np.int32)
    return out


def hierarchy(mesh, max_levels=32):
    """Meshes from fine (index 0) to coarsest (last), by repeated coarsening."""
    levels = [mesh]
    while len(levels) < max_levels:
        c = coarsen(levels[-1])
        if c is None:
            break
        levels.append(c)
    return levels


def parent_map(fine, coarse):
    """For each fine element: (coarse element, child bits (3,) or None when the cell is identical)."""
    index = {(int(coarse["elem_macro"][e]), int(coarse["elem_level"][e]))
             + tuple(int(x) for x in coarse["elem_anchor"][e]): e
             for e in range(len(coarse["elem_p"]))}
    out = []
    for e in range(len(fine["elem_p"])):
        m, l = int(fine["elem_macro"][e]), int(fine["elem_level"][e])
        a = tuple(int(x) for x in fine["elem_anchor"][e])
        K = index.get((m, l) + a)
        if K is not None:
            out.append((K, None))
            continue
        K = index.get((m, l - 1) + tuple(x >> 1 for x in a))
        if K is None:
            raise ValueError("fine element %d has no coarse cell one level up" % e)
        out.append((K, tuple(x & 1 for x in a)))
    return out
