"""Additive Schwarz smoother (Sec. II.D, the Schwarz smoother: Alg. schwarz_smoother,
Eq. schwarz_weight).

Test infrastructure: only the tests, the smoke check and the CPU baseline of the benchmark use
this package.  Plain FP64 numpy on the dense operator of ``operator.assemble_dense``.

Subdomains, one per element e_c: the collocation points of e_c, the boundary points of other
elements that coincide with its faces, edges or corners, and N_overlap - 1 further layers of
points around those.  This oracle builds them for meshes of axis-aligned affine elements of one
degree and one refinement level without 2:1 faces (every neighbour of e_c meets it along a whole
face, edge or corner).  The extended coordinate of a point of a neighbour e' along axis d is
xi_ext = xi_e'(d) + 2 o_d, with xi_e' the point's reference coordinate in e' and o_d in
{-1, 0, 1} the side of e_c on which e' lies; the points of e_c keep their own coordinate.  The
subdomain holds the points with |xi_ext| <= 1 + delta on every axis, delta = 1 + xi_(N_overlap - 1)
(xi_0 = -1 < xi_1 < ... the LGL nodes): the coincident layer at |xi_ext| = 1 and N_overlap - 1
layers beyond it.  delta is also the overlap width of the weights.

Weights (Eq. schwarz_weight): w(xi) = (phi((xi + 1) / delta) - phi((xi - 1) / delta)) / 2,
phi(t) = sgn(t) for |t| > 1 and (15 t - 10 t^3 + 3 t^5) / 8 otherwise; the weight of a point is
the product of w over the three axes.  For N_overlap = 1 (delta = 0) this is the limit
w = 1 inside, 1/2 on |xi| = 1, 0 outside.  On a side of e_c that lies on the domain boundary the
falling half of w is dropped (its phi term is replaced by its limit, -1 on the upper and +1 on
the lower side): no other subdomain shares the points there, and the weights of all subdomains
then sum to one at every point.

``subdomains_topo`` builds the same subdomains from the mesh topology alone, for any macro
maps and face orientations and any degrees (one level, no 2:1 faces): a neighbour's points are
placed in e_c's extended coordinates by the composed maps of the faces crossed to reach it.
Where degrees differ across a face the subdomains are ragged; each face takes the narrower of
its two sides' overlap widths.  ``subdomains_boxes`` extends that to 2:1 faces on meshes of
axis-aligned affine boxes, with positions scaled to e_c's half-widths as the extended
coordinate (the library does not build this case yet).
On the six-patch shell three cells meet around the radial lines through the cube's corners;
there the subdomains cover three quadrants instead of four and their weights sum to 3/4, so
they are divided by their sum wherever it is not one.

Local solves: R_s A R_s^T d_s = R_s r solved exactly by default (the limit of the paper's
iteration, which keeps the smoother linear), or as the paper does, by CG from zero to a
relative residual of 1e-3 (``local="cg"``).

Smoother: N_iter times r = b - A x, x <- x + sum_s R_s^T W_s d_s.
"""
import itertools

import numpy as np

from . import geometry, rules
from .mesh import neighbor_cell, tangential_axes


def phi(t):
    t = np.asarray(t, float)
    return np.where(np.abs(t) > 1.0, np.sign(t), (15.0 * t - 10.0 * t ** 3 + 3.0 * t ** 5) / 8.0)


def weight_sides(xi, delta_lo, delta_hi, lower_open=True, upper_open=True):
    """w(xi) of Eq. schwarz_weight with the overlap width delta_lo on the lower and delta_hi on the
    upper side (a width 0: the step limit, one half on the face).  A side that is not open (a
    domain-boundary side) keeps the weight at its plateau."""
    xi = np.asarray(xi, float)

    def edge(t, delta):
        return np.sign(t) if delta == 0.0 else phi(t / delta)
    a = edge(xi + 1.0, delta_lo) if lower_open else np.ones_like(xi)
    b = edge(xi - 1.0, delta_hi) if upper_open else -np.ones_like(xi)
    return 0.5 * (a - b)


def weight_1d(xi, delta, lower_open=True, upper_open=True):
    """w(xi) of Eq. schwarz_weight with overlap width delta (delta = 0: the step limit)."""
    return weight_sides(xi, delta, delta, lower_open, upper_open)


def overlap_width(n, n_overlap):
    """delta = 1 + xi_(N_overlap - 1) for the n LGL nodes of the degree (0 for N_overlap = 1)."""
    if not 1 <= n_overlap <= n - 1:
        raise ValueError("N_overlap must lie in [1, n - 1]")
    x, _ = rules.lgl(n)
    return 1.0 + x[n_overlap - 1]


def _boxes(mesh):
    """Centre and half-widths of every element; refuses meshes outside the scope above."""
    E = len(mesh["elem_p"])
    if len(set(int(p) for p in mesh["elem_p"])) != 1 or len(set(int(l) for l in mesh["elem_level"])) != 1:
        raise ValueError("the Schwarz subdomains here need one degree and one level")
    x0, J = geometry.element_map(mesh, np.arange(E)[:, None], np.zeros((1, 3)))
    J = J[:, 0]
    diag = np.einsum("eii->ei", J)
    if np.abs(J - diag[:, :, None] * np.eye(3)[None]).max() > 1e-12 * np.abs(J).max() or diag.min() <= 0:
        raise ValueError("the Schwarz subdomains here need axis-aligned affine elements")
    return x0[:, 0], diag


def _neighbours(centre, half, c):
    """Elements touching e_c (closures meet) and their side o in {-1, 0, 1}^3; refuses a
    neighbour that does not meet e_c along a whole face, edge or corner."""
    out = []
    tol = 1e-10 * half[c].min()
    for e in range(len(centre)):
        if e == c:
            continue
        gap = np.abs(centre[e] - centre[c]) - (half[e] + half[c])
        if np.any(gap > tol):
            continue
        o = np.zeros(3, int)
        for d in range(3):
            dc = centre[e, d] - centre[c, d]
            if abs(dc) <= tol:
                if abs(half[e, d] - half[c, d]) > tol:
                    raise ValueError("a neighbour that overlaps e_c only in part")
            else:
                o[d] = 1 if dc > 0 else -1
                if abs(gap[d]) > tol:
                    raise ValueError("overlapping elements")
        out.append((e, o))
    return out


def subdomains(op, n_overlap, centres=None):
    """Per element (mesh order, or the elements ``centres``): (global dof indices, weights) of
    its subdomain, own points first in the element's dof order, then the neighbours' points by
    element and dof order."""
    mesh = op.mesh
    n = int(mesh["elem_p"][0]) + 1
    delta = overlap_width(n, n_overlap)
    centre, half = _boxes(mesh)
    xl, _ = rules.lgl(n)
    xi = np.stack(np.meshgrid(xl, xl, xl, indexing="ij")[::-1], axis=-1).reshape(-1, 3)  # x fastest
    out = []
    for c in (range(len(mesh["elem_p"])) if centres is None else centres):
        nb = _neighbours(centre, half, int(c))
        open_lo = [any(o[d] == -1 and not np.any(np.delete(o, d)) for _, o in nb) for d in range(3)]
        open_hi = [any(o[d] == 1 and not np.any(np.delete(o, d)) for _, o in nb) for d in range(3)]
        idx, wts = [], []
        for e, o in [(c, np.zeros(3, int))] + nb:
            ext = xi + 2.0 * o[None, :]
            inside = np.all(np.abs(ext) <= 1.0 + delta + 1e-12, axis=1)
            if not inside.any():
                continue
            w = np.ones(int(inside.sum()))
            for d in range(3):
                w = w * weight_1d(ext[inside, d], delta, open_lo[d], open_hi[d])
            idx.append(op.offsets[e] + np.flatnonzero(inside))
            wts.append(w)
        out.append((np.concatenate(idx), np.concatenate(wts)))
    return out


def _face_map(f, fb, o):
    """Affine map of the reference coordinates of the neighbour across face f of an element
    (its face fb, orientation o: swap | flip of the first | flip of the second face axis, from
    this face's coordinates to the neighbour's) into this element's extended coordinates:
    ext[i] = sign[i] xi_nb[perm[i]] + shift[i].  The shared face lies at ext[d] = +-1."""
    d, s = divmod(f, 2)
    db, sb = divmod(fb, 2)
    t0, t1 = tangential_axes(d)
    u0, u1 = tangential_axes(db)
    sc, sn = (1 if s else -1), (1 if sb else -1)
    perm, sign, shift = [0, 0, 0], [1.0, 1.0, 1.0], [0.0, 0.0, 0.0]
    perm[d], sign[d], shift[d] = db, float(-sc * sn), 2.0 * sc
    a0, a1 = (t1, t0) if o & 1 else (t0, t1)  # own axes carrying the neighbour's u0, u1
    perm[a0], sign[a0] = u0, (-1.0 if o & 2 else 1.0)
    perm[a1], sign[a1] = u1, (-1.0 if o & 4 else 1.0)
    return perm, sign, shift


def _compose(m1, m2):
    """m1 after m2 (both as in _face_map)."""
    p1, s1, h1 = m1
    p2, s2, h2 = m2
    return ([p2[p1[i]] for i in range(3)], [s1[i] * s2[p1[i]] for i in range(3)],
            [s1[i] * h2[p1[i]] + h1[i] for i in range(3)])


def _topo_neighbours(mesh, index, c):
    """Face, edge and corner neighbours of element c as (element, map into c's extended
    coordinates), found by stepping across faces in every order of the offset's axes.  An
    offset whose orders disagree, or that leads back to c or to one of its face neighbours (a
    vertex where three cells meet instead of four), has no neighbour."""
    lev = int(mesh["elem_level"][c])

    def across(e, f):
        r = neighbor_cell(mesh, int(mesh["elem_macro"][e]), lev, tuple(int(x) for x in mesh["elem_anchor"][e]), f)
        if r is None:
            return None
        mb, anc, fb, o = r
        return index[(mb, lev) + tuple(anc)], fb, o

    ident = ([0, 1, 2], [1.0, 1.0, 1.0], [0.0, 0.0, 0.0])
    found = {}
    for off in itertools.product((-1, 0, 1), repeat=3):
        axes = [a for a in range(3) if off[a]]
        if not axes:
            continue
        results = set()
        for order in itertools.permutations(axes):
            e, M = c, ident
            for a in order:
                j = M[0][a]
                face = 2 * j + (1 if off[a] * M[1][a] > 0 else 0)
                r = across(e, face)
                if r is None:
                    e = None
                    break
                e, fb, o = r[0], r[1], r[2]
                M = _compose(M, _face_map(face, fb, o))
            if e is None:
                continue
            if [float(2 * x) for x in off] != M[2]:
                results.add(None)
            else:
                results.add((e, tuple(M[0]), tuple(M[1])))
        if len(results) == 1 and None not in results:
            (e, perm, sign), = results
            found[off] = (e, (list(perm), list(sign), [2.0 * x for x in off]))
    faces = {found[o][0] for o in found if sum(map(abs, o)) == 1}
    out = []
    for off in sorted(found, key=lambda o: found[o][0]):
        e = found[off][0]
        if e == c or (sum(map(abs, off)) > 1 and e in faces):
            continue
        out.append((e, np.array(off), found[off][1]))
    if len({e for e, _, _ in out}) != len(out):
        raise ValueError("an element neighbours the centre on two sides")
    return out


def subdomains_topo(op, n_overlap, normalise=True):
    """Subdomains of every element built from the mesh topology (any macro maps and face
    orientations; one level, any degrees): neighbours' points placed in e_c's extended
    coordinates through the composed face maps, weights as in ``subdomains``.  With degrees that
    differ across a face the subdomain boundaries are ragged: each face of e_c has one overlap
    width, the narrower of its two sides' (delta of a degree p: 1 + xi_(N_overlap - 1) of its LGL
    nodes, N_overlap at most p), so that the two subdomains sharing the face use the same
    transition; a neighbour's point belongs to the subdomain when it lies within the overlap
    width of the side it is on, on every axis.  Where the weights of the subdomains covering a
    point do not sum to one (three cells around an edge, or degrees that differ around an edge)
    they are divided by their sum (``normalise``)."""
    mesh = op.mesh
    if len(set(int(l) for l in mesh["elem_level"])) != 1:
        raise ValueError("the Schwarz subdomains here need one refinement level")
    E = len(mesh["elem_p"])
    nodes = {}
    for p in set(int(p) for p in mesh["elem_p"]):
        xl, _ = rules.lgl(p + 1)
        xi = np.stack(np.meshgrid(xl, xl, xl, indexing="ij")[::-1], axis=-1).reshape(-1, 3)  # x fastest
        nodes[p] = (xi, overlap_width(p + 1, min(n_overlap, p)))
    index = {(int(mesh["elem_macro"][e]), int(mesh["elem_level"][e])) + tuple(int(x) for x in mesh["elem_anchor"][e]): e
             for e in range(E)}
    out = []
    for c in range(E):
        nb = _topo_neighbours(mesh, index, c)
        dc = nodes[int(mesh["elem_p"][c])][1]
        open_lo, open_hi, d_lo, d_hi = [False] * 3, [False] * 3, [0.0] * 3, [0.0] * 3
        for e, o, _ in nb:
            if sum(map(abs, o)) != 1:
                continue
            d = int(np.flatnonzero(o)[0])
            width = min(dc, nodes[int(mesh["elem_p"][e])][1])
            if o[d] < 0:
                open_lo[d], d_lo[d] = True, width
            else:
                open_hi[d], d_hi[d] = True, width
        idx, wts = [], []
        ident = ([0, 1, 2], [1.0, 1.0, 1.0], [0.0, 0.0, 0.0])
        for e, _, (perm, sign, shift) in [(c, None, ident)] + nb:
            xi = nodes[int(mesh["elem_p"][e])][0]
            ext = np.stack([sign[i] * xi[:, perm[i]] + shift[i] for i in range(3)], axis=1)
            bound = np.where(ext > 1.0, 1.0 + np.array(d_hi), np.where(ext < -1.0, 1.0 + np.array(d_lo), 1.0))
            inside = np.all(np.abs(ext) <= bound + 1e-12, axis=1)
            if not inside.any():
                continue
            w = np.ones(int(inside.sum()))
            for d in range(3):
                w = w * weight_sides(ext[inside, d], d_lo[d], d_hi[d], open_lo[d], open_hi[d])
            idx.append(op.offsets[e] + np.flatnonzero(inside))
            wts.append(w)
        out.append((np.concatenate(idx), np.concatenate(wts)))
    if normalise:
        total = np.zeros(op.ndof)
        for idx, w in out:
            np.add.at(total, idx, w)
        fix = np.abs(total - 1.0) > 1e-12
        if fix.any():
            out = [(idx, np.where(fix[idx], w / np.where(fix[idx], total[idx], 1.0), w)) for idx, w in out]
    return out


def subdomains_boxes(op, n_overlap, normalise=True):
    """Subdomains on meshes of axis-aligned affine boxes of any levels and degrees (2:1 faces
    included), from positions: the extended coordinate of a point is its offset from e_c's
    centre in units of e_c's half-widths (the macro reference coordinate of the paper's
    definition, scaled to e_c).  The overlap width of a cell of degree p and half-width h is
    delta_p h (delta_p = 1 + xi_(N_overlap - 1) of its LGL nodes, N_overlap at most p); each side
    of e_c takes the narrowest width, in e_c's units, of e_c and the cells touching that side
    across a face; a point of a neighbouring cell (closures touching) belongs to the subdomain
    when it lies within the width of the side it is on, on every axis.  Weights as in
    ``subdomains_topo``, normalised where they do not sum to one."""
    mesh = op.mesh
    E = len(mesh["elem_p"])
    x0, J = geometry.element_map(mesh, np.arange(E)[:, None], np.zeros((1, 3)))
    centre, J = x0[:, 0], J[:, 0]
    half = np.einsum("eii->ei", J)
    if np.abs(J - half[:, :, None] * np.eye(3)[None]).max() > 1e-12 * np.abs(J).max() or half.min() <= 0:
        raise ValueError("these subdomains need axis-aligned affine elements")
    nodes = {}
    for p in set(int(p) for p in mesh["elem_p"]):
        xl, _ = rules.lgl(p + 1)
        xi = np.stack(np.meshgrid(xl, xl, xl, indexing="ij")[::-1], axis=-1).reshape(-1, 3)  # x fastest
        nodes[p] = (xi, overlap_width(p + 1, min(n_overlap, p)))
    tol = 1e-10 * half.min()
    out = []
    for c in range(E):
        gap = np.abs(centre - centre[c]) - (half + half[c])
        touch = np.flatnonzero(np.all(gap <= tol, axis=1))
        touch = touch[touch != c]
        d_lo, d_hi = [0.0] * 3, [0.0] * 3
        open_lo, open_hi = [False] * 3, [False] * 3
        dc = nodes[int(mesh["elem_p"][c])][1]
        for e in touch:
            # across a face of e_c: touching along d, overlapping with positive extent on the others
            for d in range(3):
                t = [a for a in range(3) if a != d]
                if abs(gap[e, d]) > tol or np.any(gap[e, t] > -tol):
                    continue
                width = min(dc, nodes[int(mesh["elem_p"][e])][1] * half[e, d] / half[c, d])
                if centre[e, d] < centre[c, d]:
                    d_lo[d] = width if not open_lo[d] else min(d_lo[d], width)
                    open_lo[d] = True
                else:
                    d_hi[d] = width if not open_hi[d] else min(d_hi[d], width)
                    open_hi[d] = True
        idx, wts = [], []
        for e in [c] + sorted(int(e) for e in touch):
            xi = nodes[int(mesh["elem_p"][e])][0]
            ext = (centre[e] + half[e] * xi - centre[c]) / half[c]
            ext = np.where(np.abs(np.abs(ext) - 1.0) <= 1e-12, np.sign(ext), ext)  # points on e_c's faces
            bound = np.where(ext > 1.0, 1.0 + np.array(d_hi), np.where(ext < -1.0, 1.0 + np.array(d_lo), 1.0))
            inside = np.all(np.abs(ext) <= bound + 1e-12, axis=1)
            if not inside.any():
                continue
            w = np.ones(int(inside.sum()))
            for d in range(3):
                w = w * weight_sides(ext[inside, d], d_lo[d], d_hi[d], open_lo[d], open_hi[d])
            idx.append(op.offsets[e] + np.flatnonzero(inside))
            wts.append(w)
        out.append((np.concatenate(idx), np.concatenate(wts)))
    if normalise:
        total = np.zeros(op.ndof)
        for idx, w in out:
            np.add.at(total, idx, w)
        fix = np.abs(total - 1.0) > 1e-12
        if fix.any():
            out = [(idx, np.where(fix[idx], w / np.where(fix[idx], total[idx], 1.0), w)) for idx, w in out]
    return out


def local_cg(As, rs, rtol=1e-3, max_iter=1000):
    """Plain CG on the subdomain system As d = rs from d = 0 until |rs - As d| <= rtol |rs|."""
    d = np.zeros_like(rs)
    r = rs.copy()
    nr0 = np.linalg.norm(rs)
    if nr0 == 0.0:
        return d
    p = r.copy()
    rr = r @ r
    for _ in range(max_iter):
        if np.sqrt(rr) <= rtol * nr0:
            break
        q = As @ p
        alpha = rr / (p @ q)
        d += alpha * p
        r -= alpha * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    return d


def smooth(A, subs, b, x, n_iter, local="exact", rtol=1e-3):
    """Alg. schwarz_smoother on the dense operator A with exact local solves (``local="exact"``)
    or CG to the relative tolerance ``rtol`` (``local="cg"``)."""
    x = np.array(x, float, copy=True)
    if local == "exact":
        blocks = [(idx, w, np.linalg.inv(A[np.ix_(idx, idx)])) for idx, w in subs]
        solve = lambda blk, rs: blk @ rs
    elif local == "cg":
        blocks = [(idx, w, A[np.ix_(idx, idx)]) for idx, w in subs]
        solve = lambda blk, rs: local_cg(blk, rs, rtol)
    else:
        raise ValueError("local must be 'exact' or 'cg'")
    for _ in range(n_iter):
        r = b - A @ x
        dx = np.zeros_like(x)
        for idx, w, blk in blocks:
            np.add.at(dx, idx, w * solve(blk, r[idx]))
        x = x + dx
    return x
