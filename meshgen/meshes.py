"""Macro-meshes and refinement recipes for the synthetic workloads."""
import itertools

import numpy as np

from .forest import Forest, macro_connectivity

AFFINE, SHELL, CUBE_SPHERE = 0, 1, 2
BC_INTERIOR, BC_DIRICHLET, BC_NEUMANN, BC_ROBIN = 0, 1, 2, 3

# Rotation frames of the six cubed-sphere patches: columns are the images of the
# patch axes (xi0, xi1, outward); all have determinant +1.
SHELL_FRAMES = [
    np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]]),    # +x
    np.array([[0, 0, -1], [0, 1, 0], [1, 0, 0]]),   # -x
    np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]]),    # +y
    np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]]),   # -y
    np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1]]),    # +z
    np.array([[1, 0, 0], [0, -1, 0], [0, 0, -1]]),  # -z
]


def _finish(macro_kind, macro_params, hexes, bc_of, forest, p_of, meta, order_key=None):
    nbr, nface, nor = macro_connectivity(hexes)
    M = len(hexes)
    bc = np.zeros((M, 6), np.int32)
    for m in range(M):
        for f in range(6):
            if nbr[m, f] < 0:
                bc[m, f] = bc_of(m, f)
    macro, level, anchor, p = forest.element_arrays(p_of, order_key)
    mesh = dict(
        macro_kind=np.asarray(macro_kind, np.int32),
        macro_params=np.asarray(macro_params, np.float64).reshape(M, 16),
        macro_nbr=nbr, macro_nbr_face=nface, macro_nbr_orient=nor, macro_bc=bc,
        elem_macro=macro, elem_level=level, elem_anchor=anchor, elem_p=p,
    )
    mesh.update(meta)
    return mesh


def _forest_for(hexes):
    nbr, nface, nor = macro_connectivity(hexes)
    return Forest(len(hexes), nbr, nface, nor)


def box_grid(macros=(1, 1, 1), level=0, p=3, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
             bc=BC_DIRICHLET, p_of=None, refine=None, perturb=None):
    """Box [lo, hi] tiled by Mx*My*Mz affine macros, each refined uniformly to ``level``.

    ``p_of(key)`` overrides the constant degree; ``refine`` is a list of predicates
    (key, cell bounds) -> bool applied one level at a time, followed by 2:1 balance.
    ``perturb`` (optional dict vertex -> displacement) makes macros non-rectangular
    parallelepipeds (still affine).
    """
    Mx, My, Mz = macros
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    h = (hi - lo) / np.array([Mx, My, Mz])
    hexes, kinds, params, mpos = [], [], [], []
    for k, j, i in itertools.product(range(Mz), range(My), range(Mx)):
        v = [(i + c % 2, j + (c >> 1) % 2, k + (c >> 2)) for c in range(8)]
        hexes.append(v)
        o = lo + h * np.array([i, j, k])
        a = np.diag(h)
        par = np.zeros(16)
        par[0:3] = o
        par[3:6], par[6:9], par[9:12] = a[0], a[1], a[2]
        kinds.append(AFFINE)
        params.append(par)
        mpos.append((i, j, k))
    forest = _forest_for(hexes)
    for _ in range(level):
        forest.refine_where(lambda key: True)

    def bounds(key):
        m, l, ii, jj, kk = key
        n = 1 << l
        o = lo + h * np.array(mpos[m])
        c0 = o + h * np.array([ii, jj, kk]) / n
        return c0, c0 + h / n

    for pred in (refine or []):
        forest.refine_where(lambda key: pred(key, *bounds(key)))
        forest.balance()
    pf = p_of if p_of is not None else (lambda key: p)
    return _finish(kinds, params, hexes, lambda m, f: bc, forest, pf,
                   dict(name="box", cell_bounds=None))


def star_mesh(level=2, p=4, r0=1.0, refine_near=1):
    """The constant-density star's domain (Sec. III.B): the cube [-8 r0, 8 r0]^3, one affine
    macro refined uniformly to ``level``, then ``refine_near`` times more in the cells that
    come within 1.5 r0 of the centre while wider than r0 / 2 (2:1 balanced); degree p,
    Dirichlet faces."""
    def near(key, c0, c1):
        return np.linalg.norm(np.clip(0.0, c0, c1)) <= 1.5 * r0 and (c1 - c0).max() > 0.5 * r0
    return box_grid((1, 1, 1), level, p, lo=(-8.0 * r0,) * 3, hi=(8.0 * r0,) * 3, refine=[near] * refine_near)


def unit_cube(level=2, p=3):
    """Unit cube, one affine macro refined uniformly to ``level`` (config 1 at level 2, p 3)."""
    m = box_grid((1, 1, 1), level, p)
    m["name"] = "unit_cube_l%d_p%d" % (level, p)
    return m


def cubed_sphere_shell(level=3, p=5, r_in=1.0, r_out=1e9, zeta_break=0.5, r_break=10.0,
                       radial_kind=2, inner_refine=True):
    """Six-patch cubed-sphere shell (compactified outer part), config 2 at the defaults.

    Each patch is one SHELL macro refined uniformly to ``level``; with ``inner_refine`` the
    innermost radial layer of cells is refined once more (2:1 non-conforming mortars).
    """
    hexes, kinds, params = [], [], []
    for R in SHELL_FRAMES:
        v = []
        for c in range(8):
            c0, c1, c2 = c & 1, (c >> 1) & 1, (c >> 2) & 1
            d = R @ np.array([2 * c0 - 1, 2 * c1 - 1, 1])
            v.append((tuple(int(x) for x in d), c2))
        hexes.append(v)
        par = np.zeros(16)
        par[0:9] = R.reshape(-1)
        par[9] = radial_kind
        par[10], par[11], par[12], par[13] = r_in, r_out, zeta_break, r_break
        kinds.append(SHELL)
        params.append(par)
    forest = _forest_for(hexes)
    for _ in range(level):
        forest.refine_where(lambda key: True)
    if inner_refine:
        forest.refine_where(lambda key: key[4] == 0)
        forest.balance()
    return _finish(kinds, params, hexes, lambda m, f: BC_DIRICHLET, forest,
                   lambda key: p, dict(name="cubed_sphere_shell_l%d_p%d" % (level, p)))


def hp_sphere_cube(level=5, p_lo=2, p_hi=7, seed=0, r_cut=0.5):
    """[-1,1]^3, one macro at ``level``; random p in [p_lo, p_hi]; cells cut by |x| = r_cut refined.

    Children inherit the parent's degree (config 3 at the defaults).
    """
    rng = np.random.default_rng(seed)
    n = 1 << level
    pgrid = rng.integers(p_lo, p_hi + 1, size=(n, n, n))

    def cut(key, c0, c1):
        # the cell is cut when the sphere separates its nearest and farthest points
        near = np.clip(0.0, c0, c1)
        far = np.where(np.abs(c0) > np.abs(c1), c0, c1)
        return key[1] == level and np.linalg.norm(near) < r_cut < np.linalg.norm(far)

    def p_of(key):
        m, l, i, j, k = key
        sh = l - level
        return pgrid[k >> sh, j >> sh, i >> sh] if sh >= 0 else pgrid[k, j, i]

    mesh = box_grid((1, 1, 1), level, 0, lo=(-1, -1, -1), hi=(1, 1, 1), p_of=p_of,
                    refine=[cut])
    mesh["name"] = "hp_sphere_cube_l%d_p%d-%d_s%d" % (level, p_lo, p_hi, seed)
    return mesh


def puncture_mesh(level=2, p=6, punctures=None, n_ref=5, reach=3.0, r_cube=10.0, r_sphere=20.0, r_out=1e11):
    """Cube with a compactified exterior (13 macros) refined around punctures (config 4).

    Macros: the central cube [-r_cube, r_cube]^3 (affine), six cube-to-sphere wedges from
    its faces to the sphere r_sphere, six shell wedges from r_sphere to r_out with the
    inverse-radius (compactified) radial map.  Every macro is refined to ``level``; then,
    ``n_ref`` times, every cell of the central cube whose centre lies within ``reach`` cell
    diameters of a puncture centre is refined, each pass followed by 2:1 balance.
    ``punctures``: array of centres [K, 3] (e.g. the rows of ``puncture_problem``).
    Dirichlet data on r = r_out.
    """
    hexes, kinds, params = [], [], []
    # central cube
    hexes.append([(tuple(int(2 * ((c >> d) & 1) - 1) for d in range(3)), 0) for c in range(8)])
    par = np.zeros(16)
    par[0:3] = -r_cube
    par[3], par[7], par[11] = 2 * r_cube, 2 * r_cube, 2 * r_cube
    kinds.append(AFFINE)
    params.append(par)
    for layer in (0, 1):
        for R in SHELL_FRAMES:
            v = []
            for c in range(8):
                c0, c1, c2 = c & 1, (c >> 1) & 1, (c >> 2) & 1
                d = R @ np.array([2 * c0 - 1, 2 * c1 - 1, 1])
                v.append((tuple(int(x) for x in d), layer + c2))
            hexes.append(v)
            par = np.zeros(16)
            par[0:9] = R.reshape(-1)
            if layer == 0:
                par[10], par[11] = r_cube, r_sphere
                kinds.append(CUBE_SPHERE)
            else:
                par[9], par[10], par[11] = 1, r_sphere, r_out
                par[12], par[13] = 0.0, r_sphere  # (break of the piecewise map: unused here)
                kinds.append(SHELL)
            params.append(par)
    forest = _forest_for(hexes)
    for _ in range(level):
        forest.refine_where(lambda key: True)
    centres = np.zeros((0, 3)) if punctures is None else np.asarray(punctures, float).reshape(-1, 3)

    def near(key):
        m, l, i, j, k = key
        if m != 0 or len(centres) == 0:
            return False
        h = 2.0 * r_cube / (1 << l)
        ctr = -r_cube + h * (np.array([i, j, k]) + 0.5)
        return np.min(np.linalg.norm(centres - ctr, axis=1)) <= reach * h * np.sqrt(3.0)

    for _ in range(n_ref):
        forest.refine_where(near)
        forest.balance()

    def bc(m, f):
        return BC_DIRICHLET

    return _finish(kinds, params, hexes, bc, forest, lambda key: p,
                   dict(name="puncture_l%d_p%d_r%d" % (level, p, n_ref)))


def mesh_summary(mesh):
    p = mesh["elem_p"]
    return dict(n_elem=int(len(p)), n_dof=int(np.sum((p + 1) ** 3)),
                n_macro=int(len(mesh["macro_kind"])),
                levels=sorted(set(int(x) for x in mesh["elem_level"])),
                degrees=sorted(set(int(x) for x in p)))
