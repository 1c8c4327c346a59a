"""Helpers shared by the GPU parity tests: contexts, level matching, tolerances."""
import numpy as np

import meshgen
import paper_1907_01572_amd as hp

# GPU tests upload with the element-centric apply wherever an element qualifies (the default
# leaves it off on small mixed-degree levels, which test meshes are); tests of the other modes
# name theirs
hp.EC_MODE_DEFAULT = hp.EC_ALWAYS

# FP64 apply parity (relative L2 over the output vector).
TOL_APPLY = 1e-12
# Compactified shells (r_out = 1e9): the face-metric noise described below; measured in L2
# 7.7e-13 on the finest level, 3.0e-12 on the next and 1.2e-11 on the coarsest (one cell
# spans r = 1 .. 1e9, so the outer faces are a larger share of its rows)
TOL_APPLY_COMPACTIFIED = 5e-11


def coef_of(problem):
    return hp.coef_from_problem(problem)


def dof_perm(lib_cells, oracle_mesh):
    """Index array: library dof i of a level corresponds to oracle dof perm[i]."""
    key = {(int(oracle_mesh["elem_macro"][e]), int(oracle_mesh["elem_level"][e]),
            *map(int, oracle_mesh["elem_anchor"][e])): e for e in range(len(oracle_mesh["elem_p"]))}
    n = oracle_mesh["elem_p"].astype(np.int64) + 1
    off = np.concatenate([[0], np.cumsum(n ** 3)])
    out = []
    for e in range(len(lib_cells["elem_p"])):
        k = (int(lib_cells["elem_macro"][e]), int(lib_cells["elem_level"][e]),
             *map(int, lib_cells["elem_anchor"][e]))
        eo = key[k]
        assert oracle_mesh["elem_p"][eo] == lib_cells["elem_p"][e]
        out.append(np.arange(off[eo], off[eo + 1]))
    return np.concatenate(out)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def row_err(y, y_ref, diag, x, rows=None):
    """Largest per-row error max_i |y_i - y_ref_i| / (diag(A)_i |x|_inf): each row against the
    size of its own terms (the diagonal of the SIPG operator bounds its row to a modest factor),
    so an error confined to a few faces is not diluted as in a norm over the whole vector."""
    y, y_ref, diag = np.asarray(y), np.asarray(y_ref), np.asarray(diag)
    if rows is not None:
        y, y_ref, diag = y[rows], y_ref[rows], diag[rows]
    return float(np.max(np.abs(y - y_ref) / (np.abs(diag) * np.abs(x).max())))


# per-row FP64 apply parity (row_err): a row sums O(100) products of its own size
TOL_ROW = 1e-12
# per-row parity in the outer layer of a compactified shell (r_out = 1e9): there the FP64 face
# metric J^-1 n itself carries relative rounding noise up to 1.2e-7 against an extended-precision
# evaluation (tests/test_oracle_geometry.py, compactified face metric), so two FP64
# implementations may differ by twice that times the face terms' share of a row; measured
# 1.3e-11 on the finest level and 9.3e-11 on the coarsest, gated at 5e-10 (about 500x below
# that bound)
TOL_ROW_COMPACTIFIED = 5e-10


MESHES = {
    "cube_l2_p3": (lambda: meshgen.unit_cube(2, 3), meshgen.problem_config1()),
    # element blocks of 343 and 512 rows (several 64-row panels of the packed inverse blocks)
    "cube_l1_p6": (lambda: meshgen.unit_cube(1, 6), meshgen.problem_config1()),
    "cube_l1_p7": (lambda: meshgen.unit_cube(1, 7), meshgen.problem_config1()),
    "box_2to1_p3": (lambda: meshgen.box_grid((2, 1, 1), 1, 3,
                                             refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5]),
                    meshgen.problem_config1()),
    "hp_k": (lambda: meshgen.hp_sphere_cube(level=2, p_lo=1, p_hi=5, seed=2, r_cut=0.6),
             meshgen.problem_config3(r0=0.6)),
    # four affine macros (faces across macros), degree 2 (16 elements per wavefront)
    "box_macros_p2": (lambda: meshgen.box_grid((2, 2, 1), 1, 2), meshgen.problem_config1()),
    # every pair of degrees 2..7 across conforming faces, 2:1 faces around the refined shell
    "hp_p2_7_k1": (lambda: meshgen.hp_sphere_cube(level=2, p_lo=2, p_hi=7, seed=3, r_cut=0.6),
                   meshgen.problem_config1()),
    "shell_l2_p3_r1e3": (lambda: meshgen.cubed_sphere_shell(level=2, p=3, r_out=1e3),
                         meshgen.problem_config2()),
    "shell_l2_p4_r1e9": (lambda: meshgen.cubed_sphere_shell(level=2, p=4), meshgen.problem_config2()),
}
