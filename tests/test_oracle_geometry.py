"""Pins for the oracle's geometry and mortar bookkeeping (Sec. II.A.1, II.A.5, III.C)."""
import numpy as np
import pytest

import meshgen
from oracle import geometry, mesh as om


def test_inverse_radial_endpoints():
    # Eq. inverse_mapping: r(x1) = r1, r(x2) = r2, and 1/r is linear in x
    for (x1, x2, r1, r2) in [(0.5, 1.0, 10.0, 1e9), (-1.0, 1.0, 2.0, 3.0), (0.0, 1.0, 20.0, 1e11)]:
        r, dr = geometry.inverse_radial(np.array([x1, x2]), x1, x2, r1, r2)
        np.testing.assert_allclose(r, [r1, r2], rtol=1e-14)
        z = np.linspace(x1, x2, 7)
        rr, drr = geometry.inverse_radial(z, x1, x2, r1, r2)
        inv = 1.0 / rr
        np.testing.assert_allclose(np.diff(inv, 2), 0.0, atol=1e-14 * max(1.0, 1.0 / r1))
        h = 1e-7
        rp, _ = geometry.inverse_radial(z[1:-1] + h, x1, x2, r1, r2)
        rm, _ = geometry.inverse_radial(z[1:-1] - h, x1, x2, r1, r2)
        np.testing.assert_allclose(drr[1:-1], (rp - rm) / (2 * h), rtol=1e-5)


def test_inverse_radial_equals_printed_form_where_well_conditioned():
    # the printed form r = m/(x - t) agrees with the evaluated form away from cancellation
    x1, x2, r1, r2 = 0.5, 1.0, 10.0, 1e3
    m = (x2 - x1) / (1.0 / r2 - 1.0 / r1)
    t = (x1 * r1 - x2 * r2) / (r1 - r2)
    z = np.linspace(x1, x1 + 0.4, 9)
    r, _ = geometry.inverse_radial(z, x1, x2, r1, r2)
    np.testing.assert_allclose(r, m / (z - t), rtol=1e-12)


def _fd_jacobian(kind, par, xi, zc):
    h = 1e-6
    J = np.zeros(xi.shape[:-1] + (3, 3))
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        xp, _ = geometry.macro_map(kind, par, xi + e, zc)
        xm, _ = geometry.macro_map(kind, par, xi - e, zc)
        J[..., :, d] = (xp - xm) / (2 * h)
    return J


@pytest.mark.parametrize("kind", ["shell_lin", "shell_inv", "cube_sphere", "affine"])
def test_jacobian_matches_finite_differences(kind):
    rng = np.random.default_rng(1)
    par = np.zeros(16)
    R = meshgen.meshes.SHELL_FRAMES[3]
    par[0:9] = R.reshape(-1)
    if kind == "shell_lin":
        k = geometry.SHELL
        par[9:14] = [0, 1.0, 10.0, 0.5, 10.0]
    elif kind == "shell_inv":
        k = geometry.SHELL
        par[9:14] = [1, 10.0, 1e3, 0.5, 10.0]
    elif kind == "cube_sphere":
        k = geometry.CUBE_SPHERE
        par[10:12] = [1.0, 2.5]
    else:
        k = geometry.AFFINE
        par[0:3] = rng.uniform(-1, 1, 3)
        par[3:12] = (np.eye(3) * 2.0 + rng.uniform(-0.3, 0.3, (3, 3))).T.reshape(-1)
    xi = rng.uniform(-0.95, 0.95, (20, 3))
    x, J = geometry.macro_map(k, par, xi)
    Jfd = _fd_jacobian(k, par, xi, xi[:, 2])
    np.testing.assert_allclose(J, Jfd, rtol=1e-6, atol=1e-6 * np.max(np.abs(J)))
    assert np.all(np.linalg.det(J) > 0)


def test_shell_radius_and_positive_jacobian():
    m = meshgen.cubed_sphere_shell(level=2, p=2)
    xi = np.random.default_rng(0).uniform(-1, 1, (30, 3))
    E = len(m["elem_p"])
    x, J = geometry.element_map(m, np.arange(E)[:, None], xi[None])
    r = np.linalg.norm(x, axis=-1)
    assert r.min() >= 1.0 - 1e-12 and r.max() <= 1e9 * (1 + 1e-12)
    assert np.all(np.linalg.det(J) > 0)
    # the inner boundary (xi2 = -1 on radial-anchor-0 cells) is the unit sphere
    inner = np.where(m["elem_anchor"][:, 2] == 0)[0]
    xs, _ = geometry.element_map(m, inner[:, None], np.array([[0.3, -0.2, -1.0]])[None])
    np.testing.assert_allclose(np.linalg.norm(xs, axis=-1), 1.0, rtol=1e-14)


@pytest.mark.parametrize("maker", [
    lambda: meshgen.cubed_sphere_shell(level=2, p=2),
    lambda: meshgen.hp_sphere_cube(level=2, p_lo=2, p_hi=4, seed=3, r_cut=0.6),
    lambda: meshgen.box_grid((2, 1, 2), 1, 2),
])
def test_mortar_points_coincide_from_both_sides(maker):
    m = maker()
    s = np.array([-0.9, -0.1, 0.45, 0.8])
    t = np.array([0.7, -0.6, 0.05, -0.95])
    worst = 0.0
    for mt in om.build_mortars(m):
        if mt["ep"] < 0:
            continue
        xm, _ = geometry.element_map(m, np.full(4, mt["em"]), om.face_point(mt["fm"], s, t))
        a, b = om.minus_to_plus(mt, s, t)
        xp, _ = geometry.element_map(m, np.full(4, mt["ep"]), om.face_point(mt["fp"], a, b))
        worst = max(worst, np.max(np.abs(xm - xp)) / max(1.0, np.max(np.abs(xm))))
    assert worst < 1e-13


def test_mortar_counts_and_areas():
    # every interior face of the uniform 4^3 cube is one conforming mortar; 96 Dirichlet faces
    m = meshgen.unit_cube(2, 3)
    mts = om.build_mortars(m)
    assert sum(mt["ep"] >= 0 for mt in mts) == 3 * 4 * 4 * 3
    assert sum(mt["ep"] < 0 for mt in mts) == 6 * 16
    # 2:1: a refined corner cell in a 2^3 cube creates 4 mortars on each of its 3 inner faces
    m2 = meshgen.box_grid((1, 1, 1), 1, 2, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5])
    mts = om.build_mortars(m2)
    assert sum(mt["sub"] is not None for mt in mts) == 12


def test_hierarchy_is_strictly_coarser_and_balanced():
    m = meshgen.cubed_sphere_shell(level=2, p=3)
    H = om.hierarchy(m)
    assert len(H[-1]["elem_p"]) == 6 and np.all(H[-1]["elem_level"] == 0)
    for a, b in zip(H[:-1], H[1:]):
        assert len(b["elem_p"]) < len(a["elem_p"])
        om.build_mortars(b)  # raises on a 2:1 violation
        om.parent_map(a, b)  # every fine cell has a coarse cell at most one level up
    hp = meshgen.hp_sphere_cube(level=3, p_lo=2, p_hi=6, seed=1)
    H = om.hierarchy(hp)
    for a, b in zip(H[:-1], H[1:]):
        pm = om.parent_map(a, b)
        for k, (K, bits) in enumerate(pm):
            assert b["elem_p"][K] <= a["elem_p"][k]  # coarse degree is the min of the children


def _shell_jacobian_ld(par, xi):
    """Jacobian of a SHELL macro (radial kind 2, inverse branch) in extended precision
    (np.longdouble): the same closed form as the macro map, evaluated independently."""
    LD = np.longdouble
    R = np.asarray(par[0:9]).astype(LD).reshape(3, 3)
    r_out, zb, rb = (LD(par[i]) for i in (11, 12, 13))
    pi = LD("3.14159265358979323846264338327950288")
    X, Y, z = np.tan(pi / 4 * xi[:, 0]), np.tan(pi / 4 * xi[:, 1]), xi[:, 2]
    dX, dY = pi / 4 * (1 + X * X), pi / 4 * (1 + Y * Y)
    v = np.stack([X, Y, np.ones_like(X)], -1) @ R.T
    nv = np.sqrt(X * X + Y * Y + 1)
    u = v / nv[:, None]
    du_dX = R[:, 0][None, :] / nv[:, None] - v * (X / nv ** 3)[:, None]
    du_dY = R[:, 1][None, :] / nv[:, None] - v * (Y / nv ** 3)[:, None]
    r = 1 / (((LD(1) - z) / rb + (z - zb) / r_out) / (LD(1) - zb))
    dr = -r * r * (1 / r_out - 1 / rb) / (LD(1) - zb)
    J = np.zeros((len(z), 3, 3), dtype=LD)
    J[:, :, 0] = (r * dX)[:, None] * du_dX
    J[:, :, 1] = (r * dY)[:, None] * du_dY
    J[:, :, 2] = dr[:, None] * u
    return J


def _inv3_ld(a):
    C = np.empty_like(a)
    for i in range(3):
        for j in range(3):
            r0, r1 = [k for k in range(3) if k != j]
            c0, c1 = [k for k in range(3) if k != i]
            C[:, i, j] = (-1) ** (i + j) * (a[:, r0, c0] * a[:, r1, c1] - a[:, r0, c1] * a[:, r1, c0])
    det = np.einsum("pj,pj->p", a[:, 0, :], C[:, :, 0])
    return C / det[:, None, None]


def test_compactified_face_metric_fp64_noise_against_extended_precision():
    # The outer layer of the r_out = 1e9 shell: the face metric J^-1 n on its radial faces has
    # an exact tangential part of zero (the angles do not depend on r) and a radial part of
    # size 1/(dr/dzeta); an FP64 evaluation leaves rounding noise of relative size
    # eps (dr/dzeta)/r there.  Against an extended-precision evaluation of the same closed form,
    # FP64 (the oracle's path) is off by 1e-9 .. 1e-6 relative, while the volume metric G, scaled
    # by sqrt(G_dd G_cc), stays at rounding level.  Two FP64 implementations of the operator
    # therefore differ in the rows of that layer by up to this noise times the face terms'
    # share of the row: the bound behind the compactified-mesh tolerances of the GPU tests.
    from oracle import rules
    m = meshgen.cubed_sphere_shell(level=2, p=4)
    lev, anc = m["elem_level"], m["elem_anchor"]
    outer = np.where(anc[:, 2] == (1 << lev) - 1)[0][:12]
    eta, _ = rules.gl(6)
    LD = np.longdouble
    worst_face, worst_G = 0.0, 0.0
    xi_v = np.stack(np.meshgrid(eta, eta, eta, indexing="ij")[::-1], -1).reshape(-1, 3)
    for e in outer:
        sc = LD(1) / LD(2) ** lev[e]
        par = m["macro_params"][m["elem_macro"][e]]
        for zf in (-1.0, 1.0):
            s, t = np.meshgrid(eta, eta, indexing="xy")
            xi_f = np.stack([s.reshape(-1), t.reshape(-1), np.full(s.size, zf)], -1)
            _, J64 = geometry.element_map(m, np.full(len(xi_f), e), xi_f)
            Ji = np.linalg.inv(J64)
            nh = Ji[:, 2, :] / np.linalg.norm(Ji[:, 2, :], axis=-1)[:, None]
            v64 = np.einsum("pri,pi->pr", Ji, nh)
            Jil = _inv3_ld(_shell_jacobian_ld(par, -1 + (2 * anc[e].astype(LD) + 1 + xi_f.astype(LD)) * sc) * sc)
            nl = Jil[:, 2, :] / np.sqrt(np.sum(Jil[:, 2, :] ** 2, -1))[:, None]
            vl = np.einsum("pri,pi->pr", Jil, nl).astype(float)
            worst_face = max(worst_face, float((np.abs(v64 - vl).max(-1) / np.abs(vl).max(-1)).max()))
        _, J64 = geometry.element_map(m, np.full(len(xi_v), e), xi_v)
        Ji = np.linalg.inv(J64)
        G64 = np.einsum("pdi,pci->pdc", Ji, Ji) * np.linalg.det(J64)[:, None, None]
        Jl = _shell_jacobian_ld(par, -1 + (2 * anc[e].astype(LD) + 1 + xi_v.astype(LD)) * sc) * sc
        Jil = _inv3_ld(Jl)
        detl = np.einsum("pj,pj->p", Jl[:, 0, :], np.cross(Jl[:, 1, :], Jl[:, 2, :]))
        Gl = (np.einsum("pdi,pci->pdc", Jil, Jil) * detl[:, None, None]).astype(float)
        dg = np.abs(np.einsum("pdd->pd", Gl))
        worst_G = max(worst_G, float((np.abs(G64 - Gl) / np.sqrt(dg[:, :, None] * dg[:, None, :])).max()))
    print("FP64 vs extended precision: face metric %.3e, volume metric %.3e" % (worst_face, worst_G))
    assert 1e-9 < worst_face < 1e-6
    assert worst_G < 1e-13


def test_uniform_box_equals_octree_box():
    # the array-generated uniform box has the octree box's cells and macro tables
    a = meshgen.box_grid((2, 1, 1), 2, 3)
    b = meshgen.uniform_box((2, 1, 1), 2, 3)
    cells = lambda m: set(map(tuple, np.column_stack([m["elem_macro"], m["elem_level"], m["elem_anchor"], m["elem_p"]])))
    assert cells(a) == cells(b)
    for k in ("macro_kind", "macro_params", "macro_nbr", "macro_nbr_face", "macro_nbr_orient", "macro_bc"):
        assert np.array_equal(a[k], b[k])
