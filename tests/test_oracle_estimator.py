"""Pins of the oracle's a posteriori estimator (Eqs. Eta2_*) and smooth-pred decisions (Alg.
hpamr): values fixed by closed forms, by the exactness of the discretisation and by the
behaviour the text describes."""
import numpy as np
import pytest

import meshgen
from oracle import estimator as est
from oracle import geometry, problems
from oracle.operator import SIPG, assemble_dense

MESHES = {
    "box_2to1_p3": lambda: meshgen.box_grid((2, 1, 1), 1, 3,
                                            refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5]),
    "hp_p2_4": lambda: meshgen.hp_sphere_cube(level=1, p_lo=2, p_hi=4, seed=1, r_cut=0.6),
}


def _box_corners(mesh):
    """Per element of an axis-aligned affine mesh: its lowest and highest corner."""
    E = len(mesh["elem_p"])
    c = np.array([[-1.0, -1.0, -1.0], [1.0, 1.0, 1.0]])
    x, _ = geometry.element_map(mesh, np.arange(E)[:, None], c[None])
    return x[:, 0], x[:, 1]


def _box_widths(mesh):
    lo, hi = _box_corners(mesh)
    return hi - lo


@pytest.mark.parametrize("name", list(MESHES))
def test_solution_in_the_space_has_zero_estimate(name):
    # u in Q_2 solves -lap u = g exactly and its interpolant is continuous: no residual, no jumps
    mesh = MESHES[name]()
    prob = meshgen.polynomial_problem(2, seed=4)
    op = SIPG(mesh, prob)
    u = op.interpolate(lambda x: problems.exact_u(prob, x))
    r = est.estimate(op, u, prob)
    scale = est.estimate(op, u + np.random.default_rng(1).standard_normal(op.ndof), prob)["eta2"].max()
    assert r["eta2"].max() <= 1e-22 * scale


@pytest.mark.parametrize("name", list(MESHES))
def test_constant_laplacian_residual_closed_form(name):
    # u = x^2 with g = 0: R_e = lap u = 2 inside every element, no jumps and u_h = g_D on the
    # boundary, so eta2(e) = h_e^2 p_e^2 4 |e|
    mesh = MESHES[name]()
    C = np.zeros((3, 3, 3))
    C[2, 0, 0] = 1.0
    prob = meshgen.polynomial_dirichlet_problem(C)
    op = SIPG(mesh, prob)
    u = op.interpolate(lambda x: x[..., 0] ** 2)
    r = est.estimate(op, u, prob)
    w = _box_widths(mesh)
    vol = np.prod(w, axis=1)
    h = np.linalg.norm(w, axis=1)
    expect = h ** 2 * mesh["elem_p"] ** 2 * 4.0 * vol
    assert np.allclose(r["eta2"], expect, rtol=1e-12, atol=0)
    assert np.allclose(r["eta2"], r["eta2_vol"], rtol=1e-12)


def test_indicator_jumps_closed_form():
    # u_h = 1 on one element, 0 elsewhere, with u = g = 0: only the jump terms, sigma |face| per
    # face with sigma = C p^2 / h (h the width normal to the face)
    mesh = meshgen.box_grid((1, 1, 1), 2, 3)
    prob = meshgen.polynomial_dirichlet_problem(np.zeros((1, 1, 1)))
    op = SIPG(mesh, prob)
    e0 = 21  # an interior element of the 4^3 grid (checked below)
    u = np.zeros(op.ndof)
    u[op.offsets[e0]:op.offsets[e0 + 1]] = 1.0
    r = est.estimate(op, u, prob)
    w = _box_widths(mesh)
    p = 3
    per_face = []
    for d in range(3):
        t = [a for a in range(3) if a != d]
        per_face.append(op.C * p * p / w[e0, d] * w[e0, t[0]] * w[e0, t[1]])
    nb = [mt for mt in op.mortars if mt["ep"] >= 0 and e0 in (mt["em"], mt["ep"])]
    assert len(nb) == 6  # interior element
    assert r["eta2"][e0] == pytest.approx(2 * sum(per_face), rel=1e-12)
    for mt in nb:
        other = mt["ep"] if mt["em"] == e0 else mt["em"]
        d = mt["fm"] // 2
        assert r["eta2"][other] == pytest.approx(per_face[d], rel=1e-12)
    assert np.count_nonzero(r["eta2"]) == 7


def test_flux_jump_closed_form_on_a_kink():
    # u = |x - 1/2| is continuous and piecewise linear with the kink on element faces: the
    # normal-flux jump is -2 on the faces at x = 1/2 (eta2_{m,1} = (h/p) 4 |face|, h the width
    # normal to the face), zero on every other interior face
    mesh = meshgen.box_grid((1, 1, 1), 2, 2)
    prob = meshgen.polynomial_dirichlet_problem(np.zeros((1, 1, 1)))
    op = SIPG(mesh, prob)
    u = op.interpolate(lambda x: np.abs(x[..., 0] - 0.5))
    r = est.estimate(op, u, prob)
    lo, hi = _box_corners(mesh)
    w = hi - lo
    p = 2
    n_kink = 0
    for mi, mt in enumerate(op.mortars):
        if mt["ep"] < 0:
            continue
        em, d = mt["em"], mt["fm"] // 2
        xface = hi[em, 0] if mt["fm"] == 1 else lo[em, 0]
        if d == 0 and abs(xface - 0.5) < 1e-12:
            n_kink += 1
            assert r["eta2_face"][mi] == pytest.approx(w[em, 0] / p * 4.0 * w[em, 1] * w[em, 2], rel=1e-12)
        else:
            assert abs(r["eta2_face"][mi]) <= 1e-24
    assert n_kink == 16


def _solve(op):
    A = assemble_dense(op)
    return np.linalg.solve(A, op.rhs())


def test_estimator_follows_the_energy_error():
    # sin sin sin on refined cubes at p = 1 and 2: eta decreases like the energy error (rate
    # h^p, Eq. expectedconvergence) and stays within a bounded factor of it
    prob = meshgen.problem_config1()
    for p, levels in ((1, (1, 2, 3)), (2, (1, 2))):
        etas, errs, hs = [], [], []
        for lev in levels:
            mesh = meshgen.unit_cube(lev, p)
            op = SIPG(mesh, prob)
            u = _solve(op)
            etas.append(np.sqrt(est.estimate(op, u, prob)["eta2"].sum()))
            errs.append(op.energy_error(u, lambda x: problems.exact_u(prob, x),
                                        lambda x: problems.grad_u(prob, x)))
            hs.append(0.5 ** lev)
        rate = np.polyfit(np.log(hs), np.log(etas), 1)[0]
        ratio = np.array(etas) / np.array(errs)
        print("p", p, "eta", etas, "energy error", errs, "rate", rate, "eta / error", ratio)
        assert abs(rate - p) <= 0.35
        assert 0.5 <= ratio.min() and ratio.max() <= 50 and ratio.max() / ratio.min() <= 2.5


def test_smooth_pred_keeps_p_refining_while_eta_falls_exponentially():
    # an element whose eta2 falls by 0.05 per degree (faster than gamma_p = 0.1) keeps being
    # p-refined; one whose eta2 stalls is h-refined after its first p step; with no prediction
    # every marked element is p-refined first
    p = np.array([2, 2])
    pred = np.full(2, np.inf)
    eta2 = np.array([1.0, 1.0])
    history = []
    for step in range(4):
        marked = np.ones(2, bool)
        act, new_pred = est.smooth_pred(eta2, pred, p, marked)
        history.append(act.copy())
        p = p + (act == 2)
        pred = new_pred
        eta2 = np.array([eta2[0] * 0.05 if act[0] == 2 else eta2[0], 1.0])
    assert [h[0] for h in history] == [2, 2, 2, 2]
    assert [h[1] for h in history][:2] == [2, 1]


def test_marking_fraction_and_mean():
    eta2 = np.array([1.0, 5.0, 3.0, 5.0, 0.5])
    assert list(np.flatnonzero(est.mark_fraction(eta2, 0.4))) == [1, 3]
    assert list(np.flatnonzero(est.mark_fraction(eta2, 0.5))) == [1, 2, 3]
    assert list(np.flatnonzero(est.mark_mean(eta2, 1.0))) == [1, 2, 3]


def _scaled(mesh, s):
    """The same cells under macro maps composed with x -> s x."""
    out = dict(mesh)
    par = np.array(mesh["macro_params"], float, copy=True)
    for m, kind in enumerate(mesh["macro_kind"]):
        if kind == meshgen.meshes.AFFINE:
            par[m, 0:12] *= s
        elif kind == meshgen.meshes.SHELL:
            par[m, [10, 11, 13]] *= s  # r_in, r_out, r_break
        else:
            par[m, [10, 11]] *= s      # cube half-side, sphere radius
    out["macro_params"] = par
    return out


@pytest.mark.parametrize("name", ["box_2to1_p3", "hp_p2_4", "shell"])
def test_fiducial_grid_weights_scale_with_the_grid(name):
    # a fiducial grid equal to the physical one changes nothing; the physical grid scaled by s
    # as the fiducial one multiplies the volume parts by s^5 (h_e^2 det J), the flux-jump parts
    # by s^3 (h_m S) and the value-jump parts by s (sigma S), the integrands staying the same
    mesh = MESHES[name]() if name in MESHES else meshgen.cubed_sphere_shell(level=1, p=3, r_out=1e3)
    prob = meshgen.problem_config1()
    op = SIPG(mesh, prob)
    u = op.interpolate(lambda x: problems.exact_u(prob, x)) + 0.05 * np.random.default_rng(2).standard_normal(op.ndof)
    r = est.estimate(op, u, prob)
    same = est.estimate(op, u, prob, fiducial=mesh)
    for k in r:
        assert np.allclose(same[k], r[k], rtol=1e-13, atol=0)
    s = 3.0
    f = est.estimate(op, u, prob, fiducial=_scaled(mesh, s))
    assert np.allclose(f["eta2_vol"], s ** 5 * r["eta2_vol"], rtol=1e-11)
    assert np.allclose(f["eta2_flux"], s ** 3 * r["eta2_flux"], rtol=1e-11)
    assert np.allclose(f["eta2_jump"], s * r["eta2_jump"], rtol=1e-11)
    assert np.allclose(f["eta2_face"], f["eta2_flux"] + f["eta2_jump"], rtol=1e-14)
    assert r["eta2_flux"].max() > 0 and r["eta2_jump"].max() > 0


def test_fiducial_grid_refuses_other_cells():
    mesh = MESHES["box_2to1_p3"]()
    prob = meshgen.problem_config1()
    op = SIPG(mesh, prob)
    other = meshgen.box_grid((2, 1, 1), 1, 3)
    with pytest.raises(ValueError):
        est.estimate(op, np.zeros(op.ndof), prob, fiducial=other)


def test_compact_estimator_marks_the_inner_cells_of_a_compactified_shell():
    # Sec. III.C: on a shell compactified to r = 1e9 the estimate on the physical grid is
    # dominated by the stretched outer cells (their Jacobians), so marking refines there; on the
    # unstretched twin (radii 2..3) it marks the inner cells, where the solution varies, as
    # both estimates do on the mildly stretched shell (r = 1e3)
    prob = meshgen.problem_config2()

    def marked_outer_share(r_out, compact):
        mesh = meshgen.cubed_sphere_shell(level=2, p=3, r_out=r_out)
        op = SIPG(mesh, prob)
        u = op.interpolate(lambda x: problems.exact_u(prob, x))
        fid = None
        if compact:
            fid = dict(mesh)
            par = np.array(mesh["macro_params"], float, copy=True)
            par[:, 9], par[:, 10], par[:, 11] = 0.0, 2.0, 3.0
            fid["macro_params"] = par
        mk = est.mark_fraction(est.estimate(op, u, prob, fiducial=fid)["eta2"], 0.1)
        zc = -1 + (2 * mesh["elem_anchor"][:, 2] + 1) / 2.0 ** mesh["elem_level"]  # radial macro coordinate
        return float(np.mean(zc[mk] > 0))

    assert marked_outer_share(1e9, compact=False) > 0.8
    assert marked_outer_share(1e9, compact=True) == 0.0
    assert marked_outer_share(1e3, compact=False) == 0.0
