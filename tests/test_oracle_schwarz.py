"""Pins of the oracle's additive Schwarz smoother (Sec. II.D: Eq. schwarz_weight, Alg.
schwarz_smoother): closed forms of the weight function, the partition of unity, subdomain sizes
that follow from the construction, an independent geometric membership test, exactness on a
one-element mesh, and the robustness the text reports for the multigrid solve."""
import numpy as np
import pytest

import meshgen
from oracle import geometry, rules
from oracle import schwarz as sw
from oracle.operator import SIPG, assemble_dense
from oracle.solvers import Multigrid, fcg


def test_phi_and_weight_closed_forms():
    # phi is the C1 smoothstep from -1 to 1: phi(+-1) = +-1, phi(0) = 0, slope 15/8 at 0 and 0
    # at +-1 (one-sided differences), odd, constant outside [-1, 1]
    t = np.linspace(-1.0, 1.0, 2001)
    assert sw.phi(1.0) == 1.0 and sw.phi(-1.0) == -1.0 and sw.phi(0.0) == 0.0
    assert np.allclose(sw.phi(-t), -sw.phi(t), rtol=0, atol=1e-15)
    assert np.all(np.diff(sw.phi(t)) > 0)
    h = 1e-6
    assert abs((sw.phi(h) - sw.phi(-h)) / (2 * h) - 15.0 / 8.0) < 1e-9
    assert abs((sw.phi(1.0) - sw.phi(1.0 - h)) / h) < 1e-5
    assert np.all(sw.phi(np.array([1.5, 7.0, -2.0])) == np.array([1.0, 1.0, -1.0]))
    for delta in (0.25, 0.5, 1.0):
        # plateau 1 on |xi| <= 1 - delta, one half on the element faces, zero at the overlap's edge
        assert np.all(sw.weight_1d(np.linspace(-1 + delta, 1 - delta, 11), delta) == 1.0)
        assert np.allclose(sw.weight_1d(np.array([-1.0, 1.0]), delta), 0.5, rtol=0, atol=1e-15)
        assert np.all(sw.weight_1d(np.array([-1 - delta, 1 + delta, 3.0]), delta) == 0.0)
        # a domain-boundary side keeps the plateau up to and beyond the face
        assert np.all(sw.weight_1d(np.array([1.0, 1.0 + delta / 2]), delta, upper_open=False) == 1.0)
        assert sw.weight_1d(np.array([-1.0]), delta, upper_open=False)[0] == pytest.approx(0.5, abs=1e-15)


@pytest.mark.parametrize("delta", [0.0, 0.3, 1.0, 1.7])
def test_weights_of_a_row_of_elements_sum_to_one(delta):
    # 1-D: the subdomains centred on the elements of an infinite row see a point at offsets
    # xi - 2 c; their weights telescope to one everywhere (the points on the faces included)
    xi = np.concatenate([np.linspace(-1.0, 1.0, 101), [-1.0, 1.0]])
    total = sum(sw.weight_1d(xi - 2.0 * c, delta) for c in range(-3, 4))
    assert np.allclose(total, 1.0, rtol=0, atol=1e-14)


def test_overlap_width_from_the_lgl_nodes():
    # delta = 1 + xi_(N_overlap - 1): 0 for one layer; for n = 4 the second node -1/sqrt(5)
    assert sw.overlap_width(4, 1) == 0.0
    assert sw.overlap_width(4, 2) == pytest.approx(1.0 - 1.0 / np.sqrt(5.0), rel=1e-14)
    assert sw.overlap_width(3, 2) == pytest.approx(1.0, rel=1e-14)
    with pytest.raises(ValueError):
        sw.overlap_width(4, 4)


MESHES = {
    "cube_l2_p3": lambda: meshgen.unit_cube(2, 3),
    "box_2x1x1_l1_p2": lambda: meshgen.box_grid((2, 1, 1), 1, 2),
    "box_lopsided_l1_p3": lambda: meshgen.box_grid((1, 1, 1), 1, 3, lo=(-0.3, 0.0, 0.1), hi=(1.0, 0.5, 2.0)),
}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("n_overlap", [1, 2])
def test_weights_form_a_partition_of_unity(name, n_overlap):
    op = SIPG(MESHES[name](), meshgen.problem_config1())
    total = np.zeros(op.ndof)
    for idx, w in sw.subdomains(op, n_overlap):
        assert len(np.unique(idx)) == len(idx)
        np.add.at(total, idx, w)
    assert np.allclose(total, 1.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n_overlap", [1, 2, 3])
def test_subdomain_sizes(n_overlap):
    # on a 4^3 grid of p = 3 (n = 4): an interior element's subdomain spans n + 2 N_overlap
    # nodes per axis, a corner element's n + N_overlap (only one side has neighbours)
    mesh = meshgen.unit_cube(2, 3)
    op = SIPG(mesh, meshgen.problem_config1())
    subs = sw.subdomains(op, n_overlap)
    lo, hi = geometry.element_map(mesh, np.arange(len(mesh["elem_p"]))[:, None],
                                  np.array([[-1.0, -1.0, -1.0], [1.0, 1.0, 1.0]]))[0].transpose(1, 0, 2)
    interior = np.all((lo > 1e-12) & (hi < 1 - 1e-12), axis=1)
    corner = np.all((np.abs(lo) < 1e-12) | (np.abs(hi - 1) < 1e-12), axis=1)
    assert interior.sum() == 8 and corner.sum() == 8
    for e in range(len(subs)):
        if interior[e]:
            assert len(subs[e][0]) == (4 + 2 * n_overlap) ** 3
        if corner[e]:
            assert len(subs[e][0]) == (4 + n_overlap) ** 3


@pytest.mark.parametrize("name", list(MESHES))
def test_membership_matches_the_physical_box(name):
    # an independent derivation on these uniform grids: a point belongs to subdomain c exactly
    # when its physical position, in units of e_c's half-widths from e_c's centre, lies within
    # 1 + delta on every axis
    mesh = MESHES[name]()
    op = SIPG(mesh, meshgen.problem_config1())
    n = int(mesh["elem_p"][0]) + 1
    x = op.nodes()
    E = len(mesh["elem_p"])
    c0, J = geometry.element_map(mesh, np.arange(E)[:, None], np.zeros((1, 3)))
    centre, half = c0[:, 0], np.einsum("eii->ei", J[:, 0])
    for n_overlap in range(1, n):
        delta = sw.overlap_width(n, n_overlap)
        for c, (idx, w) in enumerate(sw.subdomains(op, n_overlap)):
            rel = np.abs(x - centre[c]) / half[c]
            expect = np.flatnonzero(np.all(rel <= 1 + delta + 1e-10, axis=1))
            assert np.array_equal(np.sort(idx), expect)
            assert np.array_equal(idx[:n ** 3], np.arange(op.offsets[c], op.offsets[c + 1]))


def test_one_element_mesh_is_solved_in_one_cycle():
    # the only subdomain is the whole mesh, every side is a domain boundary (weights 1): one
    # cycle is the exact solve
    mesh = meshgen.box_grid((1, 1, 1), 0, 3)
    op = SIPG(mesh, meshgen.problem_config1())
    A = assemble_dense(op)
    b = op.rhs()
    subs = sw.subdomains(op, 2)
    assert len(subs) == 1 and np.all(subs[0][1] == 1.0)
    x = sw.smooth(A, subs, b, np.random.default_rng(0).standard_normal(op.ndof), 1)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-12 * np.abs(x).max())


def test_smoother_is_a_linear_iteration_with_a_fixed_point():
    # the exact solution is a fixed point; the error after one cycle is a linear function of
    # the error before it
    mesh = MESHES["box_2x1x1_l1_p2"]()
    op = SIPG(mesh, meshgen.problem_config1())
    A = assemble_dense(op)
    subs = sw.subdomains(op, 2)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(op.ndof)
    b = A @ u
    assert np.allclose(sw.smooth(A, subs, b, u, 2), u, rtol=0, atol=1e-12)
    e1, e2 = rng.standard_normal((2, op.ndof))
    f = lambda e: sw.smooth(A, subs, b, u + e, 1) - u
    assert np.allclose(f(e1 + 2 * e2), f(e1) + 2 * f(e2), rtol=0, atol=1e-11)


@pytest.mark.parametrize("p", [2, 3])
def test_schwarz_multigrid_is_robust(p):
    # Sec. III.C (the comparison of preconditioners): with N_overlap = 2 and 3 Schwarz cycles per
    # smoothing call the multigrid-preconditioned FCG solve needs a handful of iterations, far
    # fewer than with 4 point-Jacobi Chebyshev steps
    mesh = meshgen.unit_cube(2, p)
    prob = meshgen.problem_config1()
    mg_s = Multigrid(mesh, prob, n_cheb=3, smoother="schwarz", schwarz_overlap=2)
    mg_c = Multigrid(mesh, prob, n_cheb=4, smoother="point")
    b = mg_s.ops[0].rhs()
    u, its, hist = fcg(mg_s.ops[0].apply, b, mg_s.vcycle, tol=1e-10, max_iter=50)
    _, itc, _ = fcg(mg_c.ops[0].apply, b, mg_c.vcycle, tol=1e-10, max_iter=50)
    print("p", p, "Schwarz iterations", its, "Chebyshev iterations", itc, "history", hist)
    assert its <= 4 and itc >= 3 * its
    A = assemble_dense(mg_s.ops[0])
    assert np.allclose(u, np.linalg.solve(A, b), rtol=0, atol=1e-8 * np.abs(u).max())


def test_local_cg_reaches_its_tolerance_and_the_exact_solve():
    # the paper's local solver: CG from zero until the subdomain residual falls by 1e-3; with a
    # tolerance near rounding it reproduces the exact local solve
    mesh = MESHES["box_2x1x1_l1_p2"]()
    op = SIPG(mesh, meshgen.problem_config1())
    A = assemble_dense(op)
    rng = np.random.default_rng(4)
    for idx, _ in sw.subdomains(op, 2)[:4]:
        As = A[np.ix_(idx, idx)]
        rs = rng.standard_normal(len(idx))
        d = sw.local_cg(As, rs, 1e-3)
        assert np.linalg.norm(rs - As @ d) <= 1e-3 * np.linalg.norm(rs)
        assert np.allclose(sw.local_cg(As, rs, 1e-14), np.linalg.solve(As, rs), rtol=0, atol=1e-10 * np.abs(d).max())
    assert np.all(sw.local_cg(As, np.zeros(len(idx))) == 0.0)


def test_cg_local_solves_keep_the_multigrid_iterations():
    # R34: the exact local solve is the limit of the paper's CG to 1e-3; the two multigrid
    # preconditioners take the same number of FCG iterations on the 4^3, p = 2 cube
    mesh = meshgen.unit_cube(2, 2)
    prob = meshgen.problem_config1()
    its = {}
    for local in ("exact", "cg"):
        mg = Multigrid(mesh, prob, n_cheb=3, smoother="schwarz", schwarz_overlap=2, schwarz_local=local)
        b = mg.ops[0].rhs()
        _, its[local], _ = fcg(mg.ops[0].apply, b, mg.vcycle, tol=1e-10, max_iter=50)
    print("FCG iterations", its)
    assert its["cg"] <= its["exact"] + 1 and its["exact"] <= 4


@pytest.mark.parametrize("name", list(MESHES) + ["box_2x2x1_l1_p2"])
@pytest.mark.parametrize("n_overlap", [1, 2])
def test_topological_subdomains_equal_the_geometric_ones_on_boxes(name, n_overlap):
    # the construction from face maps (any orientation) reproduces the box construction
    mesh = MESHES[name]() if name in MESHES else meshgen.box_grid((2, 2, 1), 1, 2)
    op = SIPG(mesh, meshgen.problem_config1())
    for (i1, w1), (i2, w2) in zip(sw.subdomains(op, n_overlap), sw.subdomains_topo(op, n_overlap)):
        assert np.array_equal(np.sort(i1), np.sort(i2))
        assert np.allclose(w1[np.argsort(i1)], w2[np.argsort(i2)], rtol=0, atol=1e-15)


def test_face_maps_compose_to_the_identity_around_a_regular_edge():
    # four quarter turns around an edge of the box: stepping +x, +y, -x, -y returns to the
    # start with the identity map (same-macro faces); a rotated face map and its inverse compose
    # to the identity
    ident = ([0, 1, 2], [1.0, 1.0, 1.0], [0.0, 0.0, 0.0])
    M = ident
    for f, fb in ((1, 0), (3, 2), (0, 1), (2, 3)):
        M = sw._compose(M, sw._face_map(f, fb, 0))
    assert M == ident
    for o in range(8):
        fwd = sw._face_map(1, 4, o)  # +x face meeting a -z face, orientation o
        # the inverse map: from the neighbour's face 4 back across to face 1
        back = [m for m in (sw._face_map(4, 1, q) for q in range(8)) if sw._compose(fwd, m)[:2] == ident[:2]]
        assert len(back) == 1
        assert sw._compose(fwd, back[0]) == ident


SHELL = {
    "shell_l2_p3": lambda: meshgen.cubed_sphere_shell(level=2, p=3, r_out=1e3, inner_refine=False),
}


@pytest.mark.parametrize("n_overlap", [1, 2])
def test_shell_weights_are_three_quarters_next_to_the_three_cell_edges(n_overlap):
    # on the six-patch shell cells meet three around the eight radial lines through the cube's
    # corners: the points whose subdomains miss the fourth quadrant sum to exactly 3/4 (before
    # normalisation), all in the cells touching those lines; everywhere else the weights sum to
    # one; inner subdomains have (n + 2 N_overlap)^3 points; after normalisation all sum to one
    mesh = SHELL["shell_l2_p3"]()
    op = SIPG(mesh, meshgen.problem_config2())
    subs = sw.subdomains_topo(op, n_overlap, normalise=False)
    total = np.zeros(op.ndof)
    for idx, w in subs:
        np.add.at(total, idx, w)
    off = np.abs(total - 1.0) > 1e-12
    assert np.allclose(total[off], 0.75, rtol=0, atol=1e-14) and off.sum() > 0
    elems = np.unique(np.searchsorted(op.offsets, np.flatnonzero(off), side="right") - 1)
    a = mesh["elem_anchor"][elems]
    assert np.all((a[:, :2] == 0) | (a[:, :2] == 3))
    A = mesh["elem_anchor"]
    inner = np.flatnonzero(np.all((A >= 1) & (A <= 2), axis=1))
    assert len(inner) == 6 * 8 and {len(subs[e][0]) for e in inner} == {(4 + 2 * n_overlap) ** 3}
    total = np.zeros(op.ndof)
    for idx, w in sw.subdomains_topo(op, n_overlap):
        np.add.at(total, idx, w)
    assert np.allclose(total, 1.0, rtol=0, atol=1e-14)


def test_schwarz_restores_multigrid_on_the_stretched_shell():
    # Sec. III.C: on the shell compactified to r = 1e9 the Chebyshev-smoothed multigrid loses
    # efficiency while the Schwarz smoother keeps a handful of iterations
    mesh = meshgen.cubed_sphere_shell(level=1, p=3, r_out=1e9, inner_refine=False)
    prob = meshgen.problem_config2()
    its = {}
    for name, kw in (("schwarz", dict(n_cheb=3, smoother="schwarz", schwarz_overlap=2)),
                     ("point", dict(n_cheb=4, smoother="point")), ("block", dict(n_cheb=4, smoother="block"))):
        mg = Multigrid(mesh, prob, **kw)
        b = mg.ops[0].rhs()
        _, its[name], _ = fcg(mg.ops[0].apply, b, mg.vcycle, tol=1e-10, max_iter=300)
    print("FCG iterations", its)
    assert its["schwarz"] <= 6 and its["block"] >= 4 * its["schwarz"] and its["point"] >= 10 * its["schwarz"]


def _mixed_degrees(mesh, degrees, seed):
    out = dict(mesh)
    out["elem_p"] = np.random.default_rng(seed).choice(degrees, size=len(mesh["elem_p"])).astype(mesh["elem_p"].dtype)
    return out


@pytest.mark.parametrize("n_overlap,sizes", [(1, [27 + 16, 64 + 9]), (2, [27 + 32, 64 + 9])])
def test_ragged_subdomains_of_two_cells_of_different_degrees(n_overlap, sizes):
    # degrees 2 and 3 side by side: the shared face takes the narrower overlap width (that of
    # degree 3 for N_overlap 2: 1 - 1/sqrt(5), against 1 for degree 2); the degree-2 subdomain
    # takes N_overlap layers of the 4 x 4 face layers of its neighbour, the degree-3 one only the
    # coincident 3 x 3 layer (the next degree-2 layer lies at the face's far side, beyond the
    # width); the weights sum to one without normalisation
    mesh = dict(meshgen.box_grid((2, 1, 1), 0, 2))
    mesh["elem_p"] = np.array([2, 3], dtype=mesh["elem_p"].dtype)
    op = SIPG(mesh, meshgen.problem_config1())
    subs = sw.subdomains_topo(op, n_overlap, normalise=False)
    assert [len(i) for i, _ in subs] == sizes
    total = np.zeros(op.ndof)
    for idx, w in subs:
        np.add.at(total, idx, w)
    assert np.allclose(total, 1.0, rtol=0, atol=1e-14)


def test_ragged_subdomains_on_a_random_degree_cube():
    # degrees 2..4 drawn per cell: with one layer the weights sum to one everywhere; with two,
    # points whose sum differs from one lie only in cells with a neighbour of another degree, and
    # normalisation restores the partition of unity
    mesh = _mixed_degrees(meshgen.unit_cube(2, 2), [2, 3, 4], 1)
    op = SIPG(mesh, meshgen.problem_config1())
    for n_overlap in (1, 2):
        total = np.zeros(op.ndof)
        for idx, w in sw.subdomains_topo(op, n_overlap, normalise=False):
            np.add.at(total, idx, w)
        off = np.abs(total - 1.0) > 1e-12
        if n_overlap == 1:
            assert not off.any()
            continue
        assert off.any()
        elems = np.unique(np.searchsorted(op.offsets, np.flatnonzero(off), side="right") - 1)
        p = mesh["elem_p"]
        mixed = {int(mt["em"]) for mt in op.mortars if mt["ep"] >= 0 and p[mt["em"]] != p[mt["ep"]]}
        mixed |= {int(mt["ep"]) for mt in op.mortars if mt["ep"] >= 0 and p[mt["em"]] != p[mt["ep"]]}
        assert set(int(e) for e in elems) <= mixed
        total = np.zeros(op.ndof)
        for idx, w in sw.subdomains_topo(op, n_overlap):
            np.add.at(total, idx, w)
        assert np.allclose(total, 1.0, rtol=0, atol=1e-14)


def test_schwarz_multigrid_on_a_random_degree_cube():
    mesh = _mixed_degrees(meshgen.unit_cube(2, 2), [2, 3, 4], 1)
    prob = meshgen.problem_config1()
    its = {}
    for name, kw in (("schwarz", dict(n_cheb=3, smoother="schwarz", schwarz_overlap=2)),
                     ("point", dict(n_cheb=4, smoother="point"))):
        mg = Multigrid(mesh, prob, **kw)
        _, its[name], _ = fcg(mg.ops[0].apply, mg.ops[0].rhs(), mg.vcycle, tol=1e-10, max_iter=200)
    print("FCG iterations", its)
    assert its["schwarz"] <= 8 and its["point"] >= 3 * its["schwarz"]


BOX_2TO1 = {
    "box_2to1_p3": lambda: meshgen.box_grid((2, 1, 1), 1, 3, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5]),
    "box_2to1_l2_p2": lambda: meshgen.box_grid((1, 1, 1), 2, 2, refine=[lambda k, c0, c1: c1.max() <= 0.5]),
}


@pytest.mark.parametrize("name", ["cube_l2_p3", "box_lopsided_l1_p3", "cube_l2_p2to4"])
@pytest.mark.parametrize("n_overlap", [1, 2])
def test_subdomains_from_positions_equal_the_topological_ones_at_one_level(name, n_overlap):
    mesh = _mixed_degrees(meshgen.unit_cube(2, 2), [2, 3, 4], 1) if name == "cube_l2_p2to4" else MESHES[name]()
    op = SIPG(mesh, meshgen.problem_config1())
    for (i1, w1), (i2, w2) in zip(sw.subdomains_topo(op, n_overlap), sw.subdomains_boxes(op, n_overlap)):
        assert np.array_equal(np.sort(i1), np.sort(i2))
        assert np.allclose(w1[np.argsort(i1)], w2[np.argsort(i2)], rtol=0, atol=1e-14)


def test_subdomains_across_2to1_faces():
    # a box refined 2:1 on part of it: with one layer the weights sum to one everywhere (the
    # fine side's narrower width is shared by both sides of every 2:1 face); with two, the
    # points whose sum differs from one lie in cells at a 2:1 face; normalisation restores the
    # partition of unity
    mesh = BOX_2TO1["box_2to1_p3"]()
    op = SIPG(mesh, meshgen.problem_config1())
    lev = mesh["elem_level"]
    at_2to1 = {int(e) for mt in op.mortars if mt["ep"] >= 0 and lev[mt["em"]] != lev[mt["ep"]]
               for e in (mt["em"], mt["ep"])}
    for n_overlap in (1, 2):
        total = np.zeros(op.ndof)
        for idx, w in sw.subdomains_boxes(op, n_overlap, normalise=False):
            np.add.at(total, idx, w)
        off = np.abs(total - 1.0) > 1e-12
        assert off.any() == (n_overlap == 2)
        elems = np.searchsorted(op.offsets, np.flatnonzero(off), side="right") - 1
        assert {int(e) for e in elems} <= at_2to1
        total = np.zeros(op.ndof)
        for idx, w in sw.subdomains_boxes(op, n_overlap):
            np.add.at(total, idx, w)
        assert np.allclose(total, 1.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("name", list(BOX_2TO1))
def test_schwarz_multigrid_across_2to1_faces(name):
    mesh = BOX_2TO1[name]()
    prob = meshgen.problem_config1()
    its = {}
    for sm, kw in (("schwarz", dict(n_cheb=3, smoother="schwarz", schwarz_overlap=2)),
                   ("point", dict(n_cheb=4, smoother="point"))):
        mg = Multigrid(mesh, prob, **kw)
        _, its[sm], _ = fcg(mg.ops[0].apply, mg.ops[0].rhs(), mg.vcycle, tol=1e-10, max_iter=200)
    print(name, "FCG iterations", its)
    assert its["schwarz"] <= 6 and its["point"] >= 3 * its["schwarz"]
