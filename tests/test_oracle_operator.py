"""Pins for the oracle's SIPG operator (Eqs. lh2/Fh2, harald-stiff, temp-E, penaltyparameter).

Each pin is fixed by the mathematics, not by the oracle's own formulas:
* the matrix-free apply equals a brute-force assembled matrix built from the vector
  jump/average form of Eq. 20 (different algebra, same bilinear form);
* symmetry and positive definiteness of the SIPG form with an adequate penalty;
* A 1 = 0 with Neumann boundaries (constants are in the kernel of the broken
  gradient and have no jumps), on curved, 2:1 and variable-degree meshes;
* polynomial consistency: on affine meshes all integrals are exact, SIPG is
  consistent, so A u_I = F for u in Q_pmin with g = -lap u and g_D = u, also with Neumann
  data g_N = n.grad u on part of the boundary (Eq. NeumannBC); with Neumann data on all of
  it, the data satisfy the divergence theorem (F . 1 = 0);
* L2 convergence of order p + 1 for a smooth solution (the L2 rate of the
  adjoint-consistent SIPG method) and energy-norm convergence of order p (Eq. energynorm,
  the rate stated with Eq. expectedconvergence);
* the energy norm's closed forms: the H1 seminorm of sin(pi x) sin(pi y) sin(pi z) on the
  unit cube is 3 pi^2 / 8, and a constant u_h = 1 with u = 0 has only the Dirichlet-face
  penalty term 6 C p^2 N on N^3 cells;
* the element-diagonal blocks equal the diagonal blocks of the brute-force assembled matrix.
"""
import numpy as np
import pytest

import meshgen
from meshgen.problems import polynomial_problem
from oracle import problems as P
from oracle.operator import SIPG, assemble_dense, element_blocks
from oracle.solvers import Multigrid, fcg

MESHES = {
    "cube_p2": lambda: meshgen.unit_cube(1, 2),
    "box_2to1_p2": lambda: meshgen.box_grid((1, 1, 1), 1, 2,
                                            refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5]),
    "hp_var_p": lambda: meshgen.hp_sphere_cube(level=1, p_lo=1, p_hi=3, seed=2, r_cut=0.9),
    "shell_l1_p2": lambda: meshgen.cubed_sphere_shell(level=1, p=2, zeta_break=0.0, r_out=50.0),
    "shell_l1_p1": lambda: meshgen.cubed_sphere_shell(level=1, p=1, zeta_break=0.0, r_out=50.0),
    "skew_affine": lambda: _skew(),
}


def _skew():
    m = meshgen.box_grid((2, 1, 1), 1, 2)
    # shear both macros (still affine; faces still match)
    for i in range(len(m["macro_params"])):
        a0 = m["macro_params"][i, 3:6].copy()
        a2 = m["macro_params"][i, 9:12]
        m["macro_params"][i, 9:12] = a2 + 0.3 * np.array([1.0, 0.5, 0.0]) * a2[2]
        m["macro_params"][i, 0:3] = m["macro_params"][i, 0:3] + 0.0 * a0
    return m


@pytest.mark.parametrize("name", [k for k in MESHES if k != "shell_l1_p2"])
def test_matrix_free_equals_assembled_and_spd(name):
    m = MESHES[name]()
    op = SIPG(m, meshgen.problem_config1(), C=10.0)
    A = assemble_dense(op)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(op.ndof)
    y = op.apply(x)
    assert np.linalg.norm(y - A @ x) <= 1e-13 * np.linalg.norm(A @ x)
    assert np.max(np.abs(A - A.T)) <= 1e-13 * np.max(np.abs(A))
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() > 0


@pytest.mark.parametrize("name", ["shell_l1_p2", "hp_var_p", "box_2to1_p2"])
def test_symmetry_matrix_free(name):
    op = SIPG(MESHES[name](), meshgen.problem_config3(r0=0.4), C=10.0)
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal((2, op.ndof))
    a, b = x @ op.apply(y), y @ op.apply(x)
    assert abs(a - b) <= 1e-13 * (abs(a) + abs(b))


@pytest.mark.parametrize("name", ["shell_l1_p2", "hp_var_p", "box_2to1_p2", "skew_affine"])
def test_constants_in_kernel_with_neumann(name):
    op = SIPG(MESHES[name](), meshgen.problem_config3(r0=0.4), bc_override=2)
    one = np.ones(op.ndof)
    ref = np.abs(op.apply(np.random.default_rng(1).standard_normal(op.ndof))).max()
    assert np.abs(op.apply(one)).max() <= 1e-13 * ref


@pytest.mark.parametrize("name,deg", [("cube_p2", 2), ("box_2to1_p2", 2), ("hp_var_p", 1),
                                      ("skew_affine", 2)])
def test_polynomial_consistency(name, deg):
    # sheared cells map Q_p onto a larger space; total degree <= p is preserved by affine maps
    prob = polynomial_problem(deg, seed=7, total=(name == "skew_affine"))
    op = SIPG(MESHES[name](), prob)
    u = op.interpolate(lambda X: P.exact_u(prob, X))
    F = op.rhs()
    assert np.linalg.norm(op.apply(u) - F) <= 1e-13 * np.linalg.norm(F)


def test_polynomial_consistency_fails_with_planted_sign_error():
    # a flipped consistency term must break the consistency pin (guards the pin itself)
    prob = polynomial_problem(2, seed=7)
    op = SIPG(MESHES["box_2to1_p2"](), prob)
    for g in op.fgroups:
        g["mvec_m"] = -g["mvec_m"]
    u = op.interpolate(lambda X: P.exact_u(prob, X))
    F = op.rhs()
    assert np.linalg.norm(op.apply(u) - F) > 1e-6 * np.linalg.norm(F)


def _neumann_faces(m, faces):
    # the listed macro faces that lie on the boundary carry Neumann data (Eq. NeumannBC)
    m = dict(m)
    bc = np.array(m["macro_bc"], copy=True)
    for f in faces:
        bc[bc[:, f] == 1, f] = 2
    m["macro_bc"] = bc
    return m


@pytest.mark.parametrize("name,deg", [("cube_p2", 2), ("box_2to1_p2", 2), ("hp_var_p", 1),
                                      ("skew_affine", 2)])
def test_polynomial_consistency_with_neumann_faces(name, deg):
    # SIPG stays consistent with Neumann data g_N = n.grad u on part of the boundary: A u_I = F
    prob = polynomial_problem(deg, seed=11, total=(name == "skew_affine"))
    op = SIPG(_neumann_faces(MESHES[name](), (0, 3, 4)), prob)
    u = op.interpolate(lambda X: P.exact_u(prob, X))
    F = op.rhs()
    assert np.linalg.norm(op.apply(u) - F) <= 1e-13 * np.linalg.norm(F)


def test_neumann_consistency_fails_with_planted_sign_error(monkeypatch):
    # outward normal taken inward in the Neumann data: the consistency pin above must fail
    prob = polynomial_problem(2, seed=11)
    good = P.neumann_g
    monkeypatch.setattr(P, "neumann_g", lambda pr, x, n, k: good(pr, x, -n, k))
    op = SIPG(_neumann_faces(MESHES["box_2to1_p2"](), (0, 3, 4)), prob)
    u = op.interpolate(lambda X: P.exact_u(prob, X))
    F = op.rhs()
    assert np.linalg.norm(op.apply(u) - F) > 1e-6 * np.linalg.norm(F)


@pytest.mark.parametrize("name", ["cube_p2", "box_2to1_p2", "skew_affine"])
def test_pure_neumann_data_satisfy_divergence_theorem(name):
    # all faces Neumann: the constant test function (all ones in the LGL basis) sees
    # int g + int_boundary n.grad u = int (-lap u) + int n.grad u = 0 (exact quadrature)
    prob = polynomial_problem(2, seed=3, total=True)
    op = SIPG(_neumann_faces(MESHES[name](), range(6)), prob)
    F = op.rhs()
    src = SIPG(MESHES[name](), dict(prob, kind="polynomial")).rhs()  # scale: the source part alone
    assert abs(F.sum()) <= 1e-12 * np.abs(src).sum()


@pytest.mark.parametrize("prob", [dict(kind="sinsinsin", params=np.zeros(0)), polynomial_problem(3, seed=5)])
def test_grad_u_matches_differences_of_u(prob):
    rng = np.random.default_rng(0)
    x = rng.uniform(0.1, 0.9, (20, 3))
    h = 1e-5
    fd = np.stack([(P.exact_u(prob, x + h * e) - P.exact_u(prob, x - h * e)) / (2 * h) for e in np.eye(3)], -1)
    assert np.abs(P.grad_u(prob, x) - fd).max() <= 1e-8 * max(1.0, np.abs(fd).max())


def test_penalty_length_is_element_size():
    # uniform cube of N^3 cells on [0,1]^3: h_m = 1/N, sigma = C p^2 N
    N, p, C = 4, 3, 10.0
    op = SIPG(meshgen.unit_cube(2, p), meshgen.problem_config1(), C=C)
    for g in op.fgroups:
        np.testing.assert_allclose(g["sigma"], C * p * p * N, rtol=1e-14)
        np.testing.assert_allclose(g["wS"].sum(axis=1), 1.0 / N ** 2, rtol=1e-14)


def _solve_sin(level, p, norm="l2"):
    prob = meshgen.problem_config1()
    mg = Multigrid(meshgen.unit_cube(level, p), prob, n_cheb=4)
    op = mg.ops[0]
    u, it, hist = fcg(op.apply, op.rhs(), mg.vcycle, tol=1e-12)
    if norm == "energy":
        return op.energy_error(u, lambda X: P.exact_u(prob, X), lambda X: P.grad_u(prob, X))
    return op.l2_error(u, lambda X: P.exact_u(prob, X))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_l2_convergence_order(p):
    e1, e2 = _solve_sin(2, p), _solve_sin(3, p)
    rate = np.log2(e1 / e2)
    assert abs(rate - (p + 1)) < 0.35, rate


@pytest.mark.parametrize("p", [1, 2, 3])
def test_energy_convergence_order(p):
    # Eq. expectedconvergence: |u - u_h|_* <= C h^p for a smooth solution
    e1, e2 = _solve_sin(2, p, "energy"), _solve_sin(3, p, "energy")
    rate = np.log2(e1 / e2)
    print("energy rate p=%d: %.3f" % (p, rate))
    assert abs(rate - p) < 0.2, rate


def test_energy_norm_closed_forms():
    prob = meshgen.problem_config1()
    op = SIPG(meshgen.unit_cube(2, 3), prob)
    u_ex = lambda X: P.exact_u(prob, X)
    g_ex = lambda X: P.grad_u(prob, X)
    # u_h = 0: only the broken H1 seminorm of u (u vanishes on the boundary): 3 pi^2 / 8
    e = op.energy_error(np.zeros(op.ndof), u_ex, g_ex, extra=6)
    assert abs(e * e - 3 * np.pi ** 2 / 8) <= 1e-10 * 3 * np.pi ** 2 / 8
    # u_h = 1 and u = 0: no gradient and no interior jumps; each Dirichlet face has jump 1 and
    # sigma = C p^2 / h with h = 1/N: 6 C p^2 N
    zero = lambda X: np.zeros(X.shape[:-1])
    e = op.energy_error(np.ones(op.ndof), zero, lambda X: np.zeros(X.shape), extra=1)
    np.testing.assert_allclose(e * e, 6 * 10.0 * 9 * 4, rtol=1e-13)
    # a Q2 solution on a 2:1 mesh is reproduced exactly (consistency): zero energy error
    prob2 = meshgen.problems.polynomial_problem(2, seed=3)
    m = meshgen.box_grid((1, 1, 1), 1, 2, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5])
    op2 = SIPG(m, prob2)
    uI = op2.interpolate(lambda X: P.exact_u(prob2, X))
    e0 = op2.energy_error(uI, lambda X: P.exact_u(prob2, X), lambda X: P.grad_u(prob2, X))
    e1 = op2.energy_error(uI + 1e-3 * np.random.default_rng(0).standard_normal(op2.ndof),
                          lambda X: P.exact_u(prob2, X), lambda X: P.grad_u(prob2, X))
    assert e0 <= 1e-12 and e1 > 1e-4


@pytest.mark.parametrize("name", ["hp_var_p", "box_2to1_p2", "shell_l1_p2"])
def test_element_blocks_equal_assembled_diagonal_blocks(name):
    op = SIPG(MESHES[name](), meshgen.problem_config3(r0=0.7))
    A = assemble_dense(op)
    blocks = element_blocks(op)
    scale = np.abs(A).max()
    for e, B in enumerate(blocks):
        sl = slice(op.offsets[e], op.offsets[e + 1])
        np.testing.assert_allclose(B, A[sl, sl], rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("name", ["hp_var_p", "shell_l1_p1", "box_2to1_p2"])
def test_diagonal_equals_assembled_diagonal(name):
    op = SIPG(MESHES[name](), meshgen.problem_config3(r0=0.7))
    A = assemble_dense(op)
    np.testing.assert_allclose(op.diagonal(), np.diag(A), rtol=1e-13, atol=1e-14 * np.abs(A).max())


# ---- tabulated coefficients (per element, per node; a k that jumps across mortars) ----------

def _kfields(m, seed=0):
    """A per-element k and a per-node k (smooth inside each element, jumping across faces)."""
    rng = np.random.default_rng(seed)
    E = len(m["elem_p"])
    ke = rng.uniform(0.5, 4.0, E)
    n = m["elem_p"].astype(np.int64) + 1
    kn = np.concatenate([ke[e] * (1.0 + 0.3 * rng.uniform(-1, 1, n[e] ** 3)) for e in range(E)])
    return dict(where="element", values=ke), dict(where="node", values=kn)


@pytest.mark.parametrize("name", ["box_2to1_p2", "hp_var_p", "shell_l1_p1"])
def test_tabulated_k_matrix_free_equals_assembled_symmetric_spd(name):
    # per-side k on every mortar: the matrix-free apply, the brute-force assembly (vector jumps
    # and averages of Eq. 20 with {{k grad u}} = (k- grad u- + k+ grad u+)/2), the diagonal and
    # the element blocks agree; the form stays symmetric positive definite
    m = MESHES[name]()
    for kf in _kfields(m):
        op = SIPG(m, None, kfield=kf)
        A = assemble_dense(op)
        x = np.random.default_rng(1).standard_normal(op.ndof)
        np.testing.assert_allclose(op.apply(x), A @ x, rtol=1e-12, atol=1e-12 * np.abs(A @ x).max())
        np.testing.assert_allclose(A, A.T, atol=1e-12 * np.abs(A).max())
        assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
        np.testing.assert_allclose(op.diagonal(), np.diag(A), rtol=1e-12, atol=1e-14 * np.abs(A).max())
        for e, B in enumerate(element_blocks(op)):
            sl = slice(op.offsets[e], op.offsets[e + 1])
            np.testing.assert_allclose(B, A[sl, sl], atol=1e-12 * np.abs(A).max())


def test_tabulated_k_scaling_and_node_form():
    # k = 2 everywhere scales the whole form by 2 (volume, consistency terms and penalty); a
    # nodal field that is constant on each element equals the per-element field
    m = MESHES["box_2to1_p2"]()
    x = np.random.default_rng(2).standard_normal(meshgen.dof_count(m))
    y1 = SIPG(m, None).apply(x)
    E = len(m["elem_p"])
    np.testing.assert_allclose(SIPG(m, None, kfield=dict(where="element", values=np.full(E, 2.0))).apply(x), 2 * y1,
                               rtol=1e-13, atol=1e-13 * np.abs(y1).max())
    ke = np.random.default_rng(3).uniform(0.5, 3.0, E)
    n = m["elem_p"].astype(np.int64) + 1
    kn = np.repeat(ke, n ** 3)
    ya = SIPG(m, None, kfield=dict(where="element", values=ke)).apply(x)
    yb = SIPG(m, None, kfield=dict(where="node", values=kn)).apply(x)
    np.testing.assert_allclose(ya, yb, rtol=1e-13, atol=1e-13 * np.abs(ya).max())


@pytest.mark.parametrize("where", ["element", "node"])
def test_tabulated_k_constants_in_kernel_with_neumann(where):
    m = MESHES["shell_l1_p2"]()
    kf = _kfields(m)[0 if where == "element" else 1]
    op = SIPG(m, None, bc_override=2, kfield=kf)
    y = op.apply(np.ones(op.ndof))
    assert np.abs(y).max() <= 1e-12 * np.abs(op.diagonal()).max()


@pytest.mark.parametrize("maker", [
    lambda: meshgen.box_grid((1, 1, 1), 1, 2),
    lambda: meshgen.box_grid((1, 1, 1), 1, 1, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5]),
    lambda: meshgen.hp_sphere_cube(level=1, p_lo=1, p_hi=3, seed=2, r_cut=2.0),
])
def test_layered_k_consistency(maker):
    # k = 1 for x < 0.5 and 5 beyond (element-aligned jump): u piecewise linear in x with a
    # continuous flux solves -div(k grad u) = 0; SIPG with per-side k is consistent, so
    # A u_I = F exactly on affine meshes (every integral exact, u in Q_p on each element)
    m = maker()
    lo = np.min(m["macro_params"][:, 0:3], axis=0)
    hi = lo + np.array([m["macro_params"][0, 3], m["macro_params"][0, 7], m["macro_params"][0, 11]])
    x0 = 0.5 * (lo[0] + hi[0])
    prob = dict(kind="layered_x", params=np.array([x0, 1.0, 5.0]))
    cells = (m["elem_anchor"][:, 0] + 0.5) / (2.0 ** m["elem_level"])
    kf = dict(where="element", values=np.where(lo[0] + cells * (hi[0] - lo[0]) < x0, 1.0, 5.0))
    op = SIPG(m, prob, kfield=kf)
    uI = op.interpolate(lambda X: P.exact_u(prob, X))
    F = op.rhs()
    r = op.apply(uI) - F
    assert np.abs(r).max() <= 1e-12 * np.abs(F).max(), np.abs(r).max() / np.abs(F).max()
    # a single k on both sides of the jump (the larger one) breaks consistency
    bad = SIPG(m, prob, kfield=kf)
    for g in bad.fgroups:
        g["kp"] = g["kx"] = np.maximum(g["kx"], g["kp"]) if "ep" in g else g["kx"]
    rb = bad.apply(uI) - bad.rhs()
    assert np.abs(rb).max() > 1e-6 * np.abs(F).max()


def test_tabulated_fields_coarsen_to_the_hierarchy():
    # per element: mean over the cells inside; per node: injection, which reproduces a
    # field that is a polynomial of the coarse degree
    from oracle.solvers import Multigrid
    m = meshgen.unit_cube(2, 2)
    E = len(m["elem_p"])
    ke = np.arange(E, dtype=float) + 1.0
    mg = Multigrid(m, None, lam=[1.0] * 10, kfield=dict(where="element", values=ke))
    assert abs(np.mean(mg.ops[1].kfield["values"]) - np.mean(ke)) <= 1e-13 * np.mean(ke)
    f = lambda X: 1.0 + X[..., 0] + 2 * X[..., 1] * X[..., 2]
    op0 = SIPG(m, None)
    mg = Multigrid(m, None, lam=[1.0] * 10, kfield=dict(where="node", values=op0.interpolate(f)))
    for op in mg.ops[1:]:
        np.testing.assert_allclose(op.kfield["values"], SIPG(op.mesh, None).interpolate(f), atol=1e-13)


# ---- Robin boundary data (Eq. RobinBC, read with the sign of Eq. lh) ----------------------

def _robin_faces(m, faces):
    m = dict(m)
    bc = np.array(m["macro_bc"], copy=True)
    for f in faces:
        bc[bc[:, f] == 1, f] = 3
    m["macro_bc"] = bc
    return m


@pytest.mark.parametrize("name,deg", [("cube_p2", 2), ("box_2to1_p2", 2), ("hp_var_p", 1), ("skew_affine", 2)])
def test_polynomial_consistency_with_robin_faces(name, deg):
    # k n.grad u + gamma u = g_R on some faces: the form gains int gamma u v there and F gains
    # int g_R v; SIPG stays consistent, so A u_I = F for u in Q_p
    prob = polynomial_problem(deg, seed=12, total=(name == "skew_affine"))
    op = SIPG(_robin_faces(MESHES[name](), (1, 2, 5)), prob, robin_gamma=2.5)
    u = op.interpolate(lambda X: P.exact_u(prob, X))
    F = op.rhs()
    assert np.linalg.norm(op.apply(u) - F) <= 1e-13 * np.linalg.norm(F)


def test_robin_consistency_fails_with_planted_gamma_sign(monkeypatch):
    # gamma u subtracted in the data: the consistency pin must fail
    prob = polynomial_problem(2, seed=12)
    good = P.robin_u
    monkeypatch.setattr(P, "robin_u", lambda pr, x: -good(pr, x))
    op = SIPG(_robin_faces(MESHES["box_2to1_p2"](), (1, 2, 5)), prob, robin_gamma=2.5)
    u = op.interpolate(lambda X: P.exact_u(prob, X))
    F = op.rhs()
    assert np.linalg.norm(op.apply(u) - F) > 1e-6 * np.linalg.norm(F)


@pytest.mark.parametrize("name", ["box_2to1_p2", "shell_l1_p2", "hp_var_p"])
def test_robin_form_assembled_symmetric_spd(name):
    # all faces Robin (gamma > 0): no Dirichlet face, the form is still SPD; matrix-free,
    # brute-force assembly, diagonal and element blocks agree
    m = _robin_faces(MESHES[name](), range(6))
    op = SIPG(m, meshgen.problem_config3(r0=0.7), robin_gamma=1.5)
    A = assemble_dense(op)
    x = np.random.default_rng(3).standard_normal(op.ndof)
    np.testing.assert_allclose(op.apply(x), A @ x, rtol=1e-12, atol=1e-12 * np.abs(A @ x).max())
    np.testing.assert_allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
    np.testing.assert_allclose(op.diagonal(), np.diag(A), rtol=1e-12, atol=1e-14 * np.abs(A).max())
    for e, B in enumerate(element_blocks(op)):
        sl = slice(op.offsets[e], op.offsets[e + 1])
        np.testing.assert_allclose(B, A[sl, sl], atol=1e-12 * np.abs(A).max())
    # with gamma = 0 the Robin faces are Neumann faces: A 1 = 0
    op0 = SIPG(m, None, robin_gamma=0.0)
    assert np.abs(op0.apply(np.ones(op0.ndof))).max() <= 1e-12 * np.abs(op0.diagonal()).max()
