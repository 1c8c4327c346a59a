"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

* apply: relative L2 <= 1e-12 on conforming, 2:1, variable-degree + variable-k and curved
  meshes; compactified shells at r_out = 1e9 to the derived bound in gpu_common;
* every multigrid level's apply, the smoother and the V-cycle with the oracle's spectral
  bounds; the RHS; transfers via the V-cycle;
* solves (FCG and PCG, FP64 and mixed) reach 1e-10 relative residual recomputed by the
  oracle; determinism (bitwise repeatable applies and solves); error paths.
"""
import numpy as np
import pytest

import meshgen
from oracle import problems as P
from oracle.operator import SIPG
from oracle.solvers import Multigrid, chebyshev, fgmres
from oracle.operator import assemble_dense
from oracle.solvers import cg_lanczos, gershgorin_max, splitmix64_uniform
from tests.gpu_common import (MESHES, TOL_APPLY, TOL_APPLY_COMPACTIFIED, TOL_ROW, TOL_ROW_COMPACTIFIED, coef_of,
                               dof_perm, rel, row_err)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

hp = pytest.importorskip("paper_1907_01572_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = hp.Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _tol(name):
    return TOL_APPLY_COMPACTIFIED if name.endswith("r1e9") else TOL_APPLY


@pytest.mark.parametrize("name", list(MESHES))
def test_apply_parity_all_levels(ctx, name):
    maker, prob = MESHES[name]
    m = maker()
    print("case", name, flush=True)
    M = ctx.upload(m, coef=coef_of(prob))
    mg = Multigrid(m, prob, n_cheb=2, lam=[1.0] * 40, jacobi=False)
    assert M.n_levels == mg.nlevels
    rng = np.random.default_rng(0)
    for l in range(M.n_levels):
        op = mg.ops[l]
        perm = dof_perm(M.level_cells(l), op.mesh)
        x = rng.standard_normal(op.ndof)
        y_or = op.apply(x)[perm]
        xd = dev(x[perm])
        yd = torch.zeros_like(xd)
        M.apply(xd, yd, level=l)
        yh = host(yd)
        err = rel(yh, y_or)
        dg = op.diagonal()[perm]
        erow = row_err(yh, y_or, dg, x)
        # where the worst row is: its element (library order), local node and cell
        worst = int(np.argmax(np.abs(yh - y_or) / np.abs(dg)))
        cells = M.level_cells(l)
        offs = np.concatenate([[0], np.cumsum((cells["elem_p"].astype(np.int64) + 1) ** 3)])
        ew = int(np.searchsorted(offs, worst, side="right") - 1)
        print("  level", l, "ndof", op.ndof, "rel", err, "per-row", erow, "worst row: element", ew, "node",
              worst - offs[ew], "level", cells["elem_level"][ew], "anchor", cells["elem_anchor"][ew],
              "|dy|", abs(yh[worst] - y_or[worst]), "|y|", abs(y_or[worst]), "diag", dg[worst], flush=True)
        assert err <= _tol(name) and erow <= (TOL_ROW_COMPACTIFIED if name.endswith("r1e9") else TOL_ROW), (l, err, erow)
    M.free()


@pytest.mark.parametrize("name", ["cube_l2_p3", "hp_k", "shell_l2_p3_r1e3"])
def test_apply_f32_close_to_f64(ctx, name):
    maker, prob = MESHES[name]
    m = maker()
    M = ctx.upload(m, coef=coef_of(prob), build_f32=True)
    x = np.random.default_rng(1).standard_normal(M.n_dof[0])
    y64 = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
    y32 = torch.zeros(M.n_dof[0], dtype=torch.float32, device="cuda")
    M.apply(dev(x), y64)
    M.apply(dev(x, torch.float32), y32)
    err = rel(host(y32), host(y64))
    print("f32 vs f64", name, err, flush=True)
    assert err < 1e-5
    M.free()


def test_rhs_parity(ctx):
    for name in ["cube_l2_p3", "hp_k", "shell_l2_p3_r1e3"]:
        maker, prob = MESHES[name]
        m = maker()
        M = ctx.upload(m, coef=coef_of(prob))
        F = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
        M.assemble_rhs(prob, F)
        Fo = SIPG(m, prob).rhs()
        err = rel(host(F), Fo)
        print("rhs", name, err, flush=True)
        assert err <= TOL_APPLY
        M.free()


def _neumann_faces(m, faces):
    m = dict(m)
    bc = np.array(m["macro_bc"], copy=True)
    for f in faces:
        bc[bc[:, f] == 1, f] = 2
    m["macro_bc"] = bc
    return m


def test_rhs_parity_with_neumann_faces(ctx):
    # Neumann data g_N = k n.grad u (Eq. NeumannBC) on three of the six sides
    probs = [meshgen.polynomial_problem(2, seed=11), dict(kind="sinsinsin", params=np.zeros(0)),
             meshgen.gaussian_problem(n=4, seed=1)]
    for name in ["box_2to1_p3", "shell_l2_p3_r1e3"]:
        m = _neumann_faces(MESHES[name][0](), (0, 3, 4))
        for prob in probs:
            M = ctx.upload(m)
            F = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
            M.assemble_rhs(prob, F)
            op = SIPG(m, prob)
            err = rel(host(F), op.rhs()[dof_perm(M.level_cells(0), op.mesh)])
            print("rhs with Neumann faces", name, prob["kind"], err, flush=True)
            assert err <= TOL_APPLY
            M.free()


def test_rhs_neumann_faces_refuse_kinds_without_data(ctx):
    m = _neumann_faces(MESHES["box_2to1_p3"][0](), (0,))
    M = ctx.upload(m)
    F = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError):
        M.assemble_rhs(meshgen.problem_config2(), F)  # the shell harmonic has no Neumann data here
    M.free()


def test_solve_with_neumann_faces_reproduces_polynomial(ctx):
    # affine 2:1 box, u in Q_2, Dirichlet on three sides and Neumann on the others: SIPG is
    # consistent, so the discrete solution is the interpolant of u
    m = _neumann_faces(meshgen.box_grid((1, 1, 1), 1, 2, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5]),
                       (0, 3, 4))
    prob = meshgen.polynomial_problem(2, seed=11)
    M = ctx.upload(m)
    M.setup_smoother(n_cheb=4, smoother="block")
    F = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
    M.assemble_rhs(prob, F)
    u = torch.zeros_like(F)
    st = M.solve(F, u, tol=1e-12, max_iter=300)
    op = SIPG(m, prob)
    ui = op.interpolate(lambda X: P.exact_u(prob, X))[dof_perm(M.level_cells(0), op.mesh)]
    err = np.abs(host(u) - ui).max() / np.abs(ui).max()
    print("Neumann solve", st, "max err vs interpolant", err, flush=True)
    assert err <= 1e-9
    M.free()


def _robin_faces(m, faces):
    m = dict(m)
    bc = np.array(m["macro_bc"], copy=True)
    for f in faces:
        bc[bc[:, f] == 1, f] = 3
    m["macro_bc"] = bc
    return m


@pytest.mark.parametrize("name", ["box_2to1_p3", "shell_l2_p3_r1e3"])
def test_robin_faces_apply_all_levels_and_rhs(ctx, name):
    # Robin faces k n.grad u + gamma u = g_R (Eq. RobinBC): int gamma u v in the operator on every
    # level, int g_R v in the right-hand side
    m = _robin_faces(MESHES[name][0](), (1, 2, 5))
    M = ctx.upload(m, robin_gamma=2.5)
    mg = Multigrid(m, None, n_cheb=2, lam=[1.0] * 40, jacobi=False, robin_gamma=2.5)
    rng = np.random.default_rng(4)
    for l in range(M.n_levels):
        op = mg.ops[l]
        perm = dof_perm(M.level_cells(l), op.mesh)
        x = rng.standard_normal(op.ndof)
        y = torch.zeros(op.ndof, dtype=torch.float64, device="cuda")
        M.apply(dev(x[perm]), y, level=l)
        yo = op.apply(x)[perm]
        err, erow = rel(host(y), yo), row_err(host(y), yo, op.diagonal()[perm], x)
        print(name, "Robin level", l, "rel", err, "per-row", erow, flush=True)
        assert err <= TOL_APPLY and erow <= TOL_ROW
    for prob in [meshgen.polynomial_problem(2, seed=12), dict(kind="sinsinsin", params=np.zeros(0)),
                 meshgen.gaussian_problem(n=4, seed=2)]:
        F = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
        M.assemble_rhs(prob, F)
        op = SIPG(m, prob, robin_gamma=2.5)
        err = rel(host(F), op.rhs()[dof_perm(M.level_cells(0), op.mesh)])
        print(name, "Robin rhs", prob["kind"], err, flush=True)
        assert err <= TOL_APPLY
    M.free()


def test_solve_with_robin_faces_reproduces_polynomial(ctx):
    # affine 2:1 box, u in Q_2, Dirichlet on three sides and Robin on the others: the discrete
    # solution is the interpolant (SIPG with Robin data is consistent)
    m = _robin_faces(meshgen.box_grid((1, 1, 1), 1, 2, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5]),
                     (1, 2, 5))
    prob = meshgen.polynomial_problem(2, seed=12)
    M = ctx.upload(m, robin_gamma=2.5)
    M.setup_smoother(n_cheb=4, smoother="block")
    F = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
    M.assemble_rhs(prob, F)
    u = torch.zeros_like(F)
    st = M.solve(F, u, tol=1e-12, max_iter=300)
    op = SIPG(m, prob, robin_gamma=2.5)
    ui = op.interpolate(lambda X: P.exact_u(prob, X))[dof_perm(M.level_cells(0), op.mesh)]
    err = np.abs(host(u) - ui).max() / np.abs(ui).max()
    print("Robin solve", st, "max err vs interpolant", err, flush=True)
    assert err <= 1e-9
    M.free()


def test_rhs_parity_with_mass_term(ctx):
    # a mass term raises the volume rule to n + 1 points; flat faces of a one-degree level
    # then run with that rule too, but Dirichlet data that are not polynomials must still be
    # integrated with the face's own n-point rule
    m = meshgen.box_grid((1, 1, 1), 1, 2, lo=(-32.0,) * 3, hi=(32.0,) * 3)
    for prob in [meshgen.problem_config2(), meshgen.star_problem(0.001, 4.0)[1]]:
        M = ctx.upload(m, mass_term=True)
        F = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
        M.assemble_rhs(prob, F)
        Fo = SIPG(m, prob).rhs()
        perm = dof_perm(M.level_cells(0), SIPG(m, prob).mesh)
        err = rel(host(F), Fo[perm])
        print("rhs with mass term", prob["kind"], err, flush=True)
        assert err <= TOL_APPLY
        M.free()


@pytest.mark.parametrize("name,smoother", [("cube_l2_p3", "none"), ("hp_k", "point"),
                                           ("shell_l2_p3_r1e3", "point"), ("hp_k", "block"),
                                           ("shell_l2_p3_r1e3", "block"), ("cube_l1_p6", "block"),
                                           ("cube_l1_p7", "block"), ("hp_p2_7_k1", "point"),
                                           ("box_macros_p2", "point")])
def test_smoother_and_vcycle_parity(ctx, name, smoother):
    maker, prob = MESHES[name]
    m = maker()
    mg = Multigrid(m, prob, n_cheb=3, smoother=smoother)
    M = ctx.upload(m, coef=coef_of(prob))
    lam = M.setup_smoother(n_cheb=3, smoother=smoother, lambda_max=mg.lam)
    np.testing.assert_allclose(lam, mg.lam)
    rng = np.random.default_rng(2)
    op = mg.ops[0]
    b, x0 = rng.standard_normal((2, op.ndof))
    xs = chebyshev(op.apply, b, x0, mg.lam[0], mg.Lambda, 5, mg.minv[0])
    xd = dev(x0)
    M.smooth(dev(b), xd, level=0, n_iter=5)
    e1 = rel(host(xd), xs)
    r = rng.standard_normal(op.ndof)
    z = torch.zeros(op.ndof, dtype=torch.float64, device="cuda")
    M.vcycle(dev(r), z)
    e2 = rel(host(z), mg.vcycle(r))
    print("smooth", e1, "vcycle", e2, flush=True)
    assert e1 <= 1e-12 and e2 <= 1e-11
    M.free()


def test_element_centric_path_used(ctx):
    # affine axis-aligned constant-k meshes run entirely element-centrically (the mortar kernel
    # only for 2:1 faces); a variable-k mesh mixes the two paths; curved meshes use the element
    # and mortar kernels only
    for name, expect in (("cube_l2_p3", "all"), ("box_macros_p2", "all"), ("hp_p2_7_k1", "all+2:1"),
                         ("hp_k", "mixed"), ("shell_l2_p3_r1e3", "none")):
        maker, prob = MESHES[name]
        M = ctx.upload(maker(), coef=coef_of(prob))
        ec, tasks, ne = M.n_elem_centric, M.n_mortar_tasks, M.n_elem
        print(name, "element-centric", ec, "of", ne, "mortar tasks", tasks, flush=True)
        if expect == "all":
            assert ec == ne and all(t == 0 for t in tasks)
        elif expect == "all+2:1":
            assert ec == ne and tasks[0] > 0
        elif expect == "none":
            assert all(v == 0 for v in ec) and tasks[0] > 0
        else:
            assert 0 < ec[0] < ne[0] and tasks[0] > 0
        M.free()
    # by level (the default outside the tests): small mixed-degree levels keep the element and
    # mortar kernels, one-degree levels take the element-centric apply; never: none anywhere
    for name, mode, expect in (("hp_p2_7_k1", hp.EC_AUTO, "none"), ("cube_l2_p3", hp.EC_ALWAYS, "all"),
                               ("cube_l2_p3", hp.EC_NEVER, "none")):
        maker, prob = MESHES[name]
        M = ctx.upload(maker(), coef=coef_of(prob), ec_mode=mode)
        ec = M.n_elem_centric
        print(name, "mode", mode, "element-centric", ec, flush=True)
        if expect == "all":
            assert ec == M.n_elem
        elif expect == "none":
            assert all(v == 0 for v in ec)
        M.free()
    # by level on a one-degree mesh of 8192 cells (next level 1024): the element-centric apply on
    # the finest level only
    M = ctx.upload(meshgen.uniform_box((2, 1, 1), 4, 2), ec_mode=hp.EC_AUTO, max_levels=2)
    print("box 2x1x1 level 4: element-centric", M.n_elem_centric, "of", M.n_elem, flush=True)
    assert M.n_elem_centric[0] == M.n_elem[0] == 8192 and M.n_elem_centric[1] == 0
    M.free()


@pytest.mark.parametrize("name", ["cube_l2_p3", "hp_p2_7_k1"])
def test_apply_parity_without_element_centric(ctx, name):
    # the element and mortar kernels alone (EC_NEVER) on meshes the element-centric apply covers
    maker, prob = MESHES[name]
    m = maker()
    M = ctx.upload(m, coef=coef_of(prob), ec_mode=hp.EC_NEVER)
    op = SIPG(m, prob)
    perm = dof_perm(M.level_cells(0), m)
    x = np.random.default_rng(5).standard_normal(op.ndof)
    y_or = op.apply(x)[perm]
    xd = dev(x[perm])
    yd = torch.zeros_like(xd)
    M.apply(xd, yd)
    err = rel(host(yd), y_or)
    print(name, "rel", err, flush=True)
    assert err <= TOL_APPLY
    M.free()


@pytest.mark.parametrize("name,smoother", [("shell_l2_p3_r1e3", "block"), ("cube_l1_p7", "block"),
                                           ("shell_l2_p3_r1e3", "point"), ("hp_k", "point"),
                                           ("hp_p2_7_k1", "point"), ("box_macros_p2", "point")])
def test_fused_block_step_matches_separate_kernels(ctx, name, smoother):
    # on one-degree levels each Jacobi-scaled Chebyshev step that needs A x runs as one kernel
    # per element; the arithmetic is the separate kernels' (the block partial sums may be
    # taken by a different number of waves, so FP32 agrees to rounding)
    maker, prob = MESHES[name]
    m = maker()
    out = {}
    for fused in (True, False):
        M = ctx.upload(m, coef=coef_of(prob), build_f32=True)
        M.setup_smoother(n_cheb=3, smoother=smoother, fused=fused, lambda_max=out.get("lam"))
        out["lam"] = M.lambda_max
        n = M.n_dof[0]
        b, x0, r = np.random.default_rng(3).standard_normal((3, n))
        M.timing_enable(1)
        res = {}
        for dt in (torch.float64, torch.float32):
            # one fused step (no trace hand-off), two (one hand-off), four
            xs = []
            for n_iter in (1, 2, 4):
                x = torch.tensor(x0, dtype=dt, device="cuda")
                M.smooth(torch.tensor(b, dtype=dt, device="cuda"), x, level=0, n_iter=n_iter)
                xs.append(host(x))
            z = torch.zeros(n, dtype=dt, device="cuda")
            M.vcycle(torch.tensor(r, dtype=dt, device="cuda"), z)
            res[dt] = (np.concatenate(xs), host(z))
        launches = {k: M.kernel_timing(k, 0, hp.F64)[1] for k in ("smooth", "block")}
        M.timing_enable(0)
        ec = M.n_elem_centric[0] > 0
        out[fused] = (res, launches)
        M.free()
    (rf, lf), (ru, lu) = out[True], out[False]
    print(name, "launches fused", lf, "separate", lu, flush=True)
    if ec and smoother == "block":
        # element-centric levels fuse only the point-Jacobi step: block smoothing keeps the
        # apply and the block step apart there
        assert lf["smooth"] == 0 and lu["smooth"] == 0
    else:
        # the fused path ran (smoothing from a given x, and every V-cycle step but the first of
        # each pre-smoothing), the separate one never did
        assert lf["smooth"] > 0 and lu["smooth"] == 0
        if smoother == "block":
            assert lu["block"] > lf["block"]
    for dt, tol in ((torch.float64, 1e-13), (torch.float32, 1e-5)):
        ex, ez = rel(rf[dt][0], ru[dt][0]), rel(rf[dt][1], ru[dt][1])
        print(name, dt, "smooth", ex, "vcycle", ez, flush=True)
        assert ex <= tol and ez <= tol


def _oracle_starts(M, mg, seed):
    """Alg. 5 start vectors of the library (SplitMix64 in its DOF order) in the oracle's order."""
    starts = []
    for l, op in enumerate(mg.ops[:-1]):
        perm = dof_perm(M.level_cells(l), op.mesh)
        b = np.zeros(op.ndof)
        b[perm] = splitmix64_uniform(op.ndof, seed)
        starts.append(b)
    return starts


@pytest.mark.parametrize("name,smoother", [("hp_k", "point"), ("hp_k", "block"), ("cube_l2_p3", "none"),
                                           ("shell_l2_p3_r1e3", "block"), ("box_2to1_p3", "point")])
def test_cg_spectral_bound_matches_oracle(ctx, name, smoother):
    # Alg. 5 from the same start vector (the library's SplitMix64 values, permuted into the
    # oracle's element order): the same preconditioned CG, so the Gershgorin bounds of the two
    # Lanczos tridiagonals agree to rounding on every smoothed level
    maker, prob = MESHES[name]
    m = maker()
    M = ctx.upload(m, coef=coef_of(prob))
    lam = M.setup_smoother(n_cheb=3, smoother=smoother, seed=11)
    mg = Multigrid(m, prob, n_cheb=3, smoother=smoother, lam=[1.0] * 40)
    mg.refresh(15, 11, starts=_oracle_starts(M, mg, 11))
    print(name, smoother, "lambda gpu", lam, "oracle", mg.lam, flush=True)
    np.testing.assert_allclose(lam, mg.lam, rtol=1e-10)
    M.free()


@pytest.mark.parametrize("maker,smoother", [
    (lambda: meshgen.box_grid((1, 1, 1), 1, 2, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5]), "point"),
    (lambda: meshgen.box_grid((1, 1, 1), 1, 2, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5]), "block"),
    (lambda: meshgen.cubed_sphere_shell(level=0, p=2, r_out=50.0), "block"),
    (lambda: meshgen.hp_sphere_cube(level=1, p_lo=1, p_hi=3, seed=2, r_cut=0.9), "none"),
])
def test_spectral_bound_is_an_upper_bound(ctx, maker, smoother):
    # the library's bound of every smoothed level is >= lambda_max(M^-1 A) from a dense
    # generalised eigen-solve of the oracle's assembled operator (tiny meshes)
    import scipy.linalg
    from oracle.operator import element_blocks
    m = maker()
    prob = meshgen.problem_config3(r0=0.7)
    M = ctx.upload(m, coef=coef_of(prob))
    lam = M.setup_smoother(n_cheb=3, smoother=smoother)
    mg = Multigrid(m, prob, n_cheb=3, smoother=smoother, lam=[1.0] * 40)
    for l, op in enumerate(mg.ops[:-1]):
        A = assemble_dense(op)
        A = 0.5 * (A + A.T)
        if smoother == "point":
            Mm = np.diag(np.diag(A))
        elif smoother == "block":
            Mm = scipy.linalg.block_diag(*element_blocks(op))
        else:
            Mm = np.eye(op.ndof)
        lmax = scipy.linalg.eigh(A, Mm, eigvals_only=True).max()
        print("level", l, "bound", lam[l], "lambda_max(M^-1 A)", lmax, flush=True)
        assert lam[l] >= lmax * (1 - 1e-12)
    M.free()


@pytest.mark.parametrize("name,solver,prec", [
    ("cube_l2_p3", hp.SOLVER_FCG, hp.PREC_F64),
    ("cube_l2_p3", hp.SOLVER_PCG, hp.PREC_F64),
    ("hp_k", hp.SOLVER_FCG, hp.PREC_F64),
    ("hp_k", hp.SOLVER_FCG, hp.PREC_MIXED),
    ("shell_l2_p3_r1e3", hp.SOLVER_FCG, hp.PREC_F64),
    ("shell_l2_p3_r1e3", hp.SOLVER_FCG, hp.PREC_MIXED),
    ("shell_l2_p4_r1e9", hp.SOLVER_FCG, hp.PREC_F64),
    ("shell_l2_p3_r1e3", hp.SOLVER_FCG, hp.PREC_MIXED_BF16),
    ("shell_l2_p4_r1e9", hp.SOLVER_FCG, hp.PREC_MIXED_BF16),
])
def test_solve_reaches_oracle_residual(ctx, name, solver, prec):
    maker, prob = MESHES[name]
    m = maker()
    M = ctx.upload(m, coef=coef_of(prob), build_f32=(prec != hp.PREC_F64))
    M.setup_smoother(n_cheb=4, smoother="block" if name.startswith("shell") else "point")
    F = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
    M.assemble_rhs(prob, F)
    u = torch.zeros_like(F)
    st = M.solve(F, u, tol=5e-11, max_iter=400, solver=solver, precision=prec)
    op = SIPG(m, prob)
    Fo = op.rhs()
    uh = host(u)
    res = np.linalg.norm(Fo - op.apply(uh)) / np.linalg.norm(Fo)
    print(name, "solver", solver, "prec", prec, st, "oracle residual", res, flush=True)
    assert res <= 1e-10
    M.free()


def test_determinism_bitwise(ctx):
    maker, prob = MESHES["hp_k"]
    M = ctx.upload(maker(), coef=coef_of(prob))
    M.setup_smoother(n_cheb=3)
    x = dev(np.random.default_rng(3).standard_normal(M.n_dof[0]))
    y1, y2 = torch.zeros_like(x), torch.zeros_like(x)
    M.apply(x, y1)
    M.apply(x, y2)
    assert torch.equal(y1, y2)
    F = torch.zeros_like(x)
    M.assemble_rhs(prob, F)
    u1, u2 = torch.zeros_like(x), torch.zeros_like(x)
    M.solve(F, u1, tol=1e-10)
    M.solve(F, u2, tol=1e-10)
    assert torch.equal(u1, u2)
    M.free()


def test_error_paths(ctx):
    # unbalanced (4:1) mesh is rejected
    import itertools
    m = meshgen.box_grid((1, 1, 1), 1, 2)
    # level-1 cells except (1,1,1); that one split into level-2 cells, of which (2,2,2) is
    # split again: its level-3 children touch the level-1 cell (0,1,1) across x = 1/2 (4:1)
    cells = [(0, 1, a, 2) for a in itertools.product((0, 1), repeat=3) if a != (1, 1, 1)]
    cells += [(0, 2, tuple(2 + np.array(c)), 2) for c in itertools.product((0, 1), repeat=3)
              if c != (0, 0, 0)]
    cells += [(0, 3, tuple(4 + np.array(c)), 2) for c in itertools.product((0, 1), repeat=3)]
    bad = dict(m)
    bad["elem_macro"] = np.array([c[0] for c in cells], np.int32)
    bad["elem_level"] = np.array([c[1] for c in cells], np.int32)
    bad["elem_anchor"] = np.array([c[2] for c in cells], np.int32)
    bad["elem_p"] = np.array([c[3] for c in cells], np.int32)
    with pytest.raises(hp.HpdgError) as ei:
        ctx.upload(bad)
    assert ei.value.code == hp.ERR_INVALID_MESH
    # degree outside the supported range
    big = dict(m)
    big["elem_p"] = np.full_like(m["elem_p"], 16)
    with pytest.raises(hp.HpdgError) as ei:
        ctx.upload(big)
    assert ei.value.code == hp.ERR_INVALID_MESH
    # iteration cap and non-finite right-hand side
    maker, prob = MESHES["cube_l2_p3"]
    M = ctx.upload(maker())
    M.setup_smoother()
    F = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
    M.assemble_rhs(prob, F)
    u = torch.zeros_like(F)
    st = M.solve(F, u, tol=1e-12, max_iter=1, raise_on_error=False)
    assert st["status"] == hp.ERR_NOT_CONVERGED and st["iterations"] == 1
    F[5] = float("nan")
    st = M.solve(F, torch.zeros_like(F), raise_on_error=False)
    assert st["status"] == hp.ERR_BREAKDOWN
    M.free()


def test_budget_admission(ctx):
    small = hp.Context(0, hbm_budget_bytes=1 << 16)
    maker, prob = MESHES["cube_l2_p3"]
    with pytest.raises(hp.HpdgError) as ei:
        small.upload(maker())
    assert ei.value.code == hp.ERR_OOM
    small.close()


def test_coarse_level_too_large_for_dense_solve(ctx):
    # one level of 82,944 DOF: its dense matrix has more than 2^31 entries; the mesh still
    # applies (the coarse inverse is formed by the solver setup, which refuses it)
    M = ctx.upload(meshgen.cubed_sphere_shell(level=2, p=5), max_levels=1)
    x = torch.ones(M.n_dof[0], dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    M.apply(x, y)
    with pytest.raises(hp.HpdgError) as ei:
        M.setup_smoother()
    assert ei.value.code == hp.ERR_UNSUPPORTED
    M.free()


def test_coarse_chebyshev_degree(ctx):
    # fewer Chebyshev steps below the finest level: a different V-cycle, same converged solution
    maker, prob = MESHES["shell_l2_p3_r1e3"]
    m = maker()
    M = ctx.upload(m)
    M.setup_smoother(n_cheb=4, smoother="block")
    r = dev(np.random.default_rng(5).standard_normal(M.n_dof[0]))
    z1, z2 = torch.zeros_like(r), torch.zeros_like(r)
    M.vcycle(r, z1)
    M.setup_smoother(n_cheb=4, smoother="block", n_cheb_coarse=2, lambda_max=M.lambda_max)
    M.vcycle(r, z2)
    assert not torch.equal(z1, z2)
    F = torch.zeros_like(r)
    M.assemble_rhs(prob, F)
    u = torch.zeros_like(F)
    st = M.solve(F, u, tol=5e-11, max_iter=400)
    op = SIPG(m, prob)
    Fo = op.rhs()
    res = np.linalg.norm(Fo - op.apply(host(u))) / np.linalg.norm(Fo)
    print("n_cheb_coarse=2", st, "oracle residual", res, flush=True)
    assert res <= 1e-10
    M.free()


@pytest.mark.parametrize("name,prec,restart", [
    ("shell_l2_p3_r1e3", hp.PREC_F64, 30),
    ("cube_l2_p3", hp.PREC_F64, 3),
    ("hp_k", hp.PREC_MIXED, 30),
])
def test_fgmres_reaches_oracle_residual(ctx, name, prec, restart):
    # restarted flexible GMRES: the solution's residual recomputed by the oracle, and (FP64,
    # the oracle's V-cycle with the same frozen bounds) the iteration count of the oracle's
    # flexible GMRES
    maker, prob = MESHES[name]
    m = maker()
    smoother = "block" if name.startswith("shell") else "point"
    mg = Multigrid(m, prob, n_cheb=4, smoother=smoother)
    M = ctx.upload(m, coef=coef_of(prob), build_f32=(prec != hp.PREC_F64))
    M.setup_smoother(n_cheb=4, smoother=smoother, lambda_max=mg.lam)
    F = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
    M.assemble_rhs(prob, F)
    u = torch.zeros_like(F)
    st = M.solve(F, u, tol=5e-11, max_iter=400, solver=hp.SOLVER_FGMRES, precision=prec, restart=restart)
    op = mg.ops[0]
    Fo = op.rhs()
    res = np.linalg.norm(Fo - op.apply(host(u))) / np.linalg.norm(Fo)
    msg = "%s restart %d prec %d: %s, oracle residual %.3e" % (name, restart, prec, st, res)
    if prec == hp.PREC_F64:
        uo, ko, hist = fgmres(op.apply, Fo, mg.vcycle, tol=5e-11, max_iter=400, restart=restart)
        msg += ", oracle FGMRES %d iterations" % ko
        assert abs(st["iterations"] - ko) <= 2, msg
    print(msg, flush=True)
    assert res <= 1e-10, msg
    M.free()


@pytest.mark.timeout(400)
def test_shell_p5_bench_smoother_settings_against_oracle(ctx):
    # the benchmark's smoother configuration on a small compactified shell with 2:1 faces:
    # p = 5, r_out = 1e9, block-Jacobi Chebyshev with N_Cheb = 26, Lambda = 600; the library
    # runs its fused apply + block step (the FP64 kernel instantiation the benchmark times);
    # smoothing and the V-cycle against the oracle with the library's bounds, and the FP32
    # V-cycle (the mixed preconditioner) against the FP64 oracle V-cycle
    m = meshgen.cubed_sphere_shell(level=1, p=5)
    prob = meshgen.problem_config2()
    M = ctx.upload(m, coef=coef_of(prob), build_f32=True)
    lam = M.setup_smoother(n_cheb=26, Lambda=600.0, smoother="block")
    print("shell p=5 levels", M.n_dof, "lambda", lam, flush=True)
    mg = Multigrid(m, prob, n_cheb=26, Lambda=600.0, smoother="block", lam=list(lam))
    assert mg.nlevels == M.n_levels
    op = mg.ops[0]
    rng = np.random.default_rng(8)
    b, x0, r = rng.standard_normal((3, op.ndof))
    M.timing_enable(1)
    xd = dev(x0)
    M.smooth(dev(b), xd, level=0, n_iter=26)
    fused = M.kernel_timing("smooth", 0, hp.F64)[1]
    M.timing_enable(0)
    xs = chebyshev(op.apply, b, x0, mg.lam[0], mg.Lambda, 26, mg.minv[0])
    e1 = rel(host(xd), xs)
    zo = mg.vcycle(r)
    z = torch.zeros(op.ndof, dtype=torch.float64, device="cuda")
    M.vcycle(dev(r), z)
    e2 = rel(host(z), zo)
    z32 = torch.zeros(op.ndof, dtype=torch.float32, device="cuda")
    M.vcycle(dev(r, torch.float32), z32)
    e3 = rel(host(z32), zo)
    # both sides invert the element blocks in FP64, each to about kappa(A_ee) eps relative; the
    # difference enters every one of the 26 steps: bound n_cheb kappa_max eps, times 10
    from oracle.operator import element_blocks
    kmax = max(np.linalg.cond(B) for B in element_blocks(op))
    tol_s = 10 * 26 * kmax * np.finfo(float).eps
    print("fused launches", fused, "smooth", e1, "(bound %.2e, kappa_max %.3e)" % (tol_s, kmax), "vcycle", e2,
          "FP32 vcycle vs FP64 oracle", e3, flush=True)
    assert fused >= 25
    assert e1 <= max(1e-12, tol_s) and e2 <= max(1e-11, tol_s) and e3 <= 1e-4
    M.free()
