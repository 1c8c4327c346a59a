"""Full-size GPU checks on the three large workloads, sampled against the oracle.

At the workload sizes the oracle evaluates only the rows of a seeded sample of elements
(``SIPG(active=...)``: their volume terms and every mortar touching them), which is exact
for those rows.  The library runs the whole mesh in the same configuration as the
benchmark (FP64 level 0, FP32 copies built).

* cubed-sphere shell, p = 5, 1,244,160 DOF: operator rows;
* hp cube with k jump, p = 2..7, 8,649,651 DOF: operator rows, and the mixed-precision
  solve reaches 1e-10 (true residual by an FP64 apply) with its sampled residual rows
  matching the oracle's;
* puncture mesh, p = 6, 12,739,363 DOF: nonlinear residual rows and, after
  linearisation, Jacobian rows;
* the shell's first coarse level (1,056 cells): operator rows;
* the a posteriori estimate per sampled element (hp cube; shell on its unstretched twin);
* the shell's smoother as the benchmark runs it (the fused apply + block-Jacobi step)
  against the separate kernels, FP64 and FP32, fine and first coarse level, and a V-cycle.
"""
import numpy as np
import pytest

import meshgen
from oracle import estimator as est
from oracle import problems
from oracle.newton import _gl_values, _project
from oracle.operator import SIPG
from tests.gpu_common import TOL_APPLY, TOL_APPLY_COMPACTIFIED, coef_of

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

hp = pytest.importorskip("paper_1907_01572_amd")

N_SAMPLE = 48


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = hp.Context(0)
    yield c
    c.close()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def sample_rows(op, elems):
    return np.concatenate([np.arange(op.offsets[e], op.offsets[e + 1]) for e in elems])


def rel_rows(a, b, rows):
    return float(np.linalg.norm(a[rows] - b[rows]) / np.linalg.norm(b[rows]))


def _sample(E, seed):
    return np.sort(np.random.default_rng(seed).choice(E, N_SAMPLE, replace=False))


@pytest.mark.parametrize("name", ["shell_p5", "hp_k_p2_7"])
def test_fullsize_apply_rows(ctx, name):
    if name == "shell_p5":
        m, prob, tol = meshgen.cubed_sphere_shell(level=3, p=5), meshgen.problem_config2(), TOL_APPLY_COMPACTIFIED
    else:
        m, prob, tol = meshgen.hp_sphere_cube(), meshgen.problem_config3(), TOL_APPLY
    print(name, "upload", len(m["elem_p"]), "elements", flush=True)
    M = ctx.upload(m, coef=coef_of(prob), build_f32=True)
    elems = _sample(len(m["elem_p"]), 1)
    op = SIPG(m, prob, active=elems)
    x = np.random.default_rng(2).standard_normal(op.ndof)
    xd = torch.tensor(x, device="cuda")
    y = torch.zeros_like(xd)
    M.apply(xd, y)
    rows = sample_rows(op, elems)
    err = rel_rows(host(y), op.apply(x), rows)
    y32 = torch.zeros(op.ndof, dtype=torch.float32, device="cuda")
    M.apply(xd.float(), y32)
    err32 = rel_rows(host(y32), host(y), rows)
    print(name, "sampled rows FP64", err, "FP32 vs FP64", err32, flush=True)
    assert err <= tol and err32 <= 1e-5
    M.free()


def _linear_twin(m):
    out = dict(m)
    par = np.array(m["macro_params"], float, copy=True)
    par[:, 9], par[:, 10], par[:, 11] = 0.0, 2.0, 3.0  # linear radial map from 2 to 3
    out["macro_params"] = par
    return out


@pytest.mark.parametrize("name", ["shell_p5_compact", "hp_k_p2_7"])
def test_fullsize_estimator_rows(ctx, name):
    # the a posteriori estimate at the benchmark's sizes, per sampled element against the
    # oracle's (its volume part and every mortar touching it): the hp cube on its physical grid,
    # the compactified shell on its unstretched twin (Sec. III.C)
    if name == "shell_p5_compact":
        m, prob = meshgen.cubed_sphere_shell(level=3, p=5), meshgen.problem_config2()
        fid = _linear_twin(m)
    else:
        m, prob, fid = meshgen.hp_sphere_cube(), meshgen.problem_config3(), None
    M = ctx.upload(m, coef=coef_of(prob), build_f32=True)
    if fid is not None:
        M.set_estimator_grid(fid)
    elems = _sample(len(m["elem_p"]), 4)
    op = SIPG(m, prob, active=elems)
    x = np.random.default_rng(5).standard_normal(op.ndof)
    eta2 = torch.zeros(M.n_elem[0], dtype=torch.float64, device="cuda")
    M.estimate(prob, torch.tensor(x, device="cuda"), eta2)
    ref = est.estimate(op, x, prob, fiducial=fid)["eta2"][elems]
    got = host(eta2)[elems]
    err = float(np.max(np.abs(got - ref) / ref))
    print(name, "sampled estimates", len(elems), "max rel error", err, flush=True)
    assert err <= 1e-10
    M.free()


def test_fullsize_hp_mixed_solve(ctx):
    m, prob = meshgen.hp_sphere_cube(), meshgen.problem_config3()
    M = ctx.upload(m, coef=coef_of(prob), build_f32=True)
    M.setup_smoother(smoother="point", n_cheb=4)
    N = M.n_dof[0]
    F = torch.zeros(N, dtype=torch.float64, device="cuda")
    M.assemble_rhs(prob, F)
    u = torch.zeros_like(F)
    st = M.solve(F, u, tol=1e-10, max_iter=500, precision=hp.PREC_MIXED)
    r = torch.zeros_like(F)
    M.apply(u, r)
    r = F - r
    true_rel = float(torch.linalg.norm(r) / torch.linalg.norm(F))
    elems = _sample(len(m["elem_p"]), 3)
    op = SIPG(m, prob, active=elems)
    rows = sample_rows(op, elems)
    uh = host(u)
    r_or = op.rhs()[rows] - op.apply(uh)[rows]
    err_rows = float(np.linalg.norm(host(r)[rows] - r_or) / np.linalg.norm(host(F)[rows]))
    ex = op.interpolate(lambda x: problems.exact_u(prob, x))
    err_u = float(np.abs(uh[rows] - ex[rows]).max() / np.abs(ex[rows]).max())
    print("hp mixed solve", st, "true residual", true_rel, "sampled residual rows vs oracle", err_rows,
          "nodal error vs exact u on the sample", err_u, flush=True)
    assert true_rel <= 1e-10 and err_rows <= 1e-13
    M.free()


@pytest.mark.timeout(400)
def test_fullsize_shell_solve_residual_rows(ctx):
    # the shell solve as the benchmark runs it (4 levels, block-Jacobi Chebyshev with
    # N_Cheb = 26 and Lambda = 600, FCG to 1e-10), FP64 and mixed: the true residual by an FP64
    # apply, and the residual rows of a seeded element sample recomputed by the oracle
    m, prob = meshgen.cubed_sphere_shell(level=3, p=5), meshgen.problem_config2()
    M = ctx.upload(m, coef=coef_of(prob), build_f32=True, max_levels=4)
    M.setup_smoother(n_cheb=26, Lambda=600.0, smoother="block")
    N = M.n_dof[0]
    F = torch.zeros(N, dtype=torch.float64, device="cuda")
    M.assemble_rhs(prob, F)
    elems = _sample(len(m["elem_p"]), 5)
    op = SIPG(m, prob, active=elems)
    rows = sample_rows(op, elems)
    Fo = op.rhs()
    Fh = host(F)
    assert np.linalg.norm(Fh[rows] - Fo[rows]) <= TOL_APPLY * np.linalg.norm(Fo[rows])
    for prec in (hp.PREC_F64, hp.PREC_MIXED):
        u = torch.zeros_like(F)
        st = M.solve(F, u, tol=1e-10, max_iter=200, precision=prec)
        r = torch.zeros_like(F)
        M.apply(u, r)
        r = F - r
        true_rel = float(torch.linalg.norm(r) / torch.linalg.norm(F))
        uh = host(u)
        r_or = Fo[rows] - op.apply(uh)[rows]
        err_rows = float(np.linalg.norm(host(r)[rows] - r_or) / np.linalg.norm(Fo[rows]))
        ex = op.interpolate(lambda x: problems.exact_u(prob, x))
        err_u = float(np.abs(uh[rows] - ex[rows]).max() / np.abs(ex[rows]).max())
        print("shell solve prec", prec, st, "true residual", true_rel, "sampled residual rows vs oracle", err_rows,
              "nodal error vs exact u on the sample", err_u, flush=True)
        assert true_rel <= 1e-10 and err_rows <= 1e-12
    M.free()


def test_fullsize_puncture_residual_and_jacobian_rows(ctx):
    nl = meshgen.puncture_problem()
    m = meshgen.puncture_mesh(punctures=nl["params"][1:].reshape(-1, 5)[:, :3])
    print("puncture upload", len(m["elem_p"]), "elements", flush=True)
    M = ctx.upload(m, mass_term=True, build_f32=True)
    M.setup_smoother(smoother="point")
    elems = _sample(len(m["elem_p"]), 5)
    op = SIPG(m, None, mass=lambda x: np.zeros(x.shape[:-1]), active=elems)
    rng = np.random.default_rng(6)
    u = 0.05 * rng.standard_normal(op.ndof)
    ud = torch.tensor(u, device="cuda")
    R = torch.zeros_like(ud)
    M.nonlinear_residual(nl, ud, R)
    # oracle rows: A u - N(u) on the sampled elements
    N = np.zeros(op.ndof)
    for g in op.vgroups:
        a, b = problems.nl_alpha_beta(nl, g["x"])
        N[g["idx"]] += _project(g, g["W"] * g["det"] * b * (1.0 + a * _gl_values(g, u)) ** -7)
        g["M"] = g["W"] * g["det"] * 7.0 * a * b * (1.0 + a * _gl_values(g, u)) ** -8
    Au = np.zeros(op.ndof)
    saved = [g["M"] for g in op.vgroups]
    for g in op.vgroups:
        g["M"] = None
    Au = op.apply(u)
    for g, s in zip(op.vgroups, saved):
        g["M"] = s
    rows = sample_rows(op, elems)
    e_res = rel_rows(host(R), Au - N, rows)
    M.linearize(nl, ud)
    v = rng.standard_normal(op.ndof)
    y = torch.zeros_like(ud)
    M.apply(torch.tensor(v, device="cuda"), y)
    e_jac = rel_rows(host(y), op.apply(v), rows)
    print("puncture sampled rows: residual", e_res, "Jacobian", e_jac, flush=True)
    assert e_res <= TOL_APPLY and e_jac <= TOL_APPLY
    M.free()


def test_fullsize_shell_level1_apply_rows(ctx):
    # level 1 of the shell (1,056 cells at p = 5), the first coarse level of the bench's V-cycle,
    # against the oracle on the same coarse cells
    m, prob = meshgen.cubed_sphere_shell(level=3, p=5), meshgen.problem_config2()
    M = ctx.upload(m, coef=coef_of(prob), build_f32=True, max_levels=4)
    cells = M.level_cells(1)
    m1 = dict(m)
    for k in ("elem_macro", "elem_level", "elem_anchor", "elem_p"):
        m1[k] = np.ascontiguousarray(cells[k])
    elems = _sample(len(m1["elem_p"]), 3)
    op = SIPG(m1, prob, active=elems)
    assert op.ndof == M.n_dof[1]
    x = np.random.default_rng(4).standard_normal(op.ndof)
    xd = torch.tensor(x, device="cuda")
    y = torch.zeros_like(xd)
    M.apply(xd, y, level=1)
    rows = sample_rows(op, elems)
    err = rel_rows(host(y), op.apply(x), rows)
    print("shell level 1:", len(m1["elem_p"]), "cells, sampled rows FP64", err, flush=True)
    assert err <= TOL_APPLY_COMPACTIFIED
    M.free()


def test_fullsize_shell_fused_smoothing_matches_separate_kernels(ctx):
    # the bench's smoother on the bench's mesh and hierarchy: block-Jacobi Chebyshev steps as
    # one fused kernel per element (the timed path) against the separate apply and block
    # kernels (whose apply rows are checked against the oracle above), on the fine level and
    # the first coarse level, FP64 and FP32, and one V-cycle
    m, prob = meshgen.cubed_sphere_shell(level=3, p=5), meshgen.problem_config2()
    M = ctx.upload(m, coef=coef_of(prob), build_f32=True, max_levels=4)
    rng = np.random.default_rng(5)
    vecs = {l: rng.standard_normal((2, M.n_dof[l])) for l in (0, 1)}
    r = rng.standard_normal(M.n_dof[0])
    out, lam = {}, None
    for fused in (True, False):
        M.setup_smoother(n_cheb=26, Lambda=600.0, smoother="block", fused=fused, lambda_max=lam)
        lam = M.lambda_max
        M.timing_enable(1)
        res = {}
        for dt in (torch.float64, torch.float32):
            for l in (0, 1):
                b, x0 = vecs[l]
                x = torch.tensor(x0, dtype=dt, device="cuda")
                M.smooth(torch.tensor(b, dtype=dt, device="cuda"), x, level=l, n_iter=4)
                res[(dt, l)] = host(x)
            z = torch.zeros(M.n_dof[0], dtype=dt, device="cuda")
            M.vcycle(torch.tensor(r, dtype=dt, device="cuda"), z)
            res[(dt, "v")] = host(z)
        fused_launches = M.kernel_timing("smooth", 0, hp.F64)[1]
        M.timing_enable(0)
        out[fused] = (res, fused_launches)
    assert out[True][1] > 0 and out[False][1] == 0
    for key, a in out[True][0].items():
        b = out[False][0][key]
        err = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        tol = 1e-13 if key[0] == torch.float64 else 1e-5
        print("shell fused vs separate", key, err, flush=True)
        assert err <= tol, key
    M.free()
