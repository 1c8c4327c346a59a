"""GPU parity of hpdg_set_coefficient (the coefficients k and c of -div(k grad u) + c u = g):

* a per-node k (varying inside elements, jumping across faces) on a curved 2:1 shell: every
  multigrid level's apply against the oracle with the same table (coarse levels by injection);
* a per-element k with an element-aligned jump: the solve reproduces the piecewise-linear
  solution of the layered problem (SIPG with each side's own k is consistent);
* a per-node mass coefficient c on a mesh with the mass form: the apply against the oracle;
* the analytic placement equals the upload-time coefficient; error paths.
"""
import numpy as np
import pytest

import meshgen
from oracle import problems as P
from oracle.operator import SIPG
from oracle.solvers import Multigrid
from tests.gpu_common import MESHES, TOL_APPLY, TOL_ROW, dof_perm, rel, row_err

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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _node_field(m, seed, lo=0.5, hi=4.0, spread=0.3):
    rng = np.random.default_rng(seed)
    n = m["elem_p"].astype(np.int64) + 1
    ke = rng.uniform(lo, hi, len(n))
    return np.concatenate([ke[e] * (1.0 + spread * rng.uniform(-1, 1, n[e] ** 3)) for e in range(len(n))])


def _all_levels(M, mg, label):
    rng = np.random.default_rng(0)
    for l in range(M.n_levels):
        op = mg.ops[l]
        perm = dof_perm(M.level_cells(l), op.mesh)
        x = rng.standard_normal(op.ndof)
        y_or = op.apply(x)[perm]
        xd = torch.tensor(x[perm], device="cuda")
        yd = torch.zeros_like(xd)
        M.apply(xd, yd, level=l)
        yh = host(yd)
        err, erow = rel(yh, y_or), row_err(yh, y_or, op.diagonal()[perm], x)
        print(label, "level", l, "ndof", op.ndof, "rel", err, "per-row", erow, flush=True)
        assert err <= TOL_APPLY and erow <= TOL_ROW, (l, err, erow)


def test_node_k_on_curved_2to1_shell_all_levels(ctx):
    maker, prob = MESHES["shell_l2_p3_r1e3"]
    m = maker()
    kn = _node_field(m, 4)
    M = ctx.upload(m)
    M.set_coefficient("diffusion", "node", kn)
    mg = Multigrid(m, prob, n_cheb=2, lam=[1.0] * 40, jacobi=False, kfield=dict(where="node", values=kn))
    assert M.n_levels == mg.nlevels
    _all_levels(M, mg, "node k shell")
    M.free()


def test_element_k_all_levels_and_layered_solve(ctx):
    m = meshgen.box_grid((1, 1, 1), 1, 2, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5])
    # all levels with a random per-element k (coarse levels: the mean over the cells inside)
    ke = np.random.default_rng(5).uniform(0.5, 4.0, len(m["elem_p"]))
    M = ctx.upload(m)
    M.set_coefficient("diffusion", "element", ke)
    mg = Multigrid(m, None, n_cheb=2, lam=[1.0] * 40, jacobi=False, kfield=dict(where="element", values=ke))
    _all_levels(M, mg, "element k box")
    # layered k = 1 / 5 across x = 1/2: u is piecewise linear with a continuous flux, so the
    # discrete solution is its interpolant (F from the oracle, which tests may pass in)
    prob = dict(kind="layered_x", params=np.array([0.5, 1.0, 5.0]))
    cells = (m["elem_anchor"][:, 0] + 0.5) / (2.0 ** m["elem_level"])
    kl = np.where(cells < 0.5, 1.0, 5.0)
    M.set_coefficient("diffusion", "element", kl)
    M.setup_smoother(n_cheb=4, smoother="point")
    op = SIPG(m, prob, kfield=dict(where="element", values=kl))
    F = torch.tensor(op.rhs(), device="cuda")
    u = torch.zeros_like(F)
    st = M.solve(F, u, tol=1e-12, max_iter=300)
    uI = op.interpolate(lambda X: P.exact_u(prob, X))
    err = np.abs(host(u) - uI).max() / np.abs(uI).max()
    print("layered k solve", st, "max error vs interpolant", err, flush=True)
    assert err <= 1e-9
    M.free()


def test_node_mass_coefficient(ctx):
    maker, prob = MESHES["hp_k"]
    m = maker()
    cn = _node_field(m, 6, lo=0.0, hi=3.0, spread=0.5)
    M = ctx.upload(m, coef=hp.coef_from_problem(prob), mass_term=True, build_f32=True)
    M.set_coefficient("mass", "node", cn)
    mg = Multigrid(m, prob, n_cheb=2, lam=[1.0] * 40, jacobi=False, cfield=dict(where="node", values=cn))
    _all_levels(M, mg, "node c hp")
    # a solve with the mass term reaches the oracle's residual
    M.setup_smoother(n_cheb=4, smoother="point")
    op = mg.ops[0]
    Fo = op.rhs()
    F = torch.tensor(Fo, device="cuda")
    u = torch.zeros_like(F)
    st = M.solve(F, u, tol=5e-11, max_iter=400, precision=hp.PREC_MIXED)
    res = np.linalg.norm(Fo - op.apply(host(u))) / np.linalg.norm(Fo)
    print("mass solve", st, "oracle residual", res, flush=True)
    assert res <= 1e-10
    M.free()


def test_analytic_placement_and_errors(ctx):
    maker, prob = MESHES["hp_k"]
    m = maker()
    A = ctx.upload(m, coef=hp.coef_from_problem(prob))
    B = ctx.upload(m)
    r0, k_in, k_out = prob["params"][:3]
    B.set_coefficient("diffusion", "analytic", params=[hp.COEF_RADIAL_STEP, r0, k_in, k_out, 0.0])
    x = torch.tensor(np.random.default_rng(1).standard_normal(A.n_dof[0]), device="cuda")
    ya, yb = torch.zeros_like(x), torch.zeros_like(x)
    A.apply(x, ya)
    B.apply(x, yb)
    assert torch.equal(ya, yb)
    with pytest.raises(hp.HpdgError) as ei:
        B.set_coefficient("mass", "element", np.ones(A.n_elem[0]))
    assert ei.value.code == hp.ERR_UNSUPPORTED
    with pytest.raises(hp.HpdgError) as ei:
        B.set_coefficient("diffusion", "element", -np.ones(A.n_elem[0]))
    assert ei.value.code == hp.ERR_INVALID_ARG
    A.free()
    B.free()
