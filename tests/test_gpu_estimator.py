"""GPU parity of the a posteriori estimator (Eqs. Eta2_Ingredients, Eta2_Integrals, Eta2_Local)
against the oracle's, element by element, on affine, 2:1, mixed-degree, variable-k, curved and
mass-term meshes."""
import numpy as np
import pytest

import meshgen
from oracle import estimator as est
from oracle import problems as P
from oracle.operator import SIPG
from tests.gpu_common import MESHES, coef_of, dof_perm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

hp = pytest.importorskip("paper_1907_01572_amd")

# per element: |gpu - oracle| <= TOL_EST_REL eta2 + TOL_EST_ABS max(eta2).  Both sides evaluate
# the same point sums in FP64; the residual R = g + div(k grad u) - c u and the jumps are
# differences of O(1) terms, so their rounding is relative to the terms, not to R
TOL_EST_REL = 1e-10
TOL_EST_ABS = 1e-12


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = hp.Context(0)
    yield c
    c.close()


def elem_perm(lib_cells, mesh):
    """Index array: library element e of level 0 is oracle element perm[e]."""
    key = {(int(mesh["elem_macro"][e]), int(mesh["elem_level"][e]), *map(int, mesh["elem_anchor"][e])): e
           for e in range(len(mesh["elem_p"]))}
    return np.array([key[(int(lib_cells["elem_macro"][e]), int(lib_cells["elem_level"][e]),
                          *map(int, lib_cells["elem_anchor"][e]))] for e in range(len(lib_cells["elem_p"]))])


def _vector(op, prob, seed, noise):
    u = op.interpolate(lambda x: P.exact_u(prob, x))
    return u + noise * np.random.default_rng(seed).standard_normal(op.ndof) * max(np.abs(u).max(), 1.0)


def _compare(M, m, op, prob, u_o, label, fiducial=None):
    cells = M.level_cells(0)
    perm = dof_perm(cells, m)
    ep = elem_perm(cells, m)
    u = torch.tensor(u_o[perm], device="cuda")
    eta2 = torch.zeros(M.n_elem[0], dtype=torch.float64, device="cuda")
    vol = torch.zeros_like(eta2)
    M.estimate(prob, u, eta2, vol)
    torch.cuda.synchronize()
    ref = est.estimate(op, u_o, prob, fiducial=fiducial)
    g, gv = eta2.cpu().numpy(), vol.cpu().numpy()
    o, ov = ref["eta2"][ep], ref["eta2_vol"][ep]
    err = np.max(np.abs(g - o) / (TOL_EST_REL * o + TOL_EST_ABS * o.max()))
    errv = np.max(np.abs(gv - ov) / (TOL_EST_REL * ov + TOL_EST_ABS * max(ov.max(), 1e-300)))
    print(label, "eta total", np.sqrt(o.sum()), "volume share", ov.sum() / o.sum(),
          "max err / tol", err, errv, flush=True)
    assert err <= 1.0 and errv <= 1.0
    return eta2


@pytest.mark.parametrize("name", ["cube_l2_p3", "box_2to1_p3", "box_macros_p2", "hp_k", "hp_p2_7_k1",
                                  "shell_l2_p3_r1e3"])
@pytest.mark.parametrize("noise", [0.0, 0.1])
def test_estimator_parity(ctx, name, noise):
    maker, prob = MESHES[name]
    m = maker()
    op = SIPG(m, prob)
    M = ctx.upload(m, coef=coef_of(prob))
    _compare(M, m, op, prob, _vector(op, prob, 5, noise), "%s noise %g" % (name, noise))
    M.free()


def test_estimator_parity_mass_term_and_repeat(ctx):
    # c u enters R (the shell harmonic problem with c = 1 on an affine box); a second problem on
    # the same mesh rebuilds the point data; a repeated call is bit-identical (no atomics)
    m = meshgen.box_grid((1, 1, 1), 1, 3, lo=(1.0, 1.0, 1.0), hi=(3.0, 3.0, 3.0))
    prob = meshgen.problem_config2(1.0)
    M = ctx.upload(m, mass_term=True)
    M.set_coefficient("mass", "analytic", params=[1.0])
    op = SIPG(m, prob, mass=lambda x: np.ones(x.shape[:-1]))
    u_o = _vector(op, prob, 7, 0.05)
    a = _compare(M, m, op, prob, u_o, "mass term")
    b = _compare(M, m, op, prob, u_o, "mass term again")
    assert torch.equal(a, b)
    M.free()
    prob2 = meshgen.problem_config1()
    M = ctx.upload(m)
    op2 = SIPG(m, prob2)
    _compare(M, m, op2, prob, _vector(op2, prob, 8, 0.05), "first problem")
    _compare(M, m, op2, prob2, _vector(op2, prob2, 8, 0.05), "second problem")
    M.free()


def test_estimator_refuses_bad_arguments(ctx):
    maker, prob = MESHES["cube_l2_p3"]
    M = ctx.upload(maker())
    u = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
    eta2 = torch.zeros(M.n_elem[0], dtype=torch.float64, device="cuda")
    with pytest.raises(hp.HpdgError) as ei:
        M.estimate(dict(kind="sinsinsin", params=np.zeros(0)), u, eta2, eta2)
    assert ei.value.code == hp.ERR_INVALID_ARG
    M.free()


def _linear_shell_twin(mesh, r_in=2.0, r_out=3.0):
    """The cells of a (compactified) shell under the linear radial map from r_in to r_out."""
    out = dict(mesh)
    par = np.array(mesh["macro_params"], float, copy=True)
    par[:, 9] = 0.0  # linear radial map
    par[:, 10], par[:, 11] = r_in, r_out
    out["macro_params"] = par
    return out


def _scaled_box(mesh, s):
    out = dict(mesh)
    par = np.array(mesh["macro_params"], float, copy=True)
    par[:, 0:12] *= s
    out["macro_params"] = par
    return out


@pytest.mark.parametrize("name,twin", [("shell_l2_p4_r1e9", _linear_shell_twin),
                                       ("shell_l2_p3_r1e3", _linear_shell_twin),
                                       ("box_2to1_p3", lambda m: _scaled_box(m, 3.0)),
                                       ("hp_k", lambda m: _scaled_box(m, 0.5))])
def test_estimator_parity_on_a_fiducial_grid(ctx, name, twin):
    # the compactified estimator of the shell (integrals on an unstretched twin with radii 2..3)
    # and scaled twins of affine meshes; resetting the grid restores the physical estimate
    maker, prob = MESHES[name]
    m = maker()
    op = SIPG(m, prob)
    M = ctx.upload(m, coef=coef_of(prob))
    u_o = _vector(op, prob, 9, 0.05)
    phys = _compare(M, m, op, prob, u_o, name + " physical grid")
    fid = twin(m)
    M.set_estimator_grid(fid)
    comp = _compare(M, m, op, prob, u_o, name + " fiducial grid", fiducial=fid)
    assert not torch.equal(comp, phys)
    M.set_estimator_grid(None)
    again = _compare(M, m, op, prob, u_o, name + " physical grid again")
    assert torch.equal(again, phys)
    other = meshgen.box_grid((1, 1, 2), 0, 2)  # two macros stacked in z: other connectivity
    with pytest.raises(hp.HpdgError) as ei:
        M.set_estimator_grid(other)
    assert ei.value.code == hp.ERR_INVALID_MESH
    M.free()


def test_compact_estimator_moves_the_marks_inwards(ctx):
    # the library's estimates of the interpolated solution on the shell compactified to r = 1e9:
    # marking the largest 10% picks the stretched outer cells on the physical grid and the inner
    # cells on the unstretched twin (Sec. III.C)
    maker, prob = MESHES["shell_l2_p4_r1e9"]
    m = maker()
    op = SIPG(m, prob)
    M = ctx.upload(m, coef=coef_of(prob))
    u = torch.tensor(op.interpolate(lambda x: P.exact_u(prob, x))[dof_perm(M.level_cells(0), m)], device="cuda")
    cells = M.level_cells(0)
    zc = -1 + (2 * cells["elem_anchor"][:, 2] + 1) / 2.0 ** cells["elem_level"]
    eta2 = torch.zeros(M.n_elem[0], dtype=torch.float64, device="cuda")
    shares = []
    for grid in (None, _linear_shell_twin(m)):
        M.set_estimator_grid(grid)
        M.estimate(prob, u, eta2)
        marked = hp.amr_mark(eta2.cpu().numpy(), hp.MARK_FRACTION, 0.1)
        shares.append(float(np.mean(zc[marked] > 0)))
    print("share of marked cells in the outer half: physical grid", shares[0], "twin", shares[1], flush=True)
    assert shares[0] > 0.8 and shares[1] == 0.0
    M.free()
