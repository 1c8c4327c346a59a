"""GPU tests of the continuous-batching solve server.

* a mix of requests (cube / hp + k / shell meshes, degrees 2..5, Poisson and variable k,
  Gaussian-sum sources) submitted at once runs concurrently (requests in flight together) and
  gives, for every request,
  the same result as solving it alone through the mesh API (the kernels and reductions are
  deterministic and private to a request), and each reaches the 1e-10 residual;
* admission by device footprint: with a budget that holds one request at a time, no two
  requests are in flight together, and all finish;
* the mixed-precision server reaches the same tolerance.
"""
import numpy as np
import pytest

import meshgen
from oracle.operator import SIPG

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


def _mix():
    out = []
    for i, (maker, prob) in enumerate([
        (lambda: meshgen.unit_cube(2, 3), meshgen.gaussian_problem(lo=(0, 0, 0), hi=(1, 1, 1), seed=1)),
        (lambda: meshgen.unit_cube(3, 2), meshgen.gaussian_problem(lo=(0, 0, 0), hi=(1, 1, 1), seed=2)),
        (lambda: meshgen.hp_sphere_cube(level=2, p_lo=2, p_hi=4, seed=3, r_cut=0.6), meshgen.problem_config3(r0=0.6)),
        (lambda: meshgen.cubed_sphere_shell(level=1, p=4, r_out=3.0, radial_kind=0), meshgen.problem_config2()),
        (lambda: meshgen.unit_cube(2, 5), meshgen.gaussian_problem(lo=(0, 0, 0), hi=(1, 1, 1), seed=5)),
        (lambda: meshgen.hp_sphere_cube(level=2, p_lo=2, p_hi=3, seed=6, r_cut=0.4), meshgen.problem_config3(r0=0.4)),
    ]):
        out.append((maker(), prob))
    return out


def _alone(ctx, mesh, prob, precision):
    M = ctx.upload(mesh, coef=hp.coef_from_problem(prob), build_f32=(precision == hp.PREC_MIXED))
    M.setup_smoother(n_cheb=4, smoother="point", Lambda=20.0)
    F = torch.zeros(M.n_dof[0], dtype=torch.float64, device="cuda")
    M.assemble_rhs(prob, F)
    u = torch.zeros_like(F)
    M.solve(F, u, tol=1e-10, max_iter=1000, precision=precision)
    torch.cuda.synchronize()
    out = u.cpu().numpy()
    M.free()
    return out


@pytest.mark.parametrize("precision", [hp.PREC_F64, hp.PREC_MIXED])
def test_results_in_the_mix_equal_results_alone(ctx, precision):
    mix = _mix()
    sv = hp.Server(ctx, max_active=3, precision=precision, n_cheb=4, smoother="point", Lambda=20.0)
    outs, tickets = [], []
    for mesh, prob in mix:
        outs.append(np.zeros(meshgen.dof_count(mesh)))
        tickets.append(sv.submit(mesh, prob, outs[-1]))
    sts = [sv.wait(t, timeout_ms=120000) for t in tickets]
    sv.close()
    overlap = any(a["start_ms"] < b["end_ms"] and b["start_ms"] < a["end_ms"]
                  for i, a in enumerate(sts) for b in sts[i + 1:])
    busy = sum(s["end_ms"] - s["start_ms"] for s in sts)
    span = max(s["end_ms"] for s in sts) - min(s["start_ms"] for s in sts)
    print("states", [s["state"] for s in sts], "iterations", [s["iterations"] for s in sts],
          "in flight together", overlap, "summed run time %.1f ms over a %.1f ms span" % (busy, span), flush=True)
    # continuous batching: the six requests were submitted at once to three slots, so requests
    # ran concurrently (their [start, end) intervals intersect, and the summed run time exceeds
    # the span); the equality below then shows each result is the same in the mix as alone
    assert overlap and busy > span
    for (mesh, prob), u, st in zip(mix, outs, sts):
        assert st["state"] == "done" and st["rel_residual"] <= 1e-10
        ua = _alone(ctx, mesh, prob, precision)
        d = np.abs(u - ua).max() / np.abs(ua).max()
        print("mix vs alone", meshgen.dof_count(mesh), "max rel diff", d, "bitwise", bool(np.all(u == ua)),
              flush=True)
        assert d <= 1e-14
    # one residual recomputed by the oracle
    mesh, prob = mix[0]
    op = SIPG(mesh, prob)
    Fo = op.rhs()
    assert np.linalg.norm(Fo - op.apply(outs[0])) / np.linalg.norm(Fo) <= 1e-10


def test_admission_by_footprint(ctx):
    mesh, prob = meshgen.unit_cube(2, 4), meshgen.gaussian_problem(lo=(0, 0, 0), hi=(1, 1, 1), seed=7)
    sv = hp.Server(ctx, max_active=4)
    u0 = np.zeros(meshgen.dof_count(mesh))
    est = sv.wait(sv.submit(mesh, prob, u0))["device_bytes"]
    sv.close()
    sv = hp.Server(ctx, max_active=4, hbm_budget_bytes=int(1.5 * est))
    outs = [np.zeros_like(u0) for _ in range(6)]
    tickets = [sv.submit(mesh, prob, o) for o in outs]
    sts = [sv.wait(t, timeout_ms=120000) for t in tickets]
    sv.close()
    assert all(s["state"] == "done" for s in sts)
    for i, a in enumerate(sts):
        for b in sts[i + 1:]:
            assert a["end_ms"] <= b["start_ms"] or b["end_ms"] <= a["start_ms"]
    for o in outs:
        assert np.array_equal(o, u0)
