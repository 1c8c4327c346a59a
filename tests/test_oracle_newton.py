"""Pins of the oracle's Newton-Krylov path (semilinear puncture-type problem)."""
import numpy as np
import pytest

import meshgen
from oracle import problems
from oracle.newton import NewtonSolver, inject
from oracle.solvers import Transfer


def _poly(C, x):
    return sum(C[a, b, c] * x[..., 0] ** a * x[..., 1] ** b * x[..., 2] ** c
               for a in range(3) for b in range(3) for c in range(3))


@pytest.mark.parametrize("alpha", [0.0, 0.5])
@pytest.mark.parametrize("maker", [
    lambda: meshgen.unit_cube(1, 2),
    lambda: meshgen.box_grid((2, 1, 1), 1, 3, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5]),
])
def test_quadratic_manufactured_solution_is_reproduced(maker, alpha):
    # u* quadratic, beta = (-lap u*)(1 + alpha u*)^7: on affine meshes with p >= 2 the
    # interpolant of u* satisfies the discrete equations exactly (SIPG consistency and
    # exact quadrature of -lap u* times the basis), so Newton must return it
    m = maker()
    nl, C = meshgen.quadratic_nonlinear_problem(alpha=alpha, seed=3)
    ns = NewtonSolver(m, nl, n_cheb=3)
    F = ns.ops[0].rhs(meshgen.polynomial_dirichlet_problem(C))
    u, k, hist, _ = ns.solve(F, tol=1e-13, lin_tol=1e-10)
    ustar = ns.ops[0].interpolate(lambda x: _poly(C, x))
    assert hist[-1] <= 1e-13
    assert np.abs(u - ustar).max() <= 1e-11 * np.abs(ustar).max()


def test_jacobian_matches_central_differences():
    m = meshgen.cubed_sphere_shell(level=1, p=2, r_out=30.0, zeta_break=0.0, r_break=4.0)
    nl = meshgen.puncture_problem(seed=1, r_ball=3.0)
    nl["params"][5::5] *= 1e3  # stronger source: a clearly nonlinear residual
    ns = NewtonSolver(m, nl)
    rng = np.random.default_rng(0)
    F = np.zeros(ns.ops[0].ndof)
    u = 0.05 * rng.standard_normal(ns.ops[0].ndof)
    v = rng.standard_normal(ns.ops[0].ndof)
    ns.set_state(u)
    Jv = ns.jacobian_apply(v)
    errs = []
    for eps in (1e-2, 1e-3):
        fd = (ns.residual(u + eps * v, F) - ns.residual(u - eps * v, F)) / (2 * eps)
        errs.append(np.linalg.norm(fd - Jv) / np.linalg.norm(Jv))
    # second-order differences: the error falls by ~100 per decade of eps
    assert errs[1] < 3e-2 * errs[0] or errs[1] < 1e-12
    assert errs[1] < 1e-5


def test_newton_converges_quadratically():
    m = meshgen.unit_cube(1, 3)
    nl, C = meshgen.quadratic_nonlinear_problem(alpha=0.9, seed=1)
    ns = NewtonSolver(m, nl, n_cheb=3)
    F = ns.ops[0].rhs(meshgen.polynomial_dirichlet_problem(C))
    u, k, hist, _ = ns.solve(F, tol=1e-14, lin_tol=1e-13, max_lin=500)
    h = [x for x in hist if x > 1e-13]
    # once in the basin, each step at least squares the residual (up to a modest constant)
    for a, b in zip(h[1:], h[2:]):
        assert b <= 10.0 * a * a


def test_injection_inverts_prolongation():
    m = meshgen.hp_sphere_cube(level=2, p_lo=1, p_hi=4, seed=2, r_cut=0.6)
    ns = NewtonSolver(m, dict(kind="nl_quadratic", params=np.r_[0.0, np.zeros(27)]))
    rng = np.random.default_rng(1)
    for lvl in range(len(ns.ops) - 1):
        fine, coarse = ns.ops[lvl], ns.ops[lvl + 1]
        uc = rng.standard_normal(coarse.ndof)
        uf = Transfer(fine, coarse).prolong(uc)
        assert np.abs(inject(fine, coarse, uf) - uc).max() <= 1e-12 * np.abs(uc).max()


def test_puncture_coefficients_limits():
    nl = meshgen.puncture_problem(seed=0)
    rows = nl["params"][1:].reshape(-1, 5)
    far = np.array([[1e6, 0.0, 0.0]])
    a, b = problems.nl_alpha_beta(nl, far)
    assert abs(a[0] - 1.0) < 1e-5 and 0 <= b[0] < 1e-20
    c, mI = rows[0, :3], rows[0, 3]
    near = c[None, :] + np.array([[1e-7, 0, 0]])
    a, b = problems.nl_alpha_beta(nl, near)
    # alpha ~ 2 r / m next to a puncture
    assert abs(a[0] / (2e-7 / mI) - 1.0) < 1e-3 and b[0] >= 0


def test_star_closed_form():
    # constant-density star (Sec. III.B): psi and dpsi/dr continuous at r0, psi -> 1 far
    # away, and psi solves psi'' + 2 psi' / r + 2 pi rho psi^5 = 0 inside and outside
    rho0, r0 = 0.001, 4.0
    C, alpha, beta = problems.star_parameters(rho0, r0)
    assert alpha >= np.sqrt(5.0)
    assert abs(3.0 / (2.0 * np.pi) * alpha ** 10 / (1.0 + alpha ** 2) ** 6 - rho0 * r0 * r0) <= 1e-12
    psi = lambda r: problems.star_psi(rho0, r0, r)  # noqa: E731
    h = 1e-5
    d_in = (psi(r0) - psi(r0 - h)) / h
    d_out = (psi(r0 + 2 * h) - psi(r0 + h)) / h
    assert abs(psi(r0) - (beta / r0 + 1.0)) <= 1e-14
    assert abs(d_in - d_out) <= 1e-4 * abs(d_in)  # one-sided differences: O(h) each
    assert abs(psi(1e6) - 1.0) <= 1e-6
    for r in (0.5, 2.0, 3.5, 5.0, 9.0):
        rho = rho0 if r <= r0 else 0.0
        hh = 1e-3
        lap = (psi(r + hh) - 2 * psi(r) + psi(r - hh)) / hh ** 2 + (psi(r + hh) - psi(r - hh)) / (r * hh)
        assert abs(lap + 2 * np.pi * rho * psi(r) ** 5) <= 1e-6


def test_star_newton_jacobian_and_convergence():
    rho0, r0 = 0.001, 4.0
    nl, dirichlet = meshgen.star_problem(rho0, r0)
    errs = []
    for nref in (1, 2):
        m = meshgen.star_mesh(level=2, p=2, r0=r0, refine_near=nref)
        ns = NewtonSolver(m, nl, n_cheb=3)
        F = ns.ops[0].rhs(dirichlet)
        if nref == 1:
            # the Jacobian (mass coefficient -5 (2 pi rho) psi^4) is the derivative of R
            rng = np.random.default_rng(0)
            u = 1.0 + 0.1 * rng.standard_normal(ns.ops[0].ndof)
            v = rng.standard_normal(ns.ops[0].ndof)
            ns.set_state(u)
            Jv = ns.jacobian_apply(v)
            eps = 1e-4
            fd = (ns.residual(u + eps * v, F) - ns.residual(u - eps * v, F)) / (2 * eps)
            assert np.linalg.norm(fd - Jv) <= 1e-6 * np.linalg.norm(Jv)
        u, k, hist, _ = ns.solve(F, tol=1e-11, lin_tol=1e-8)
        assert hist[-1] <= 1e-11
        exact = ns.ops[0].interpolate(lambda x: problems.star_psi(rho0, r0, np.linalg.norm(x, axis=-1)))
        errs.append(np.abs(u - exact).max())
    # the discrete solution approaches the closed form as the cells at the star shrink
    assert errs[1] < 0.5 * errs[0], errs
