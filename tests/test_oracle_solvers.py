"""Pins for the oracle's multigrid and Krylov layer (Algs. 2-5, Eqs. psi-interpolation, temp-G)."""
import numpy as np
import pytest

import meshgen
from oracle import problems as P
from oracle.operator import SIPG
from oracle.solvers import (Multigrid, Transfer, cg_lanczos, chebyshev, fcg, fgmres, gershgorin_max,
                            pcg, splitmix64_uniform)


def test_chebyshev_matches_closed_form_polynomial():
    # Alg. 4 from x0 = 0 leaves the error e_k = T_k((d - A)/c) / T_k(d/c) e_0
    lam = np.linspace(0.05, 3.0, 40)
    A = np.diag(lam)
    b = np.random.default_rng(0).standard_normal(40)
    xstar = b / lam
    lmax, Lam = 3.2, 10.0
    lmin = lmax / Lam
    c, d = 0.5 * (lmax - lmin), 0.5 * (lmax + lmin)
    for k in (1, 2, 3, 8):
        x = chebyshev(lambda v: A @ v, b, np.zeros(40), lmax, Lam, k)
        Tk = np.polynomial.chebyshev.Chebyshev.basis(k)
        e = Tk((d - lam) / c) / Tk(d / c) * (-xstar)
        np.testing.assert_allclose(x - xstar, e, atol=1e-13)


def test_cg_lanczos_tridiagonal_bounds():
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    lam = np.sort(rng.uniform(0.1, 7.3, 60))
    lam[-1] = 7.3
    A = Q @ np.diag(lam) @ Q.T
    b = rng.uniform(-1, 1, 60)
    x, T = cg_lanczos(lambda v: A @ v, b, 15)
    ritz = np.linalg.eigvalsh(T)
    assert ritz.min() >= lam.min() - 1e-10 and ritz.max() <= lam.max() + 1e-10
    assert gershgorin_max(T) >= ritz.max()
    assert ritz.max() > 0.9 * lam.max()
    # the Lanczos T is similar to A restricted to the Krylov space: its eigenvalues
    # after n steps of CG on an n x n system are A's eigenvalues
    _, Tn = cg_lanczos(lambda v: A[:8, :8] @ v, b[:8], 8)
    np.testing.assert_allclose(np.linalg.eigvalsh(Tn), np.linalg.eigvalsh(A[:8, :8]), rtol=1e-8)


def test_splitmix64_reference_values():
    # first outputs of SplitMix64 with seed 0 (published generator): 0xe220a8397b1dcdaf, ...
    u = splitmix64_uniform(2, 0)
    ref = [(0xE220A8397B1DCDAF >> 11) * 2.0 ** -53 * 2 - 1, (0x6E789E6AA1B965F4 >> 11) * 2.0 ** -53 * 2 - 1]
    np.testing.assert_allclose(u, ref, rtol=0, atol=0)


@pytest.mark.parametrize("maker", [
    lambda: meshgen.cubed_sphere_shell(level=1, p=2, zeta_break=0.0, r_out=50.0),
    lambda: meshgen.hp_sphere_cube(level=2, p_lo=1, p_hi=3, seed=2, r_cut=0.6),
])
def test_transfer_reproduces_coarse_functions_and_is_transposed(maker):
    mg = Multigrid(maker(), None, n_cheb=2, lam=[1.0] * 10, jacobi=False)
    rng = np.random.default_rng(0)
    for T in mg.transfers:
        # a linear function of the physical coordinates on an affine mesh / any coarse
        # nodal vector: the prolongation is exact interpolation (coarse space embeds)
        xc = rng.standard_normal(T.coarse.ndof)
        xf = T.prolong(xc)
        yf = rng.standard_normal(T.fine.ndof)
        assert abs(xf @ yf - xc @ T.restrict(yf)) <= 1e-13 * np.linalg.norm(xf) * np.linalg.norm(yf)
        # embedding: the coarse bilinear form of (x, x) equals the fine form of (P x, P x) for
        # the broken stiffness part when no face jumps are created is not general; instead
        # check exact reproduction of the coarse polynomial at the fine nodes via point values
    fine, coarse = mg.ops[0], mg.ops[1]
    f = lambda X: 1.0 + X[..., 0] - 0.5 * X[..., 1] + 0.25 * X[..., 2]
    if np.all(fine.affine):
        np.testing.assert_allclose(mg.transfers[0].prolong(coarse.interpolate(f)), fine.interpolate(f),
                                   atol=1e-13)


def test_vcycle_symmetric_positive_and_fcg_equals_pcg():
    m = meshgen.hp_sphere_cube(level=2, p_lo=1, p_hi=3, seed=2, r_cut=0.6)
    prob = meshgen.problem_config3(r0=0.6)
    mg = Multigrid(m, prob, n_cheb=3)
    rng = np.random.default_rng(5)
    r1, r2 = rng.standard_normal((2, mg.ops[0].ndof))
    a, b = r2 @ mg.vcycle(r1), r1 @ mg.vcycle(r2)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    assert r1 @ mg.vcycle(r1) > 0
    op = mg.ops[0]
    F = op.rhs()
    u1, k1, h1 = fcg(op.apply, F, mg.vcycle, tol=1e-10)
    u2, k2, h2 = pcg(op.apply, F, mg.vcycle, tol=1e-10)
    assert k1 == k2
    np.testing.assert_allclose(h1, h2, rtol=1e-6)
    assert np.linalg.norm(F - op.apply(u1)) <= 1e-10 * np.linalg.norm(F)
    np.testing.assert_allclose(u1, u2, atol=1e-9 * np.abs(u1).max())


def test_solve_polynomial_exactly_on_2to1_mesh():
    # consistency + exact quadrature: the discrete solution is the interpolant
    prob = meshgen.problems.polynomial_problem(2, seed=3)
    m = meshgen.box_grid((1, 1, 1), 1, 2, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5])
    mg = Multigrid(m, prob, n_cheb=4)
    op = mg.ops[0]
    u, k, h = fcg(op.apply, op.rhs(), mg.vcycle, tol=1e-12)
    uI = op.interpolate(lambda X: P.exact_u(prob, X))
    assert np.abs(u - uI).max() < 1e-9


def test_paper_literal_smoother_also_solves():
    # the printed (unscaled) Chebyshev smoother gives the same discrete solution
    m = meshgen.unit_cube(1, 3)
    prob = meshgen.problem_config1()
    a = Multigrid(m, prob, n_cheb=4, jacobi=False)
    b = Multigrid(m, prob, n_cheb=4, jacobi=True)
    F = a.ops[0].rhs()
    ua, ka, _ = fcg(a.ops[0].apply, F, a.vcycle, tol=1e-11)
    ub, kb, _ = fcg(b.ops[0].apply, F, b.vcycle, tol=1e-11)
    np.testing.assert_allclose(ua, ub, atol=1e-9 * np.abs(ua).max())


def test_fgmres_pins():
    # flexible GMRES, pinned against properties that do not depend on its code:
    rng = np.random.default_rng(11)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.linspace(1.0, 50.0, n)) @ Q.T
    b = rng.standard_normal(n)
    exact = np.linalg.solve(A, b)
    # (1) with a fixed preconditioner it solves the system (up to rounding)
    Minv = np.linalg.inv(A + 0.3 * np.diag(rng.uniform(0.5, 1.5, n)))
    u, k, hist = fgmres(lambda x: A @ x, b, lambda r: Minv @ r, tol=1e-13, max_iter=200, restart=10)
    assert np.linalg.norm(u - exact) <= 1e-11 * np.linalg.norm(exact)
    # (2) finite termination: without preconditioning and without restart, a matrix with 5
    # distinct eigenvalues is solved in at most 5 steps
    D = np.diag(np.repeat([1.0, 2.0, 3.0, 5.0, 8.0], 8))
    u, k, hist = fgmres(lambda x: D @ x, b, lambda r: r, tol=1e-12, max_iter=100, restart=50)
    assert k <= 5 and np.allclose(u, b / np.diag(D), rtol=1e-10, atol=0)
    # (3) within a cycle the minimised residual does not grow
    u, k, hist = fgmres(lambda x: A @ x, b, lambda r: r, tol=1e-12, max_iter=30, restart=30)
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 2))
    # (4) flexible: a preconditioner that changes at every call (two alternating SPD
    # approximate inverses) still converges to the solution
    M1, M2 = np.diag(1.0 / np.diag(A)), Minv
    calls = [0]

    def varying(r):
        calls[0] += 1
        return (M1 if calls[0] % 2 else M2) @ r
    u, k, hist = fgmres(lambda x: A @ x, b, varying, tol=1e-12, max_iter=200, restart=8)
    assert np.linalg.norm(A @ u - b) <= 1e-11 * np.linalg.norm(b)
    # (5) a planted error in a copy of the oracle (a Gram-Schmidt sign flipped) fails (1)
    import inspect

    import oracle.solvers as solvers
    src = inspect.getsource(solvers.fgmres).replace("w = w - Hbar[i, j] * V[i]", "w = w + Hbar[i, j] * V[i]")
    ns = {"np": np}
    exec(src, ns)
    u, k, hist = ns["fgmres"](lambda x: A @ x, b, lambda r: Minv @ r, tol=1e-13, max_iter=200, restart=10)
    assert np.linalg.norm(u - exact) > 1e-6 * np.linalg.norm(exact)
