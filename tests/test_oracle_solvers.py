"""Pins for the oracle's multigrid and Krylov layer (Algs. 2-5, Eqs. psi-interpolation, temp-G)."""
import numpy as np
import pytest
import scipy.linalg

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


def _tiny_operator():
    # two p = 1 cells and a 2:1 refined box: small enough for dense eigen-decompositions
    m = meshgen.box_grid((1, 1, 1), 1, 1, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5])
    return Multigrid(m, meshgen.problem_config3(r0=0.6), n_cheb=2, lam=[1.0] * 10, smoother="point")


@pytest.mark.parametrize("smoother", ["point", "block"])
def test_preconditioned_lanczos_gives_eigenvalues_of_minv_a(smoother):
    # Alg. 5 with M: after n CG steps on an n x n system (distinct eigenvalues) the Lanczos
    # tridiagonal holds the eigenvalues of M^-1 A (the generalised problem A v = lambda M v),
    # and the Gershgorin bound after 15 steps bounds lambda_max(M^-1 A) from above
    from oracle.operator import assemble_dense, element_blocks
    rng = np.random.default_rng(21)
    n = 24
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.linspace(1.0, 9.0, n) ** 2) @ Q.T
    A = 0.5 * (A + A.T)
    blocks = [A[i:i + 8, i:i + 8] for i in range(0, n, 8)]
    M = np.diag(np.diag(A)) if smoother == "point" else scipy.linalg.block_diag(*blocks)
    Minv = np.linalg.inv(M)
    lam = scipy.linalg.eigh(A, M, eigvals_only=True)
    b = splitmix64_uniform(n, 7)
    _, T = cg_lanczos(lambda v: A @ v, b, n, minv=lambda r: Minv @ r)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(T)), lam, rtol=1e-6)
    _, T15 = cg_lanczos(lambda v: A @ v, b, 15, minv=lambda r: Minv @ r)
    assert gershgorin_max(T15) >= lam.max() * (1 - 1e-12)
    # unpreconditioned steps do not give the spectrum of M^-1 A (the pin tells the two apart)
    _, Tn = cg_lanczos(lambda v: A @ v, b, n)
    assert np.abs(np.sort(np.linalg.eigvalsh(Tn)) - lam).max() > 1e-3 * lam.max()
    # on a mesh level, the oracle's own M (Multigrid smoother scaling) is diag(A) / the
    # element-diagonal blocks of the assembled A
    mg = _tiny_operator()
    op = mg.ops[-2]
    Ad = assemble_dense(op)
    Md = np.diag(np.diag(Ad)) if smoother == "point" else scipy.linalg.block_diag(*element_blocks(op))
    mg.smoother = smoother
    r = rng.standard_normal(op.ndof)
    z = np.linalg.solve(Md, r)
    np.testing.assert_allclose(mg._make_minv(op)(r), z, rtol=0, atol=1e-10 * np.abs(z).max())


@pytest.mark.parametrize("smoother", ["point", "block"])
def test_preconditioned_chebyshev_matches_closed_form(smoother):
    # Alg. 4 on M^-1 A from x0: e_k = P_k(M^-1 A) e_0 with P_k(l) = T_k((d - l)/c) / T_k(d/c)
    from oracle.operator import assemble_dense, element_blocks
    mg = _tiny_operator()
    op = mg.ops[0]
    A = assemble_dense(op)
    A = 0.5 * (A + A.T)
    M = np.diag(np.diag(A)) if smoother == "point" else scipy.linalg.block_diag(*element_blocks(op))
    Minv = np.linalg.inv(M)
    lam, V = scipy.linalg.eigh(A, M)  # A V = M V diag(lam), V^T M V = I
    rng = np.random.default_rng(3)
    b, x0 = rng.standard_normal((2, op.ndof))
    xstar = np.linalg.solve(A, b)
    lmax, Lam = 1.05 * lam.max(), 30.0
    lmin = lmax / Lam
    c, d = 0.5 * (lmax - lmin), 0.5 * (lmax + lmin)
    for k in (1, 2, 3, 7):
        x = chebyshev(lambda v: A @ v, b, x0, lmax, Lam, k, minv=lambda r: Minv @ r)
        Tk = np.polynomial.chebyshev.Chebyshev.basis(k)
        Pk = Tk((d - lam) / c) / Tk(d / c)
        e = V @ (Pk * (V.T @ (M @ (x0 - xstar))))  # M^-1 A = V diag(lam) V^-1, V^-1 = V^T M
        np.testing.assert_allclose(x - xstar, e, atol=1e-10 * np.abs(x0 - xstar).max())


def test_multigrid_bounds_use_splitmix_start_and_bound_the_spectrum():
    # the bound of every smoothed level comes from CG on the SplitMix64 start vector of that
    # level (its own DOF order), and is >= lambda_max(M^-1 A) from a dense eigen-solve
    from oracle.operator import assemble_dense
    m = meshgen.box_grid((1, 1, 1), 1, 2, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5])
    mg = Multigrid(m, meshgen.problem_config1(), n_cheb=2, smoother="point", seed=5)
    for l, op in enumerate(mg.ops[:-1]):
        _, T = cg_lanczos(op.apply, splitmix64_uniform(op.ndof, 5), 15, minv=mg.minv[l])
        assert gershgorin_max(T) == mg.lam[l]
        A = assemble_dense(op)
        lam = scipy.linalg.eigh(0.5 * (A + A.T), np.diag(np.diag(A)), eigvals_only=True)
        assert mg.lam[l] >= lam.max() * (1 - 1e-12), (l, mg.lam[l], lam.max())
    # a permuted start vector (another element order of the same level) is passed through
    starts = [splitmix64_uniform(op.ndof, 9) for op in mg.ops[:-1]]
    mg.refresh(15, 5, starts=starts)
    _, T = cg_lanczos(mg.ops[0].apply, starts[0], 15, minv=mg.minv[0])
    assert gershgorin_max(T) == mg.lam[0]


def test_splitmix64_reference_values():
    # first outputs of SplitMix64 with seed 0 (published generator): 0xe220a8397b1dcdaf, ...
    u = splitmix64_uniform(2, 0)
    ref = [(0xE220A8397B1DCDAF >> 11) * 2.0 ** -53 * 2 - 1, (0x6E789E6AA1B965F4 >> 11) * 2.0 ** -53 * 2 - 1]
    np.testing.assert_allclose(u, ref, rtol=0, atol=0)
    # the vectorised form equals the generator's sequential definition (state += golden gamma)
    state, mask, seq = 1234567, (1 << 64) - 1, []
    for _ in range(50):
        state = (state + 0x9E3779B97F4A7C15) & mask
        z = ((state ^ (state >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        seq.append(((z ^ (z >> 31)) >> 11) * 2.0 ** -53 * 2 - 1)
    np.testing.assert_array_equal(splitmix64_uniform(50, 1234567), seq)


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
    # equal in exact arithmetic (Alg. 2 with a fixed SPD preconditioner is PCG); in FP64 the
    # relative residual histories agree to rounding measured against |r0| (they start at 1)
    np.testing.assert_allclose(h1, h2, rtol=1e-6, atol=1e-13)
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
