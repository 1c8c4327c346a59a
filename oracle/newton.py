"""Newton-Krylov solve of a semilinear problem with the multigrid-preconditioned FCG.

Problem (the puncture-type equation of Sec. III.D, Eq. Two_Punctures_PDE, written for the
regular part u):  -lap u = beta(x) (1 + alpha(x) u)^-7,  u = g_D on Dirichlet faces.
Discretely (Sec. II.D.1, Eq. Ru=0):

    R(u) = A u - N(u) - F,   N(u)_psi = sum_sigma w_sigma det J_sigma beta (1 + alpha u)^-7 psi,

with A the SIPG operator (Eq. lh2), F its Dirichlet / source terms (Eq. Fh2) and u
evaluated at the volume GL points.  The Jacobian (Eq. newtoncorrectionsystem) is
A + M(u), M the mass form with coefficient c = 7 alpha beta (1 + alpha u)^-8 >= 0 at the
GL points.  Newton (Alg. 1) solves J delta = -R with FCG (Alg. 2) preconditioned by the
V-cycle (Alg. 3) of the Jacobian and stops when |R(u_k)| / |R(u_0)| <= tol.

Multigrid levels carry their own Jacobian: the state is carried to the coarser levels by
injection (each coarse LGL node takes the value of the finer-level polynomial of the child
cell that contains it; a node on the cut between two children belongs to the lower one),
the coefficient c is evaluated at each level's own GL points, and the smoother scaling,
spectral bounds and coarse factorisation are recomputed for every Newton step.

Each level's volume rule uses q = p + 1 + quad_extra points (a mass term is present).

The constant-density star (Sec. III.B, Eq. Constant_Density_Star_PDE) is the same solve with
N(psi)_v = sum_sigma w det J 2 pi rho psi^5 v (rho = rho0 inside r0, 0 outside) and the
Jacobian mass coefficient c = -5 (2 pi rho) psi^4 (problems.nl_terms).
"""
import numpy as np

from . import problems, rules
from .mesh import parent_map
from .solvers import Multigrid, fcg, inject  # noqa: F401 (inject is part of this module's API)


def _gl_values(g, u):
    """Field values at the GL points of every element of a volume group."""
    n = g["n"]
    B = g["B"]
    U = u[g["idx"]].reshape(-1, n, n, n)
    return np.einsum("ck,bj,ai,ekji->ecba", B, B, B, U, optimize=True).reshape(len(U), -1)


def _project(g, vals):
    """sum_sigma vals_sigma psi(x_sigma) for every element of a volume group."""
    q, B = g["q"], g["B"]
    return np.einsum("ck,bj,ai,ecba->ekji", B, B, B, vals.reshape(-1, q, q, q),
                     optimize=True).reshape(len(vals), -1)


class NewtonSolver:
    def __init__(self, mesh, nl, C=10.0, quad_extra=1, n_cheb=4, Lambda=20.0, n_eigs=15, seed=0,
                 smoother="point"):
        if smoother == "block":
            raise ValueError("the element blocks do not follow the Newton mass terms; use point or none")
        zero = lambda x: np.zeros(x.shape[:-1])  # noqa: E731 (mass form present, values set below)
        self.nl = nl
        self.n_eigs, self.seed = n_eigs, seed
        self.mg = Multigrid(mesh, None, C=C, quad_extra=quad_extra, n_cheb=n_cheb, Lambda=Lambda,
                            n_eigs=n_eigs, seed=seed, mass=zero, smoother=smoother)
        self.ops = self.mg.ops
        for op in self.ops:
            for g in op.vgroups:
                g["alpha"], g["beta"] = problems.nl_alpha_beta(nl, g["x"])
                g["M"] = np.zeros_like(g["alpha"])

    @staticmethod
    def _check(one_plus):
        if np.any(one_plus <= 0.0):
            raise FloatingPointError("1 + alpha u <= 0 at a quadrature point")

    def nonlinear(self, u):
        """N(u) on the finest level."""
        op = self.ops[0]
        N = np.zeros(op.ndof)
        for g in op.vgroups:
            val, _ = problems.nl_terms(self.nl, g["alpha"], g["beta"], _gl_values(g, u))
            N[g["idx"]] += _project(g, g["W"] * g["det"] * val)
        return N

    def apply_A(self, u):
        """A u without the mass term."""
        op = self.ops[0]
        saved = [g["M"] for g in op.vgroups]
        for g in op.vgroups:
            g["M"] = None
        y = op.apply(u)
        for g, m in zip(op.vgroups, saved):
            g["M"] = m
        return y

    def residual(self, u, F):
        return self.apply_A(u) - self.nonlinear(u) - F

    def set_state(self, u):
        """Jacobian mass terms on every level from the state u (injected downwards)."""
        ul = u
        for lvl, op in enumerate(self.ops):
            if lvl > 0:
                ul = inject(self.ops[lvl - 1], op, ul)
            for g in op.vgroups:
                _, c = problems.nl_terms(self.nl, g["alpha"], g["beta"], _gl_values(g, ul))
                g["M"] = g["W"] * g["det"] * c
        self.mg.refresh(self.n_eigs, self.seed)

    def jacobian_apply(self, v):
        return self.ops[0].apply(v)

    def solve(self, F, u0=None, tol=1e-10, lin_tol=1e-6, max_newton=20, max_lin=300):
        """Alg. 1; returns (u, newton steps, |R_k| / |R_0| history, total FCG iterations)."""
        u = np.zeros(self.ops[0].ndof) if u0 is None else np.array(u0, float)
        R = self.residual(u, F)
        r0 = np.linalg.norm(R)
        hist = [1.0]
        lin = 0
        k = 0
        while r0 > 0 and hist[-1] > tol and k < max_newton:
            self.set_state(u)
            delta, its, _ = fcg(self.jacobian_apply, -R, self.mg.vcycle, tol=lin_tol, max_iter=max_lin)
            lin += its
            u = u + delta
            R = self.residual(u, F)
            hist.append(np.linalg.norm(R) / r0)
            k += 1
        return u, k, hist, lin
