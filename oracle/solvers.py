"""Multigrid-preconditioned Krylov solve: transfers, Chebyshev, CG spectral bound, V-cycle, FCG, PCG.

* Prolongation (Sec. II.D.6, Eq. psi-interpolation): coarse basis functions are
  interpolated exactly at the fine LGL nodes; restriction of residuals is the
  transpose (Eq. temp-G).
* Chebyshev smoother (Alg. 4) with the update p <- alpha r + beta p (the sign that
  reproduces the Chebyshev polynomial; the printed minus sign diverges).
  Optionally the residual is preconditioned by the inverse diagonal (point Jacobi) or
  the inverse element-diagonal blocks (block Jacobi) of A, i.e. the same recurrence on
  M^-1 A; the printed, unpreconditioned form is smoother="none".
* CG spectral bound (Alg. 5; preconditioned CG with the smoother's M): CG steps give the Lanczos tridiagonal of Eq. tridiag
  (diagonal 1/alpha_k + beta_{k-1}/alpha_{k-1}, off-diagonal -sqrt(beta_k)/alpha_k);
  lambda_max is the Gershgorin bound of the full tridiagonal.  It is computed once per
  level and frozen (the V-cycle is then a fixed symmetric operator).
* V-cycle (Alg. 3) over the stored hierarchy; the coarsest level is solved exactly by
  a dense FP64 Cholesky factorisation (instead of being smoothed).
* Flexible CG (Alg. 2) with r0 = b - A u0, stopping when |r|/|b| <= tol or after
  max_iter iterations; plain preconditioned CG for comparison.
* Restarted flexible GMRES (not in the paper; the method of Saad, SIAM J. Sci. Comput. 14,
  1993): right preconditioning with the preconditioned directions kept, so the
  preconditioner may change between iterations.
"""
import numpy as np
import scipy.linalg

from . import rules, schwarz
from .mesh import hierarchy, parent_map
from .operator import SIPG, assemble_dense, element_blocks


class Transfer:
    """Prolongation from a coarse cell mesh to the next finer one, and its transpose."""

    def __init__(self, fine_op, coarse_op):
        self.fine, self.coarse = fine_op, coarse_op
        pm = parent_map(fine_op.mesh, coarse_op.mesh)
        groups = {}
        for k, (K, bits) in enumerate(pm):
            key = (int(fine_op.n[k]), int(coarse_op.n[K]), bits)
            groups.setdefault(key, []).append((k, K))
        self.groups = []
        for (nf, nc, bits), pairs in groups.items():
            xf, _ = rules.lgl(nf)
            xc, _ = rules.lgl(nc)
            mats = []
            for d in range(3):
                pts = xf if bits is None else 0.5 * (xf + 2 * bits[d] - 1)
                mats.append(rules.lagrange(xc, pts))  # [fine node, coarse node]
            ks = np.array([p[0] for p in pairs])
            Ks = np.array([p[1] for p in pairs])
            self.groups.append(dict(
                nf=nf, nc=nc, P=mats,
                fidx=fine_op.offsets[ks][:, None] + np.arange(nf ** 3)[None, :],
                cidx=coarse_op.offsets[Ks][:, None] + np.arange(nc ** 3)[None, :]))

    def prolong(self, uc):
        uf = np.zeros(self.fine.ndof)
        for g in self.groups:
            P0, P1, P2 = g["P"]
            U = uc[g["cidx"]].reshape(-1, g["nc"], g["nc"], g["nc"])
            uf[g["fidx"]] = np.einsum("zc,yb,xa,ecba->ezyx", P2, P1, P0, U,
                                      optimize=True).reshape(len(U), -1)
        return uf

    def restrict(self, rf):
        rc = np.zeros(self.coarse.ndof)
        for g in self.groups:
            P0, P1, P2 = g["P"]
            R = rf[g["fidx"]].reshape(-1, g["nf"], g["nf"], g["nf"])
            out = np.einsum("zc,yb,xa,ezyx->ecba", P2, P1, P0, R, optimize=True)
            np.add.at(rc, g["cidx"], out.reshape(len(R), -1))
        return rc


def chebyshev(apply, b, x, lam_max, Lambda, n_iter, minv=None):
    """Alg. 4 with frozen lambda_max: n_iter Chebyshev steps on [lam_max/Lambda, lam_max].

    With ``minv`` (the inverse of a diagonal or element-block-diagonal part M of A, as a
    callable) the residual is preconditioned, r = M^-1 (b - A x): the same Chebyshev
    recurrence applied to M^-1 A; lam_max is then a bound of the spectrum of M^-1 A.
    """
    lam_min = lam_max / Lambda
    c = 0.5 * (lam_max - lam_min)
    d = 0.5 * (lam_max + lam_min)
    p = np.zeros_like(b)
    x = x.copy()
    alpha = 0.0
    for k in range(1, n_iter + 1):
        r = b - apply(x)
        if minv is not None:
            r = minv(r)
        if k == 1:
            alpha = 1.0 / d
        elif k == 2:
            alpha = 2.0 * d / (2.0 * d * d - c * c)
        else:
            alpha = 1.0 / (d - alpha * c * c / 4.0)
        beta = alpha * d - 1.0
        p = alpha * r + beta * p
        x = x + p
    return x


def cg_lanczos(apply, b, n_iter, x=None, minv=None):
    """Alg. 5: n_iter CG steps; returns (x, T) with the Lanczos tridiagonal T of Eq. tridiag.

    With ``minv`` the steps are preconditioned CG (z = M^-1 r, r.z in place of r.r), whose
    coefficients give the Lanczos tridiagonal of M^-1 A.
    """
    x = np.zeros_like(b) if x is None else x.copy()
    r = b - apply(x)
    z = r if minv is None else minv(r)
    p = z.copy()
    rz = r @ z
    alphas, betas = [], []
    for _ in range(n_iter):
        Ap = apply(p)
        alpha = rz / (p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        z = r if minv is None else minv(r)
        rz_new = r @ z
        beta = rz_new / rz
        alphas.append(alpha)
        betas.append(beta)
        p = z + beta * p
        rz = rz_new
    k = len(alphas)
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = -np.sqrt(betas[i]) / alphas[i]
    return x, T


def gershgorin_max(T):
    return float(np.max(np.diag(T) + np.sum(np.abs(T), axis=1) - np.abs(np.diag(T))))


def splitmix64_uniform(n, seed):
    """Uniform [-1, 1) values from the SplitMix64 generator (Steele, Lea, Flood 2014): output i
    mixes the counter state seed + (i + 1) * 0x9E3779B97F4A7C15 (mod 2^64); its top 53 bits give
    a value in [0, 1), mapped to [-1, 1).  Vectorised in uint64 arithmetic (wraps mod 2^64)."""
    i = np.arange(1, int(n) + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(int(seed) & ((1 << 64) - 1)) + i * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


def inject(fine_op, coarse_op, uf):
    """Coarse nodal values from the fine-level field: the fine polynomial of the child that
    contains each coarse LGL node (lower child on the cut), evaluated there."""
    uc = np.zeros(coarse_op.ndof)
    for k, (K, bits) in enumerate(parent_map(fine_op.mesh, coarse_op.mesh)):
        nf, nc = int(fine_op.n[k]), int(coarse_op.n[K])
        xf, _ = rules.lgl(nf)
        xc, _ = rules.lgl(nc)
        mats, owned = [], []
        for d in range(3):
            if bits is None:
                pts, own = xc, np.ones(nc, bool)
            else:
                b = bits[d]
                pts = 2.0 * xc - 2.0 * b + 1.0          # coarse node in the child's coordinates
                own = xc <= 0.0 if b == 0 else xc > 0.0  # nodes on the cut go to the lower child
            mats.append(rules.lagrange(xf, pts))        # [coarse node, fine node]
            owned.append(own)
        U = uf[fine_op.offsets[k]:fine_op.offsets[k + 1]].reshape(nf, nf, nf)
        vals = np.einsum("zc,yb,xa,cba->zyx", mats[2], mats[1], mats[0], U)
        mask = owned[2][:, None, None] & owned[1][None, :, None] & owned[0][None, None, :]
        block = uc[coarse_op.offsets[K]:coarse_op.offsets[K + 1]].reshape(nc, nc, nc)
        block[mask] = vals[mask]
    return uc


def coarsen_field(fine_op, coarse_mesh, field):
    """A tabulated coefficient on the next coarser mesh: per element, the mean of the values of
    the fine cells inside each coarse cell; per node, the injection of the fine field."""
    if field is None:
        return None
    pm = parent_map(fine_op.mesh, coarse_mesh)
    if field["where"] == "element":
        vals = np.asarray(field["values"], float)
        acc = np.zeros(len(coarse_mesh["elem_p"]))
        cnt = np.zeros(len(coarse_mesh["elem_p"]))
        for k, (K, _) in enumerate(pm):
            acc[K] += vals[k]
            cnt[K] += 1
        return dict(where="element", values=acc / cnt)
    coarse_op = SIPG(coarse_mesh, None)
    return dict(where="node", values=inject(fine_op, coarse_op, np.asarray(field["values"], float)))


class Multigrid:
    """Stored multigrid hierarchy with frozen Chebyshev bounds and an exact coarse solve."""

    def __init__(self, mesh, problem=None, C=10.0, quad_extra=1, n_cheb=4, Lambda=20.0,
                 n_eigs=15, lam=None, seed=0, mass=None, levels=None, jacobi=True, smoother=None,
                 starts=None, max_levels=32, kfield=None, cfield=None, robin_gamma=0.0,
                 schwarz_overlap=2, schwarz_local="exact"):
        """``smoother``: "none" (Alg. 4 as printed), "point" (Jacobi), "block"
        (element-block Jacobi) or "schwarz" (Alg. schwarz_smoother with ``n_cheb`` cycles per
        call and ``schwarz_overlap`` = N_overlap, at most p on a level of degree p; local
        solves exact or, ``schwarz_local="cg"``, CG to 1e-3 as in the paper; no spectral
        bound); ``jacobi`` selects
        "point" / "none" when it is not given.
        ``starts``: Alg. 5 start vectors per smoothed level (see ``refresh``).
        ``kfield`` / ``cfield``: tabulated coefficients of the finest level (SIPG), carried to
        the coarser levels by ``coarsen_field``."""
        meshes = hierarchy(mesh, max_levels) if levels is None else levels
        self.ops = []
        for m in meshes:
            if self.ops:
                kfield = coarsen_field(self.ops[-1], m, kfield)
                cfield = coarsen_field(self.ops[-1], m, cfield)
            self.ops.append(SIPG(m, problem, C=C, quad_extra=quad_extra, mass=mass, kfield=kfield,
                                 cfield=cfield, robin_gamma=robin_gamma))
        self.transfers = [Transfer(self.ops[i], self.ops[i + 1]) for i in range(len(self.ops) - 1)]
        self.n_cheb, self.Lambda = n_cheb, Lambda
        self.smoother = smoother if smoother is not None else ("point" if jacobi else "none")
        self.schwarz_overlap = schwarz_overlap
        self.schwarz_local = schwarz_local
        self.refresh(n_eigs, seed, lam, starts)

    def refresh(self, n_eigs=15, seed=0, lam=None, starts=None):
        """(Re)compute what depends on the level operators: the smoother scaling, the
        coarsest factorisation and the frozen spectral bounds (given ``lam`` or by Alg. 5).

        Alg. 5's start vector b of a level is ``starts[l]`` when given, else the SplitMix64
        uniform values ``splitmix64_uniform(ndof, seed)`` in this level's DOF order (x0 = 0, so
        the first residual is b).  A caller whose DOF order differs (a permutation of the same
        elements) passes the permuted generator output to reproduce the same Krylov process."""
        self.minv = [self._make_minv(op) for op in self.ops[:-1]]
        A0 = np.column_stack([self.ops[-1].apply(e) for e in np.eye(self.ops[-1].ndof)])
        self.A0 = 0.5 * (A0 + A0.T)
        self.chol = scipy.linalg.cho_factor(self.A0)
        self.lanczos = []
        if self.smoother == "schwarz":
            self.schwarz = []
            for op in self.ops[:-1]:
                A = assemble_dense(op)
                # (an element of degree p < N_overlap holds at most p layers beyond the coincident
                # one; levels with 2:1 faces take the construction from positions)
                if len(set(int(x) for x in op.mesh["elem_level"])) > 1:
                    subs = schwarz.subdomains_boxes(op, self.schwarz_overlap)
                else:
                    subs = schwarz.subdomains_topo(op, self.schwarz_overlap)
                self.schwarz.append((A, subs))
            lam = [0.0] * (len(self.ops) - 1)
        if lam is None:
            lam = []
            for l, (op, minv) in enumerate(zip(self.ops[:-1], self.minv)):
                b = starts[l] if starts is not None else splitmix64_uniform(op.ndof, seed)
                _, T = cg_lanczos(op.apply, b, n_eigs, minv=minv)
                self.lanczos.append(T)
                lam.append(gershgorin_max(T))
        self.lam = list(lam)

    def _make_minv(self, op):
        if self.smoother == "schwarz":
            return None
        if self.smoother == "point":
            dinv = 1.0 / op.diagonal()
            return lambda r: dinv * r
        if self.smoother == "block":
            inv = [np.linalg.inv(B) for B in element_blocks(op)]
            off = op.offsets

            def apply_blocks(r):
                z = np.empty_like(r)
                for e, Bi in enumerate(inv):
                    z[off[e]:off[e + 1]] = Bi @ r[off[e]:off[e + 1]]
                return z
            return apply_blocks
        return None

    @property
    def nlevels(self):
        return len(self.ops)

    def smooth(self, level, b, x):
        if self.smoother == "schwarz":
            A, subs = self.schwarz[level]
            return schwarz.smooth(A, subs, b, x, self.n_cheb, local=self.schwarz_local)
        return chebyshev(self.ops[level].apply, b, x, self.lam[level], self.Lambda, self.n_cheb,
                         self.minv[level])

    def coarse_solve(self, f):
        return scipy.linalg.cho_solve(self.chol, f)

    def vcycle(self, f):
        """Alg. 3: z = V(f), from zero initial guesses on every level."""
        L = self.nlevels - 1
        fs = [None] * (L + 1)
        vs = [None] * (L + 1)
        fs[0] = f
        for l in range(L):
            vs[l] = self.smooth(l, fs[l], np.zeros_like(fs[l]))
            fs[l + 1] = self.transfers[l].restrict(fs[l] - self.ops[l].apply(vs[l]))
        vs[L] = self.coarse_solve(fs[L])
        for l in range(L - 1, -1, -1):
            vs[l] = self.transfers[l].prolong(vs[l + 1]) + vs[l]
            vs[l] = self.smooth(l, fs[l], vs[l])
        return vs[0]


def fcg(apply, b, precond, u0=None, tol=1e-10, max_iter=200):
    """Alg. 2 (flexible CG, one-vector truncation); returns (u, iterations, rel. residual history)."""
    u = np.zeros_like(b) if u0 is None else u0.copy()
    r = b - apply(u)
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    d = q = None
    rho = None
    k = 0
    while hist[-1] > tol and k < max_iter:
        v = precond(r)
        w = apply(v)
        alpha = v @ r
        beta = v @ w
        if k == 0:
            d, q, rho = v, w, beta
        else:
            gamma = v @ q
            d = v - (gamma / rho) * d
            q = w - (gamma / rho) * q
            rho = beta - gamma * gamma / rho
        u = u + (alpha / rho) * d
        r = r - (alpha / rho) * q
        k += 1
        hist.append(np.linalg.norm(r) / nb)
    return u, k, hist


def pcg(apply, b, precond, u0=None, tol=1e-10, max_iter=200):
    """Preconditioned CG (textbook); returns (u, iterations, rel. residual history)."""
    u = np.zeros_like(b) if u0 is None else u0.copy()
    r = b - apply(u)
    nb = np.linalg.norm(b)
    z = precond(r)
    p = z.copy()
    rz = r @ z
    hist = [np.linalg.norm(r) / nb]
    k = 0
    while hist[-1] > tol and k < max_iter:
        Ap = apply(p)
        alpha = rz / (p @ Ap)
        u = u + alpha * p
        r = r - alpha * Ap
        z = precond(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        k += 1
        hist.append(np.linalg.norm(r) / nb)
    return u, k, hist


def fgmres(apply, b, precond, u0=None, tol=1e-10, max_iter=200, restart=30):
    """Restarted flexible GMRES (Saad 1993).  Each cycle builds, from r0 = b - A u0, an
    orthonormal basis V by Arnoldi (modified Gram-Schmidt) on the preconditioned directions
    z_j = M_j v_j, A Z = V Hbar, and takes u = u0 + Z y with y minimising |beta e1 - Hbar y|
    (a least-squares solve); the cycle stops when that minimum is <= tol |b| or after
    ``restart`` steps.  Returns (u, iterations, relative residuals: the least-squares value
    after every step)."""
    u = np.zeros_like(b) if u0 is None else u0.copy()
    nb = np.linalg.norm(b)
    r = b - apply(u)
    hist = [np.linalg.norm(r) / nb]
    k = 0
    while hist[-1] > tol and k < max_iter:
        beta = np.linalg.norm(r)
        V = [r / beta]
        Z = []
        Hbar = np.zeros((restart + 1, restart))
        y = np.zeros(0)
        for j in range(restart):
            Z.append(precond(V[j]))
            w = apply(Z[j])
            for i in range(j + 1):
                Hbar[i, j] = w @ V[i]
                w = w - Hbar[i, j] * V[i]
            Hbar[j + 1, j] = np.linalg.norm(w)
            V.append(w / Hbar[j + 1, j] if Hbar[j + 1, j] > 0 else w)
            e1 = np.zeros(j + 2)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(Hbar[:j + 2, :j + 1], e1, rcond=None)
            k += 1
            hist.append(np.linalg.norm(e1 - Hbar[:j + 2, :j + 1] @ y) / nb)
            if hist[-1] <= tol or k >= max_iter or Hbar[j + 1, j] == 0:
                break
        u = u + np.array(Z).T @ y
        r = b - apply(u)
        hist[-1] = np.linalg.norm(r) / nb  # the true residual at the end of the cycle
    return u, k, hist
