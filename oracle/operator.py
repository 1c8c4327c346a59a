"""SIPG operator of the paper, applied matrix-free by quadrature; assembled form; RHS; norms.

Bilinear form (Sec. II.A.2, Eqs. lh / lh2 / lh3, read as -div(k grad u) + c u = g):
  L(u, v) = sum_e int_e k grad u . grad v + c u v
          - sum_{m in M_ID} int_m [[u]] . {{k grad v}} + [[v]] . {{k grad u}}
          + sum_{m in M_ID} int_m sigma [[u]] . [[v]]
with [[q]] = q+ n+ + q- n-, {{q}} = (q+ + q-)/2 inside (Eq. 20), [[q]] = q n,
{{q}} = q on Dirichlet faces.  Neumann faces add no operator term.

Quadrature (Sec. II.A.5, Eqs. stiffness-3, harald-stiff, temp-E): polynomials are
interpolated from LGL nodes to GL points; geometry is evaluated at GL points.  The
number of GL points is one of the readings listed with the design notes: q = p + 1 on
affine elements with constant k (exact), q = p + 1 + quad_extra otherwise; mortars use
q_m = p_m + 1 (+ quad_extra when a side is curved or k varies), p_m = max(p-, p+).
Mortar geometry (S^m, normal) comes from the finer side (equal levels: the lower
element index), whose face coordinates parametrise the mortar.

Penalty (Eq. penaltyparameter): sigma = C p_m^2 / h_m, h_m = 2 min_side 1/|grad xi_j|
(the thickness of the side normal to the face), evaluated at each mortar point,
multiplied by max(k-, k+) at the point.

Coefficients k (diffusion) and c (mass, the f u term of Eq. Laplacian read with the sign of
Eq. lh) come from the problem (k analytic), from a mass callable c(x), or from tables: one
value per element, or nodal values in the level-vector layout whose LGL interpolant on each
element gives the value at any point of that element.  A tabulated k may jump across a
mortar; each side then uses its own value: {{k grad u}} = (k- grad u- + k+ grad u+) / 2.
"""
import numpy as np

from . import geometry, rules, problems
from .mesh import build_mortars, face_point, minus_to_plus

DIRICHLET, NEUMANN, ROBIN = 1, 2, 3


def _basis_at(n, xi):
    """Tensor LGL basis of n nodes per axis at reference points xi [P, 3].

    Returns V [P, n^3] and Dxi [3, P, n^3]; local index alpha = i + n j + n^2 k
    (x fastest) for the node (xi_i, xi_j, xi_k).
    """
    nodes, _ = rules.lgl(n)
    L = [rules.lagrange(nodes, xi[:, d]) for d in range(3)]
    D = [rules.lagrange_deriv(nodes, xi[:, d]) for d in range(3)]
    V = np.einsum("pk,pj,pi->pkji", L[2], L[1], L[0]).reshape(len(xi), -1)
    D0 = np.einsum("pk,pj,pi->pkji", L[2], L[1], D[0]).reshape(len(xi), -1)
    D1 = np.einsum("pk,pj,pi->pkji", L[2], D[1], L[0]).reshape(len(xi), -1)
    D2 = np.einsum("pk,pj,pi->pkji", D[2], L[1], L[0]).reshape(len(xi), -1)
    return V, np.stack([D0, D1, D2])


class SIPG:
    """The discrete operator A (y = A u) and right-hand side F on one cell mesh."""

    def __init__(self, mesh, problem=None, C=10.0, quad_extra=1, bc_override=None,
                 mass=None, active=None, kfield=None, cfield=None, robin_gamma=0.0):
        """``active``: optional element subset; the operator is then formed only for the
        rows of those elements (their volume terms and the mortars touching them), so that
        (A x) restricted to them is exact while the rest of the output stays zero.
        ``kfield`` / ``cfield``: tabulated diffusion / mass coefficient, dict(where="element",
        values=[E]) or dict(where="node", values=[ndof]) (replaces the problem's k / ``mass``)."""
        self.mesh = mesh
        self.problem = problem
        self.C = float(C)
        self.gamma = float(robin_gamma)  # Robin coefficient: k n.grad u + gamma u = g_R
        self.quad_extra = int(quad_extra)
        self.mass = mass  # callable c(x) >= 0 or None
        self.kfield, self.cfield = kfield, cfield
        if cfield is not None:
            self.mass = self._mass_from_field
        p = mesh["elem_p"].astype(np.int64)
        self.E = len(p)
        self.n = p + 1
        self.offsets = np.concatenate([[0], np.cumsum(self.n ** 3)])
        self.ndof = int(self.offsets[-1])
        self.kconst = problems.k_is_constant(problem) and kfield is None
        self.affine = geometry.is_affine_macro(mesh["macro_kind"][mesh["elem_macro"]])
        self.mortars = build_mortars(mesh)
        self.active = None
        if active is not None:
            self.active = np.zeros(self.E, bool)
            self.active[np.asarray(active)] = True
        if bc_override is not None:
            for mt in self.mortars:
                if mt["ep"] < 0:
                    mt["bc"] = bc_override
        self._setup_volume()
        self._setup_faces()

    # -- quadrature choices -----------------------------------------------------
    def q_volume(self, e):
        exact = self.affine[e] and self.kconst and self.mass is None
        return int(self.n[e]) + (0 if exact else self.quad_extra)

    def q_mortar(self, mt):
        pm = int(self.n[mt["em"]])
        curved = not self.affine[mt["em"]]
        if mt["ep"] >= 0:
            pm = max(pm, int(self.n[mt["ep"]]))
            curved = curved or not self.affine[mt["ep"]]
        return pm + (self.quad_extra if (curved or not self.kconst) else 0)

    def k(self, x):
        return problems.k_of(self.problem, x)

    def _field_at(self, field, elems, xi):
        """A tabulated coefficient at reference points xi [..., 3] of elements ``elems``
        (broadcast against xi[..., 0])."""
        elems = np.broadcast_to(np.asarray(elems), xi.shape[:-1])
        vals = np.asarray(field["values"], float)
        if field["where"] == "element":
            return vals[elems]
        out = np.zeros(xi.shape[:-1])
        for e in np.unique(elems):
            sel = elems == e
            V, _ = _basis_at(int(self.n[e]), xi[sel])
            out[sel] = V @ vals[self.offsets[e]:self.offsets[e + 1]]
        return out

    def k_at(self, elems, xi, x):
        """k at the physical points x = Phi_e(xi) of elements ``elems``."""
        if self.kfield is None:
            return self.k(x)
        return self._field_at(self.kfield, elems, xi)

    def _mass_from_field(self, x, elems=None, xi=None):
        return self._field_at(self.cfield, elems, xi)

    def c_at(self, elems, xi, x):
        """Mass coefficient c at the points x = Phi_e(xi) of elements ``elems``."""
        if self.cfield is not None:
            return self._field_at(self.cfield, elems, xi)
        return self.mass(x)

    # -- volume -------------------------------------------------------------------
    def _setup_volume(self):
        groups = {}
        for e in range(self.E):
            if self.active is not None and not self.active[e]:
                continue
            groups.setdefault((int(self.n[e]), self.q_volume(e)), []).append(e)
        self.vgroups = []
        for (n, q), elems in sorted(groups.items()):
            elems = np.array(elems)
            lgl_x, _ = rules.lgl(n)
            eta, w = rules.gl(q)
            B = rules.lagrange(lgl_x, eta)
            Dt = rules.lagrange_deriv(lgl_x, eta)
            xi = np.stack(np.meshgrid(eta, eta, eta, indexing="ij")[::-1], axis=-1).reshape(-1, 3)
            W = np.einsum("c,b,a->cba", w, w, w).reshape(-1)
            x, J = geometry.element_map(self.mesh, elems[:, None], xi[None])
            det = np.linalg.det(J)
            if np.any(det <= 0):
                raise ValueError("non-positive Jacobian determinant")
            Ji = np.linalg.inv(J)  # Ji[d, i] = dxi_d / dx_i
            xie = np.broadcast_to(xi, x.shape)
            G = np.einsum("epdi,epci->epdc", Ji, Ji) * (W * det * self.k_at(elems[:, None], xie, x))[:, :, None, None]
            M = None
            if self.mass is not None:
                M = W * det * self.c_at(elems[:, None], xie, x)
            idx = self.offsets[elems][:, None] + np.arange(n ** 3)[None, :]
            self.vgroups.append(dict(n=n, q=q, elems=elems, B=B, Dt=Dt, G=G, M=M, idx=idx,
                                     x=x, W=W, det=det, xi=xi))

    def _volume(self, u, y):
        for g in self.vgroups:
            n, q = g["n"], g["q"]
            B, Dt = g["B"], g["Dt"]
            U = u[g["idx"]].reshape(-1, n, n, n)
            d0 = np.einsum("ck,bj,ai,ekji->ecba", B, B, Dt, U, optimize=True)
            d1 = np.einsum("ck,bj,ai,ekji->ecba", B, Dt, B, U, optimize=True)
            d2 = np.einsum("ck,bj,ai,ekji->ecba", Dt, B, B, U, optimize=True)
            grad = np.stack([d0, d1, d2], axis=-1).reshape(len(U), q ** 3, 3)
            F = np.einsum("epdc,epc->epd", g["G"], grad).reshape(len(U), q, q, q, 3)
            Y = (np.einsum("ck,bj,ai,ecba->ekji", B, B, Dt, F[..., 0], optimize=True)
                 + np.einsum("ck,bj,ai,ecba->ekji", B, Dt, B, F[..., 1], optimize=True)
                 + np.einsum("ck,bj,ai,ecba->ekji", Dt, B, B, F[..., 2], optimize=True))
            if g["M"] is not None:
                uq = np.einsum("ck,bj,ai,ekji->ecba", B, B, B, U, optimize=True).reshape(len(U), -1)
                Y += np.einsum("ck,bj,ai,ecba->ekji", B, B, B,
                               (g["M"] * uq).reshape(len(U), q, q, q), optimize=True)
            y[g["idx"]] += Y.reshape(len(U), -1)

    # -- faces --------------------------------------------------------------------
    def _setup_faces(self):
        groups = {}
        for mi, mt in enumerate(self.mortars):
            if mt["ep"] < 0 and mt["bc"] not in (DIRICHLET, ROBIN):
                continue  # Neumann faces: no operator term
            if self.active is not None and not (self.active[mt["em"]] or
                                                (mt["ep"] >= 0 and self.active[mt["ep"]])):
                continue
            nm = int(self.n[mt["em"]])
            npl = int(self.n[mt["ep"]]) if mt["ep"] >= 0 else 0
            key = (nm, npl, self.q_mortar(mt), mt["fm"], mt["fp"], mt["o"], mt["sub"], mt["bc"])
            groups.setdefault(key, []).append(mi)
        self.fgroups = []
        for key, mis in groups.items():
            nm, npl, qm, fm, fp, o, sub, bc = key
            eta, w = rules.gl(qm)
            s, t = np.meshgrid(eta, eta, indexing="xy")  # point rho = c + qm d: s = eta_c, t = eta_d
            s, t = s.reshape(-1), t.reshape(-1)
            wst = np.outer(w, w).reshape(-1)
            mt0 = self.mortars[mis[0]]
            xim = face_point(fm, s, t)
            Vm, Dm = _basis_at(nm, xim)
            em = np.array([self.mortars[i]["em"] for i in mis])
            x, Jm = geometry.element_map(self.mesh, em[:, None], xim[None])
            Jim = np.linalg.inv(Jm)
            detm = np.linalg.det(Jm)
            dm, sm = divmod(fm, 2)
            row = Jim[:, :, dm, :]
            nrm = np.linalg.norm(row, axis=-1)
            S = detm * nrm
            nhat = (1.0 if sm else -1.0) * row / nrm[..., None]
            wS = wst[None, :] * S
            hmin = 2.0 / nrm
            pm = nm - 1
            km = self.k_at(em[:, None], np.broadcast_to(xim, x.shape), x)
            kp = km
            g = dict(key=key, mis=np.array(mis), em=em, wS=wS, x=x, Vm=Vm, Dm=Dm, xim=xim, wst=wst,
                     mvec_m=np.einsum("mpdi,mpi->mpd", Jim, nhat), nhat=nhat,
                     idx_m=self.offsets[em][:, None] + np.arange(nm ** 3)[None, :])
            if npl:
                a, b = minus_to_plus(mt0, s, t)
                xip = face_point(fp, a, b)
                Vp, Dp = _basis_at(npl, xip)
                ep = np.array([self.mortars[i]["ep"] for i in mis])
                xp, Jp = geometry.element_map(self.mesh, ep[:, None], xip[None])
                Jip = np.linalg.inv(Jp)
                dp_ = fp // 2
                nrp = np.linalg.norm(Jip[:, :, dp_, :], axis=-1)
                hmin = np.minimum(hmin, 2.0 / nrp)
                pm = max(pm, npl - 1)
                kp = self.k_at(ep[:, None], np.broadcast_to(xip, xp.shape), xp)
                g.update(ep=ep, Vp=Vp, Dp=Dp, xp=xp, xip=xip,
                         mvec_p=np.einsum("mpdi,mpi->mpd", Jip, -nhat),
                         idx_p=self.offsets[ep][:, None] + np.arange(npl ** 3)[None, :])
            g["robin"] = bc == ROBIN
            g["hmin"] = hmin      # h_m at each point (Eq. penaltyparameter, reading R3)
            g["pm"] = pm          # p_m = max(p-, p+)
            g["kx"] = km          # the minus side's k (its own side of the mortar)
            g["kp"] = kp          # the plus side's k (= km where k is continuous)
            g["sigma"] = self.C * pm * pm / hmin * np.maximum(km, kp)
            self.fgroups.append(g)

    def _faces(self, u, y):
        for g in self.fgroups:
            wS, kx, sig = g["wS"], g["kx"], g["sigma"]
            Um = u[g["idx_m"]]
            um = Um @ g["Vm"].T
            # physical normal derivative n.grad u = (J^-1 n) . grad_xi u
            gm = np.einsum("mpd,dpa,ma->mp", g["mvec_m"], g["Dm"], Um)
            if "ep" in g:
                Up = u[g["idx_p"]]
                up = Up @ g["Vp"].T
                gp = np.einsum("mpd,dpa,ma->mp", g["mvec_p"], g["Dp"], Up)
                # side -: jump j = u- - u+, n-.({{k grad u}}) = (k- g- - k+ g+) / 2
                kp = g["kp"]
                jm = um - up
                Am = wS * (sig * jm - 0.5 * (kx * gm - kp * gp))
                Bm = -0.5 * wS * kx * jm
                Ap, Bp = -Am, 0.5 * wS * kp * jm  # side +: j+ = -j-, n+ = -n-, its own k
                ym = Am @ g["Vm"] + np.einsum("mp,mpd,dpa->ma", Bm, g["mvec_m"], g["Dm"])
                yp = Ap @ g["Vp"] + np.einsum("mp,mpd,dpa->ma", Bp, g["mvec_p"], g["Dp"])
                np.add.at(y, g["idx_m"], ym)
                np.add.at(y, g["idx_p"], yp)
            elif g["robin"]:  # Robin face: int gamma u v (the flux k n.grad u enters as data)
                np.add.at(y, g["idx_m"], (wS * self.gamma * um) @ g["Vm"])
            else:  # Dirichlet face: [[u]] = u n, {{k grad u}} = k grad u
                A = wS * (sig * um - kx * gm)
                Bc = -wS * kx * um
                ym = A @ g["Vm"] + np.einsum("mp,mpd,dpa->ma", Bc, g["mvec_m"], g["Dm"])
                np.add.at(y, g["idx_m"], ym)

    # -- public ---------------------------------------------------------------------
    def apply(self, u):
        u = np.asarray(u, float)
        y = np.zeros(self.ndof)
        self._volume(u, y)
        self._faces(u, y)
        return y

    def diagonal(self):
        """diag(A): the bilinear form of each basis function with itself.

        Volume: sum_sigma grad psi . G grad psi (+ mass).  Faces, side s with u = psi on
        that side only: sum_rho wS (sigma psi^2 - k psi n.grad psi) inside (the two
        halves of the consistency and symmetry terms), sum_rho wS (sigma psi^2 -
        2 k psi n.grad psi) on Dirichlet faces.
        """
        dg = np.zeros(self.ndof)
        for g in self.vgroups:
            n, q = g["n"], g["q"]
            B, Dt = g["B"], g["Dt"]
            G = g["G"].reshape(-1, q, q, q, 3, 3)
            ops = [(Dt, B, B), (B, Dt, B), (B, B, Dt)]  # (x, y, z) factor of d/dxi_d
            out = np.zeros((len(G), n, n, n))
            for d in range(3):
                for e in range(3):
                    fx = ops[d][0] * ops[e][0]
                    fy = ops[d][1] * ops[e][1]
                    fz = ops[d][2] * ops[e][2]
                    out += np.einsum("ecba,ck,bj,ai->ekji", G[..., d, e], fz, fy, fx, optimize=True)
            if g["M"] is not None:
                out += np.einsum("ecba,ck,bj,ai->ekji", g["M"].reshape(-1, q, q, q),
                                 B * B, B * B, B * B, optimize=True)
            dg[g["idx"]] += out.reshape(len(G), -1)
        for g in self.fgroups:
            wS, kx, sig = g["wS"], g["kx"], g["sigma"]
            if g["robin"]:
                np.add.at(dg, g["idx_m"], (wS * self.gamma) @ (g["Vm"] * g["Vm"]))
                continue
            sides = [("Vm", "Dm", "mvec_m", "idx_m", kx)]
            if "ep" in g:
                sides.append(("Vp", "Dp", "mvec_p", "idx_p", g["kp"]))
            factor = 1.0 if "ep" in g else 2.0
            for V, D, mv, idx, ks in sides:
                psi = g[V]                                      # [p, a]
                gn = np.einsum("mpd,dpa->mpa", g[mv], g[D])     # n.grad psi per mortar
                val = (wS * sig) @ (psi * psi) - factor * np.einsum("mp,pa,mpa->ma", wS * ks, psi, gn)
                np.add.at(dg, g[idx], val)
        return dg

    def rhs(self, problem=None):
        """F(psi) = int g psi + sum_{Dirichlet} int g_D (-k n.grad psi + sigma psi)  (Eq. Fh2)
        + sum_{Neumann} int g_N psi (Eq. NeumannBC) + sum_{Robin} int g_R psi (Eq. RobinBC with
        the sign of Eq. lh: k n.grad u + gamma u = g_R, whose gamma u v enters the operator)."""
        problem = problem if problem is not None else self.problem
        F = np.zeros(self.ndof)
        for g in self.vgroups:
            n, q = g["n"], g["q"]
            B = g["B"]
            gx = problems.source_g(problem, g["x"]) * g["W"] * g["det"]
            F[g["idx"]] += np.einsum("ck,bj,ai,ecba->ekji", B, B, B,
                                     gx.reshape(-1, q, q, q), optimize=True).reshape(len(gx), -1)
        for g in self.fgroups:
            if "ep" in g or g["robin"]:
                continue
            gd = problems.dirichlet_g(problem, g["x"])
            A = g["wS"] * g["sigma"] * gd
            Bc = -g["wS"] * g["kx"] * gd
            ym = A @ g["Vm"] + np.einsum("mp,mpd,dpa->ma", Bc, g["mvec_m"], g["Dm"])
            np.add.at(F, g["idx_m"], ym)
        # Neumann faces (Eq. NeumannBC): the boundary term int g_N psi of the integration by
        # parts, with the face's own rule
        for mt in self.mortars:
            if mt["ep"] >= 0 or mt["bc"] not in (NEUMANN, ROBIN):
                continue
            em, fm, nm, qm = mt["em"], mt["fm"], int(self.n[mt["em"]]), self.q_mortar(mt)
            eta, w = rules.gl(qm)
            s_, t_ = np.meshgrid(eta, eta, indexing="xy")
            xim = face_point(fm, s_.reshape(-1), t_.reshape(-1))
            Vm, _ = _basis_at(nm, xim)
            x, J = geometry.element_map(self.mesh, np.array([[em]]), xim[None])
            row = np.linalg.inv(J)[0, :, fm // 2, :]
            nrm = np.linalg.norm(row, axis=-1)
            nhat = (1.0 if fm % 2 else -1.0) * row / nrm[:, None]
            wS = np.outer(w, w).reshape(-1) * np.linalg.det(J)[0] * nrm
            gN = problems.neumann_g(problem, x[0], nhat, self.k_at(np.full(len(xim), em), xim, x[0]))
            if mt["bc"] == ROBIN:  # g_R = k n.grad u + gamma u (Eq. RobinBC, sign of Eq. lh)
                gN = gN + self.gamma * problems.robin_u(problem, x[0])
            F[self.offsets[em] + np.arange(nm ** 3)] += (wS * gN) @ Vm
        return F

    def interpolate(self, func):
        """Nodal interpolant: the value of func at every element's LGL nodes."""
        u = np.zeros(self.ndof)
        for n in sorted(set(int(x) for x in self.n)):
            elems = np.where(self.n == n)[0]
            xl, _ = rules.lgl(n)
            xi = np.stack(np.meshgrid(xl, xl, xl, indexing="ij")[::-1], axis=-1).reshape(-1, 3)
            x, _ = geometry.element_map(self.mesh, elems[:, None], xi[None])
            u[self.offsets[elems][:, None] + np.arange(n ** 3)[None, :]] = func(x)
        return u

    def nodes(self):
        """Physical coordinates of every degree of freedom, [ndof, 3]."""
        X = np.zeros((self.ndof, 3))
        for n in sorted(set(int(x) for x in self.n)):
            elems = np.where(self.n == n)[0]
            xl, _ = rules.lgl(n)
            xi = np.stack(np.meshgrid(xl, xl, xl, indexing="ij")[::-1], axis=-1).reshape(-1, 3)
            x, _ = geometry.element_map(self.mesh, elems[:, None], xi[None])
            X[self.offsets[elems][:, None] + np.arange(n ** 3)[None, :]] = x
        return X

    def l2_error(self, u, func, extra=3):
        """||u_h - func||_{L2} with q = p + 1 + extra GL points per axis (Eq. l2norm)."""
        err2 = 0.0
        for n in sorted(set(int(x) for x in self.n)):
            elems = np.where(self.n == n)[0]
            q = n + extra
            eta, w = rules.gl(q)
            xl, _ = rules.lgl(n)
            B = rules.lagrange(xl, eta)
            xi = np.stack(np.meshgrid(eta, eta, eta, indexing="ij")[::-1], axis=-1).reshape(-1, 3)
            W = np.einsum("c,b,a->cba", w, w, w).reshape(-1)
            x, J = geometry.element_map(self.mesh, elems[:, None], xi[None])
            U = u[self.offsets[elems][:, None] + np.arange(n ** 3)[None, :]].reshape(-1, n, n, n)
            uq = np.einsum("ck,bj,ai,ekji->ecba", B, B, B, U, optimize=True).reshape(len(elems), -1)
            err2 += float(np.sum(W * np.linalg.det(J) * (uq - func(x)) ** 2))
        return np.sqrt(err2)


    def energy_error(self, u, func, grad_func, extra=3):
        """||func - u_h||_* of Eq. energynorm: the broken H1 seminorm of the error on every
        element plus the penalty-weighted squared jumps on every mortar where the penalty
        acts (interior and Dirichlet faces; on a Dirichlet face the jump of nu is nu n).
        ``func`` and ``grad_func`` give the exact solution and its physical gradient at
        points [..., 3].  Integrals use q = p + 1 + extra GL points per axis (volume) and
        p_m + 1 + extra (mortars); sigma = C p_m^2 / h_m as in Eq. penaltyparameter, without
        the coefficient k (the norm as printed)."""
        u = np.asarray(u, float)
        err2 = 0.0
        for n in sorted(set(int(x) for x in self.n)):
            elems = np.where(self.n == n)[0]
            q = n + extra
            eta, w = rules.gl(q)
            xi = np.stack(np.meshgrid(eta, eta, eta, indexing="ij")[::-1], axis=-1).reshape(-1, 3)
            W = np.einsum("c,b,a->cba", w, w, w).reshape(-1)
            _, D = _basis_at(n, xi)                               # [3, P, n^3]
            x, J = geometry.element_map(self.mesh, elems[:, None], xi[None])
            Ji = np.linalg.inv(J)                                 # [E, P, d, i]
            U = u[self.offsets[elems][:, None] + np.arange(n ** 3)[None, :]]
            gxi = np.einsum("dpa,ea->epd", D, U)                  # reference gradient
            gx = np.einsum("epdi,epd->epi", Ji, gxi)              # physical gradient
            diff = grad_func(x) - gx
            err2 += float(np.sum(W * np.linalg.det(J) * np.sum(diff * diff, axis=-1)))
        for mt in self.mortars:
            if mt["ep"] < 0 and mt["bc"] != DIRICHLET:
                continue
            em, fm = mt["em"], mt["fm"]
            nm = int(self.n[em])
            pm = nm - 1
            if mt["ep"] >= 0:
                pm = max(pm, int(self.n[mt["ep"]]) - 1)
            qm = pm + 1 + extra
            eta, w = rules.gl(qm)
            s, t = np.meshgrid(eta, eta, indexing="xy")
            s, t = s.reshape(-1), t.reshape(-1)
            xim = face_point(fm, s, t)
            x, J = geometry.element_map(self.mesh, np.full(len(s), em), xim)
            row = np.linalg.inv(J)[:, fm // 2, :]
            nrm = np.linalg.norm(row, axis=-1)
            dS = np.outer(w, w).reshape(-1) * np.linalg.det(J) * nrm
            h = 2.0 / nrm
            Vm, _ = _basis_at(nm, xim)
            um = Vm @ u[self.offsets[em] + np.arange(nm ** 3)]
            if mt["ep"] >= 0:
                ep, fp = mt["ep"], mt["fp"]
                npl = int(self.n[ep])
                a, b = minus_to_plus(mt, s, t)
                xip = face_point(fp, a, b)
                _, Jp = geometry.element_map(self.mesh, np.full(len(s), ep), xip)
                h = np.minimum(h, 2.0 / np.linalg.norm(np.linalg.inv(Jp)[:, fp // 2, :], axis=-1))
                Vp, _ = _basis_at(npl, xip)
                jump = Vp @ u[self.offsets[ep] + np.arange(npl ** 3)] - um  # (u - u_h-) - (u - u_h+)
            else:
                jump = func(x) - um
            err2 += float(np.sum(dS * (self.C * pm * pm / h) * jump * jump))
        return np.sqrt(err2)


def element_blocks(op):
    """Diagonal blocks A_ee (element with itself) of the operator, one dense matrix per element.

    The volume term of the element plus, for every mortar it touches, its own-side block
    (the four-block face term of ``assemble_dense`` restricted to trial = test = this side).
    """
    blocks = [np.zeros((int(n) ** 3, int(n) ** 3)) for n in op.n]
    for g in op.vgroups:
        n, q = g["n"], g["q"]
        eta, w = rules.gl(q)
        xi = np.stack(np.meshgrid(eta, eta, eta, indexing="ij")[::-1], axis=-1).reshape(-1, 3)
        V, D = _basis_at(n, xi)
        W = np.einsum("c,b,a->cba", w, w, w).reshape(-1)
        for e in g["elems"]:
            x, J = geometry.element_map(op.mesh, np.full(len(xi), e), xi)
            Ji = np.linalg.inv(J)
            grad = np.einsum("pdi,dpa->pai", Ji, D)
            kv = op.k_at(np.full(len(xi), e), xi, x)
            blocks[e] += np.einsum("p,pai,pbi->ba", W * np.linalg.det(J) * kv, grad, grad)
            if op.mass is not None:
                cv = op.c_at(np.full(len(xi), e), xi, x)
                blocks[e] += np.einsum("p,pa,pb->ba", W * np.linalg.det(J) * cv, V, V)
    for g in op.fgroups:
        wS, kx, sig = g["wS"], g["kx"], g["sigma"]
        if g["robin"]:
            for i, e in enumerate(g["em"]):
                blocks[e] += np.einsum("p,pa,pb->ba", wS[i] * op.gamma, g["Vm"], g["Vm"])
            continue
        sides = [("Vm", "Dm", "mvec_m", "em", kx)]
        if "ep" in g:
            sides.append(("Vp", "Dp", "mvec_p", "ep", g["kp"]))
        half = 0.5 if "ep" in g else 1.0
        for V, D, mv, el, ks in sides:
            psi = g[V]
            for i, e in enumerate(g[el]):
                gn = np.einsum("pd,dpa->pa", g[mv][i], g[D])   # n.grad psi at the points
                wk = wS[i] * ks[i]
                blk = (np.einsum("p,pa,pb->ba", wS[i] * sig[i], psi, psi)
                       - half * np.einsum("p,pa,pb->ba", wk, psi, gn)
                       - half * np.einsum("p,pa,pb->ba", wk, gn, psi))
                blocks[e] += blk
    return blocks


def assemble_dense(op):
    """Brute-force dense matrix A[beta, alpha] = L(psi_alpha, psi_beta) for tiny meshes.

    Written independently of the matrix-free path: every basis function's physical
    gradient is formed explicitly at every quadrature point, and the face terms use the
    vector jumps and averages of Eq. 20 directly (the four blocks --, -+, +-, ++).
    """
    N = op.ndof
    A = np.zeros((N, N))
    for g in op.vgroups:
        n, q = g["n"], g["q"]
        lgl_x, _ = rules.lgl(n)
        eta, w = rules.gl(q)
        xi = np.stack(np.meshgrid(eta, eta, eta, indexing="ij")[::-1], axis=-1).reshape(-1, 3)
        V, D = _basis_at(n, xi)
        W = np.einsum("c,b,a->cba", w, w, w).reshape(-1)
        for le, e in enumerate(g["elems"]):
            x, J = geometry.element_map(op.mesh, np.full(len(xi), e), xi)
            Ji = np.linalg.inv(J)
            det = np.linalg.det(J)
            kx = op.k_at(np.full(len(xi), e), xi, x)
            grad = np.einsum("pdi,dpa->pai", Ji, D)  # physical gradient of every basis function
            Ke = np.einsum("p,pai,pbi->ba", W * det * kx, grad, grad)
            if op.mass is not None:
                Ke += np.einsum("p,pa,pb->ba", W * det * op.c_at(np.full(len(xi), e), xi, x), V, V)
            sl = slice(op.offsets[e], op.offsets[e + 1])
            A[sl, sl] += Ke
    for mt in op.mortars:
        if mt["ep"] < 0 and mt["bc"] == ROBIN:
            # Robin face: int gamma psi_a psi_b over the face (its own rule)
            qm = op.q_mortar(mt)
            eta, w = rules.gl(qm)
            s, t = np.meshgrid(eta, eta, indexing="xy")
            xim = face_point(mt["fm"], s.reshape(-1), t.reshape(-1))
            _, J = geometry.element_map(op.mesh, np.full(len(xim), mt["em"]), xim)
            rowv = np.linalg.inv(J)[:, mt["fm"] // 2, :]
            dS = np.outer(w, w).reshape(-1) * np.linalg.det(J) * np.linalg.norm(rowv, axis=-1)
            V, _ = _basis_at(int(op.n[mt["em"]]), xim)
            sl = slice(op.offsets[mt["em"]], op.offsets[mt["em"] + 1])
            A[sl, sl] += np.einsum("p,pa,pb->ba", dS * op.gamma, V, V)
            continue
        if mt["ep"] < 0 and mt["bc"] != DIRICHLET:
            continue
        qm = op.q_mortar(mt)
        eta, w = rules.gl(qm)
        s, t = np.meshgrid(eta, eta, indexing="xy")
        s, t = s.reshape(-1), t.reshape(-1)
        wst = np.outer(w, w).reshape(-1)
        sides = []
        em, fm = mt["em"], mt["fm"]
        xim = face_point(fm, s, t)
        x, J = geometry.element_map(op.mesh, np.full(len(s), em), xim)
        Ji = np.linalg.inv(J)
        d, sd = divmod(fm, 2)
        row = Ji[:, d, :]
        nrm = np.linalg.norm(row, axis=-1)
        nvec = (1.0 if sd else -1.0) * row / nrm[:, None]
        dS = wst * np.linalg.det(J) * nrm
        V, D = _basis_at(int(op.n[em]), xim)
        km = op.k_at(np.full(len(s), em), xim, x)
        sides.append((em, V, np.einsum("pdi,dpa->pai", Ji, D), nvec, km))
        h = 2.0 / nrm
        pm = int(op.n[em]) - 1
        kmax = km
        if mt["ep"] >= 0:
            ep, fp = mt["ep"], mt["fp"]
            a, b = minus_to_plus(mt, s, t)
            xip = face_point(fp, a, b)
            xpp, Jp = geometry.element_map(op.mesh, np.full(len(s), ep), xip)
            Jip = np.linalg.inv(Jp)
            Vp, Dp = _basis_at(int(op.n[ep]), xip)
            kp = op.k_at(np.full(len(s), ep), xip, xpp)
            sides.append((ep, Vp, np.einsum("pdi,dpa->pai", Jip, Dp), -nvec, kp))
            h = np.minimum(h, 2.0 / np.linalg.norm(Jip[:, fp // 2, :], axis=-1))
            pm = max(pm, int(op.n[ep]) - 1)
            kmax = np.maximum(km, kp)
        sigma = op.C * pm * pm / h * kmax
        half = 0.5 if len(sides) == 2 else 1.0
        for (eu, Vu, Gu, nu, ku) in sides:        # trial side
            for (ev, Vv, Gv, nv, kv) in sides:    # test side
                jump_u = Vu[:, :, None] * nu[:, None, :]          # [[psi_u]]  (p, a, i)
                jump_v = Vv[:, :, None] * nv[:, None, :]
                avg_u = half * ku[:, None, None] * Gu               # {{k grad psi_u}}
                avg_v = half * kv[:, None, None] * Gv
                blk = (-np.einsum("p,pai,pbi->ba", dS, jump_u, avg_v)
                       - np.einsum("p,pbi,pai->ba", dS, jump_v, avg_u)
                       + np.einsum("p,pai,pbi->ba", dS * sigma, jump_u, jump_v))
                A[op.offsets[ev]:op.offsets[ev + 1], op.offsets[eu]:op.offsets[eu + 1]] += blk
    return A
