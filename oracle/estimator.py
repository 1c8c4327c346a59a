"""A posteriori error estimator and the smooth-pred hp-refinement decisions (Sec. II.E).

Test infrastructure: only the tests, the smoke check and the CPU baseline of the benchmark use
this package.  Plain FP64 numpy on the quadrature of ``operator.SIPG``.

Estimator (Eqs. Eta2_Ingredients, Eta2_Integrals, Eta2_Local) for -div(k grad u) + c u = g
(Eq. classofproblems with a = k grad u, f = c u - g):

  R_e     = g + div(k grad u_h) - c u_h                              on each element
  J_{m,1} = [[k grad u_h]] = k- n-.grad u- + k+ n+.grad u+            interior mortars
  J_{m,2} = [[u_h]] = u- - u+                                         interior mortars
  J_{m,3} = u_h - g_D                                                 Dirichlet mortars

  eta2_e     = h_e^2 p_e^2 int_e R_e^2
  eta2_{m,1} = int_m (h_m / p_m) J_{m,1}^2
  eta2_{m,2} = int_m sigma J_{m,2}^2,   eta2_{m,3} = int_m sigma J_{m,3}^2
  eta2(e)    = eta2_e + sum over the interior mortars touching e of eta2_{m,1} + eta2_{m,2}
               + sum over the Dirichlet mortars of e of eta2_{m,3}.

Readings (listed with the design notes): the jump weight printed as sigma h_m^-1 p_m^2 is the
penalty sigma = C p_m^2 / h_m of Eq. penaltyparameter itself (times max(k-, k+), as in the
operator), evaluated with h_m at each mortar point, and h_m / p_m likewise pointwise with p_m
= max(p-, p+); div(k grad u_h) is evaluated at the element's volume GL points as
(1 / det J) sum_d d/dxi_d (det J k (J^-1 J^-T grad_xi u_h)_d), the derivative taken by the GL
collocation derivative of the volume rule (exact on affine elements with a constant k, where the
contravariant flux is a polynomial of degree <= p in each coordinate); h_e is the largest
distance between two vertices of the element; Robin and Neumann mortars add no term.

Fiducial grid (Sec. II.E, applied to the compactified shell in Sec. III.C): the integrands
(R, the jumps) are evaluated on the physical grid, while the integration weights (W det J,
w S), h_e and h_m (and with it sigma) come from a second grid of the same cells under other
macro maps, at the same reference points.

Driver (Alg. hpamr, smooth-pred): an element marked for refinement is h-refined when its
eta2 exceeds the predicted eta2_pred, its children then predicting
gamma_h (1/2)^d (1/2)^(2 p_e) eta2(e); otherwise it is p-refined and predicts gamma_p eta2(e).
An element without a prediction (every element at the start, as the text requires: each is
p-refined first) is p-refined.  Marking takes the given fraction of elements with the largest
eta2 (ties by element index) or those above a factor times the mean.
"""
import numpy as np

from . import geometry, problems, rules

DIRICHLET, ROBIN = 1, 3


def element_diameters(mesh):
    """h_e: the largest distance between two of each element's eight vertices."""
    E = len(mesh["elem_p"])
    corners = np.array([[a, b, c] for c in (-1.0, 1.0) for b in (-1.0, 1.0) for a in (-1.0, 1.0)])
    x, _ = geometry.element_map(mesh, np.arange(E)[:, None], corners[None])
    d = np.linalg.norm(x[:, :, None, :] - x[:, None, :, :], axis=-1)
    return d.reshape(E, -1).max(axis=1)


def _face_metric(mesh, elems, xi, f):
    """S = det J |grad xi_d| and |grad xi_d| (d the face's axis) at reference points xi of elems."""
    _, J = geometry.element_map(mesh, elems[:, None], xi[None])
    nrm = np.linalg.norm(np.linalg.inv(J)[:, :, f // 2, :], axis=-1)
    return np.linalg.det(J) * nrm, nrm


def estimate(op, u, problem=None, fiducial=None):
    """eta2(e) of the nodal vector u on the mesh of ``op`` (an operator.SIPG); returns a dict
    with eta2 (per element), eta2_vol (per element), eta2_face (per mortar of op.mortars) and
    its flux-jump and value-jump parts eta2_flux, eta2_jump.  ``fiducial``: a mesh with the same
    cells (and macro connectivity) whose geometry weights the integrals and gives h_e, h_m."""
    problem = problem if problem is not None else op.problem
    u = np.asarray(u, float)
    mesh = op.mesh
    geo = mesh if fiducial is None else fiducial
    if fiducial is not None:
        for k in ("elem_macro", "elem_level", "elem_anchor", "elem_p", "macro_nbr", "macro_nbr_face",
                  "macro_nbr_orient"):
            if not np.array_equal(np.asarray(mesh[k]), np.asarray(fiducial[k])):
                raise ValueError("the fiducial grid must have the same cells and connectivity")
    h_e = element_diameters(geo)
    p_e = mesh["elem_p"].astype(float)
    eta2_vol = np.zeros(op.E)
    for g in op.vgroups:
        n, q = g["n"], g["q"]
        B, Dt = g["B"], g["Dt"]
        elems = g["elems"]
        U = u[g["idx"]].reshape(-1, n, n, n)
        d0 = np.einsum("ck,bj,ai,ekji->ecba", B, B, Dt, U, optimize=True)
        d1 = np.einsum("ck,bj,ai,ekji->ecba", B, Dt, B, U, optimize=True)
        d2 = np.einsum("ck,bj,ai,ekji->ecba", Dt, B, B, U, optimize=True)
        grad = np.stack([d0, d1, d2], axis=-1).reshape(len(U), q ** 3, 3)
        W, det = g["W"], g["det"]
        wdet = W * det  # the integration weight: physical, or the fiducial grid's
        if fiducial is not None:
            _, Jf = geometry.element_map(geo, elems[:, None], g["xi"][None])
            wdet = W * np.linalg.det(Jf)
        # contravariant flux det J k (J^-1 J^-T grad_xi u)_d = (G grad_xi u)_d / W
        F = (np.einsum("epdc,epc->epd", g["G"], grad) / W[None, :, None]).reshape(len(U), q, q, q, 3)
        eta, _ = rules.gl(q)
        Dg = rules.lagrange_deriv(eta, eta)  # Dg[a, t] = l_t'(eta_a) on the GL points
        div = (np.einsum("at,ecbt->ecba", Dg, F[..., 0])
               + np.einsum("bt,ecta->ecba", Dg, F[..., 1])
               + np.einsum("ct,etba->ecba", Dg, F[..., 2])).reshape(len(U), -1) / det
        R = problems.source_g(problem, g["x"]) + div
        if g["M"] is not None:
            uq = np.einsum("ck,bj,ai,ekji->ecba", B, B, B, U, optimize=True).reshape(len(U), -1)
            R = R - (g["M"] / (W * det)) * uq
        eta2_vol[elems] = h_e[elems] ** 2 * p_e[elems] ** 2 * np.sum(wdet * R * R, axis=1)
    eta2 = eta2_vol.copy()
    eta2_face = np.zeros(len(op.mortars))
    eta2_flux = np.zeros(len(op.mortars))
    eta2_jump = np.zeros(len(op.mortars))
    for g in op.fgroups:
        if g["robin"]:
            continue
        wS, sig, hmin = g["wS"], g["sigma"], g["hmin"]
        if fiducial is not None:
            fm, fp = g["key"][3], g["key"][4]
            Sf, nrf = _face_metric(geo, g["em"], g["xim"], fm)
            hf = 2.0 / nrf
            if "ep" in g:
                _, nrp = _face_metric(geo, g["ep"], g["xip"], fp)
                hf = np.minimum(hf, 2.0 / nrp)
            wS = g["wst"][None, :] * Sf
            sig = sig * hmin / hf  # sigma = C p_m^2 max(k) / h_m with the fiducial h_m
            hmin = hf
        Um = u[g["idx_m"]]
        um = Um @ g["Vm"].T
        gm = np.einsum("mpd,dpa,ma->mp", g["mvec_m"], g["Dm"], Um)  # n-.grad u-
        if "ep" in g:
            Up = u[g["idx_p"]]
            up = Up @ g["Vp"].T
            gp = np.einsum("mpd,dpa,ma->mp", g["mvec_p"], g["Dp"], Up)  # n+.grad u+
            J1 = g["kx"] * gm + g["kp"] * gp
            J2 = um - up
            flux = np.sum(wS * hmin / g["pm"] * J1 * J1, axis=1)
            jump = np.sum(wS * sig * J2 * J2, axis=1)
            val = flux + jump
            np.add.at(eta2, g["em"], val)
            np.add.at(eta2, g["ep"], val)
            eta2_flux[g["mis"]] = flux
        else:
            J3 = um - problems.dirichlet_g(problem, g["x"])
            val = np.sum(wS * sig * J3 * J3, axis=1)
            jump = val
            np.add.at(eta2, g["em"], val)
        eta2_face[g["mis"]] = val
        eta2_jump[g["mis"]] = jump
    return dict(eta2=eta2, eta2_vol=eta2_vol, eta2_face=eta2_face, eta2_flux=eta2_flux, eta2_jump=eta2_jump)


def mark_fraction(eta2, fraction):
    """The ceil(fraction E) elements with the largest eta2 (ties: the lower index first); the
    product is taken with a guard of 1e-9 against its representation error (0.1 x 30 rounds
    above 3 in binary)."""
    eta2 = np.asarray(eta2, float)
    k = min(len(eta2), int(np.ceil(fraction * len(eta2) - 1e-9)))
    order = np.lexsort((np.arange(len(eta2)), -eta2))
    marked = np.zeros(len(eta2), bool)
    marked[order[:k]] = True
    return marked


def mark_mean(eta2, factor):
    """Elements whose eta2 exceeds factor times the mean."""
    eta2 = np.asarray(eta2, float)
    return eta2 > factor * eta2.mean()


def smooth_pred(eta2, eta2_pred, p, marked, gamma_h=0.25, gamma_p=0.1, dim=3):
    """Alg. hpamr on every element: action (0 keep, 1 h-refine, 2 p-refine) and the prediction
    the element (p-refine, keep) or each of its children (h-refine) carries to the next step;
    eta2_pred = inf means no prediction."""
    eta2 = np.asarray(eta2, float)
    pred = np.asarray(eta2_pred, float)
    p = np.asarray(p)
    action = np.zeros(len(eta2), np.int32)
    new_pred = pred.copy()
    for e in np.flatnonzero(marked):
        if eta2[e] > pred[e]:
            action[e] = 1
            new_pred[e] = gamma_h * 0.5 ** dim * 0.5 ** (2 * int(p[e])) * eta2[e]
        else:
            action[e] = 2
            new_pred[e] = gamma_p * eta2[e]
    return action, new_pred
