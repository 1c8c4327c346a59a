"""Macro-element maps, induced element maps and their Jacobians (FP64).

Sec. II.A.1 (Eq. Phi_e): each macro-element is the image of [-1,1]^3 under Phi_e0;
a fine element's reference coordinates are linearly related to its macro's.
Sec. II.A.5 (Eqs. Jacobian, Surface-Jacobian): (J)^i_j = dx_i/dxi_j, J = det J,
S^m = J |dxi_j/dx|, n = sgn(xi_j) (J/S^m) dxi_j/dx.
Sec. III.C (Eq. inverse_mapping): inverse radial map r = m/(x - t).

Every map here is written analytically with its chain-rule Jacobian.
"""
import numpy as np

AFFINE, SHELL, CUBE_SPHERE = 0, 1, 2


def inverse_radial(z, x1, x2, r1, r2):
    """Inverse radial map of Eq. inverse_mapping: r(x1) = r1, r(x2) = r2, 1/r linear in z.

    r = m / (z - t) with m = (x2 - x1)/(1/r2 - 1/r1), t = (x1 r1 - x2 r2)/(r1 - r2) is
    evaluated in the algebraically identical form 1/r = [(x2 - z)/r1 + (z - x1)/r2]/(x2 - x1),
    which avoids the cancellation in z - t near z = x2 when r2 >> r1.  Returns r, dr/dz.
    """
    inv = ((x2 - z) / r1 + (z - x1) / r2) / (x2 - x1)
    r = 1.0 / inv
    return r, -r * r * (1.0 / r2 - 1.0 / r1) / (x2 - x1)


def radial(z, zc, par):
    """Radial coordinate of a SHELL macro at reference coordinate z.

    A piecewise map takes the branch of the point itself; only exactly at the break
    does ``zc`` (the element's cell centre) decide, so that the two elements meeting there
    each use their own smooth branch while a coarse cell spanning the break follows the
    true map at every quadrature point.
    """
    kind = par[..., 9]
    r_in, r_out, zb, rb = par[..., 10], par[..., 11], par[..., 12], par[..., 13]
    r = np.empty_like(z)
    dr = np.empty_like(z)
    lin = kind == 0
    r[lin] = (r_in + 0.5 * (z + 1.0) * (r_out - r_in))[lin]
    dr[lin] = (0.5 * (r_out - r_in) * np.ones_like(z))[lin]
    inv = kind == 1
    ri, dri = inverse_radial(z, -1.0, 1.0, r_in, r_out)
    r[inv], dr[inv] = ri[inv], dri[inv]
    pw = kind == 2
    low = pw & ((z < zb) | ((z == zb) & (zc <= zb)))
    rl = r_in + (z + 1.0) / (zb + 1.0) * (rb - r_in)
    drl = (rb - r_in) / (zb + 1.0) * np.ones_like(z)
    r[low], dr[low] = rl[low], drl[low]
    high = pw & ~low
    rh, drh = inverse_radial(z, zb, 1.0, rb, r_out)
    r[high], dr[high] = rh[high], drh[high]
    return r, dr


def macro_map(kind, par, xi, zc=None):
    """x(xi) and J = dx/dxi for macro maps; arrays broadcast over leading axes.

    kind: int[...], par: [..., 16], xi: [..., 3]; returns x [..., 3], J [..., 3, 3].
    """
    xi = np.asarray(xi, float)
    shape = xi.shape[:-1]
    kind = np.broadcast_to(kind, shape)
    par = np.broadcast_to(par, shape + (16,))
    if zc is None:
        zc = xi[..., 2]
    zc = np.broadcast_to(zc, shape)
    x = np.zeros(shape + (3,))
    J = np.zeros(shape + (3, 3))

    aff = kind == AFFINE
    if np.any(aff):
        p = par[aff]
        o = p[:, 0:3]
        A = np.stack([p[:, 3:6], p[:, 6:9], p[:, 9:12]], axis=-1)  # columns a0, a1, a2
        xa = o + np.einsum("pij,pj->pi", A, 0.5 * (xi[aff] + 1.0))
        x[aff] = xa
        J[aff] = 0.5 * A

    sh = (kind == SHELL) | (kind == CUBE_SPHERE)
    if np.any(sh):
        p = par[sh]
        R = p[:, 0:9].reshape(-1, 3, 3)
        e = xi[sh]
        X = np.tan(0.25 * np.pi * e[:, 0])
        Y = np.tan(0.25 * np.pi * e[:, 1])
        dX = 0.25 * np.pi * (1.0 + X * X)
        dY = 0.25 * np.pi * (1.0 + Y * Y)
        c = np.stack([X, Y, np.ones_like(X)], axis=-1)
        v = np.einsum("pij,pj->pi", R, c)
        nv = np.sqrt(X * X + Y * Y + 1.0)
        u = v / nv[:, None]
        # derivatives of the unit direction u = v/|v| with respect to X and Y
        du_dX = R[:, :, 0] / nv[:, None] - v * (X / nv ** 3)[:, None]
        du_dY = R[:, :, 1] / nv[:, None] - v * (Y / nv ** 3)[:, None]
        kk = kind[sh]
        xs = np.zeros_like(u)
        Js = np.zeros(u.shape + (3,))
        shell = kk == SHELL
        if np.any(shell):
            r, dr = radial(e[shell, 2], zc[sh][shell], p[shell])
            xs[shell] = r[:, None] * u[shell]
            Js[shell, :, 0] = (r * dX[shell])[:, None] * du_dX[shell]
            Js[shell, :, 1] = (r * dY[shell])[:, None] * du_dY[shell]
            Js[shell, :, 2] = dr[:, None] * u[shell]
        cs = kk == CUBE_SPHERE
        if np.any(cs):
            # blend (linear in xi2) between the flat cube-face point a R (xi0, xi1, 1),
            # parametrised linearly like the affine central cube, and the sphere point
            # r_s u along the equiangular direction (matching the shell wedges outside)
            a = p[cs, 10]
            rs = p[cs, 11]
            z = e[cs, 2]
            s = 0.5 * (z + 1.0)
            Rc = R[cs]
            lin = np.stack([e[cs, 0], e[cs, 1], np.ones_like(z)], axis=-1)
            fl = a[:, None] * np.einsum("pij,pj->pi", Rc, lin)
            sp = rs[:, None] * u[cs]
            xs[cs] = (1.0 - s)[:, None] * fl + s[:, None] * sp
            Js[cs, :, 0] = ((1.0 - s) * a)[:, None] * Rc[:, :, 0] + (s * rs * dX[cs])[:, None] * du_dX[cs]
            Js[cs, :, 1] = ((1.0 - s) * a)[:, None] * Rc[:, :, 1] + (s * rs * dY[cs])[:, None] * du_dY[cs]
            Js[cs, :, 2] = 0.5 * (sp - fl)
        x[sh] = xs
        J[sh] = Js
    return x, J


def element_map(mesh, elem, xi):
    """x(xi), J(xi) of fine elements ``elem`` (int[...]) at element reference points xi [..., 3].

    The element cell of (level l, anchor a) maps xi_e to the macro coordinate
    xi = -1 + (2 a + 1 + xi_e) / 2^l, so J_e = J_macro / 2^l.
    """
    elem = np.asarray(elem)
    xi = np.asarray(xi, float)
    lev = mesh["elem_level"][elem]
    anc = mesh["elem_anchor"][elem].astype(float)
    m = mesh["elem_macro"][elem]
    scale = 1.0 / (2.0 ** lev)
    ximac = -1.0 + (2.0 * anc + 1.0 + xi) * scale[..., None]
    zc = -1.0 + (2.0 * anc[..., 2] + 1.0) * scale
    x, J = macro_map(mesh["macro_kind"][m], mesh["macro_params"][m], ximac, zc)
    return x, J * scale[..., None, None]


def cell_map(mesh_macro_kind, mesh_macro_params, macro, level, anchor, xi):
    """Same as element_map for explicit (macro, level, anchor) cells (coarse MG levels)."""
    level = np.asarray(level)
    anc = np.asarray(anchor, float)
    scale = 1.0 / (2.0 ** level)
    ximac = -1.0 + (2.0 * anc + 1.0 + xi) * scale[..., None]
    zc = -1.0 + (2.0 * anc[..., 2] + 1.0) * scale
    x, J = macro_map(mesh_macro_kind[macro], mesh_macro_params[macro], ximac, zc)
    return x, J * scale[..., None, None]


def is_affine_macro(kind):
    return np.asarray(kind) == AFFINE
