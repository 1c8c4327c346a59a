"""Manufactured solutions, sources and coefficients for the descriptors named by ``meshgen``.

Model problem (reading of Sec. II.A.2, Eq. Laplacian, with the sign of the bilinear
form Eq. lh): -div(k grad u) + c u = g in the domain, u = g_D on Dirichlet faces.
Each source g is derived from u by hand (the derivations are in the docstrings),
never copied from a printed right-hand side.
"""
import numpy as np


def k_of(problem, x):
    """Diffusion coefficient at points x [..., 3]."""
    if problem is not None and problem["kind"] == "radial_step":
        r0, k_in, k_out = problem["params"][:3]
        r = np.linalg.norm(x, axis=-1)
        return np.where(r < r0, k_in, k_out)
    return np.ones(x.shape[:-1])


def k_is_constant(problem):
    return problem is None or problem["kind"] != "radial_step"


def exact_u(problem, x):
    kind = problem["kind"]
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    if kind == "sinsinsin":
        return np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
    if kind == "shell_harmonic":
        c = problem["params"][0]
        r = np.linalg.norm(x, axis=-1)
        return 1.0 / r + c * X * Z / r ** 5
    if kind == "radial_step":
        r0, k_in, k_out = problem["params"][:3]
        r2 = np.sum(x * x, axis=-1)
        inside = np.sqrt(r2) < r0
        c_in = r0 * r0 * (1.0 / k_out - 1.0 / k_in)
        return np.where(inside, r2 / k_in + c_in, r2 / k_out)
    if kind == "polynomial":
        C = _poly_coeffs(problem)
        P = C.shape[0]
        u = np.zeros(x.shape[:-1])
        for a in range(P):
            for b in range(P):
                for c in range(P):
                    u += C[a, b, c] * X ** a * Y ** b * Z ** c
        return u
    if kind == "gaussians":
        return np.zeros(x.shape[:-1])  # only used as Dirichlet data (g_D = 0)
    if kind == "polynomial_dirichlet":
        return exact_u(dict(kind="polynomial", params=problem["params"]), x)
    if kind == "star":
        rho0, r0 = problem["params"][:2]
        return star_psi(rho0, r0, np.linalg.norm(x, axis=-1))
    if kind == "layered_x":
        # k = k1 for x < x0, k2 beyond: u = x / k1, then x0 / k1 + (x - x0) / k2 (continuous,
        # flux k du/dx = 1 on both sides, so -div(k grad u) = 0)
        x0, k1, k2 = problem["params"][:3]
        return np.where(X < x0, X / k1, x0 / k1 + (X - x0) / k2)
    raise ValueError(kind)


def star_parameters(rho0, r0):
    """Constant-density star (Sec. III.B): C = (2 pi rho0 / 3)^(-1/4), beta = r0 (C u_alpha(r0) - 1),
    and alpha from the continuity of psi and dpsi/dr at r0, which gives
    rho0 r0^2 = (3 / (2 pi)) alpha^10 / (1 + alpha^2)^6 (the printed exponent 3 does not make
    dpsi/dr continuous).  The right side rises to its maximum at alpha^2 = 5 and then falls;
    the root taken is the one on the falling branch, alpha >= sqrt(5), where psi -> 1 as
    rho0 -> 0 (the weak-field star), found by bisection."""
    C = (2.0 * np.pi * rho0 / 3.0) ** -0.25
    target = rho0 * r0 * r0

    def f(a):
        return 3.0 / (2.0 * np.pi) * a ** 10 / (1.0 + a * a) ** 6 - target

    lo = np.sqrt(5.0)
    if f(lo) < 0:
        raise ValueError("rho0 r0^2 above the largest value a static star allows")
    hi = 2.0 * lo
    while f(hi) > 0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) > 0 else (lo, mid)
    alpha = 0.5 * (lo + hi)
    u_r0 = np.sqrt(alpha * r0) / np.sqrt(r0 * r0 + (alpha * r0) ** 2)
    return C, alpha, r0 * (C * u_r0 - 1.0)


def star_psi(rho0, r0, r):
    """psi(r) of the constant-density star: C u_alpha(r) inside r0, beta / r + 1 outside."""
    C, alpha, beta = star_parameters(rho0, r0)
    r = np.asarray(r, float)
    inside = C * np.sqrt(alpha * r0) / np.sqrt(r * r + (alpha * r0) ** 2)
    with np.errstate(divide="ignore"):
        outside = beta / r + 1.0
    return np.where(r <= r0, inside, outside)


def source_g(problem, x):
    """g = -div(k grad u) for the manufactured u (or the given source)."""
    kind = problem["kind"]
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    if kind == "sinsinsin":
        # -lap sin sin sin = 3 pi^2 sin sin sin
        return 3.0 * np.pi ** 2 * exact_u(problem, x)
    if kind == "shell_harmonic":
        # 1/r and x z / r^5 (Kelvin transform of the harmonic x z) are harmonic away from 0
        return np.zeros(x.shape[:-1])
    if kind == "radial_step":
        # k grad u = 2 x on both sides of r0, so -div(k grad u) = -6
        return np.full(x.shape[:-1], -6.0)
    if kind == "polynomial":
        C = _poly_coeffs(problem)
        P = C.shape[0]
        g = np.zeros(x.shape[:-1])
        for a in range(P):
            for b in range(P):
                for c in range(P):
                    if a >= 2:
                        g -= C[a, b, c] * a * (a - 1) * X ** (a - 2) * Y ** b * Z ** c
                    if b >= 2:
                        g -= C[a, b, c] * b * (b - 1) * X ** a * Y ** (b - 2) * Z ** c
                    if c >= 2:
                        g -= C[a, b, c] * c * (c - 1) * X ** a * Y ** b * Z ** (c - 2)
        return g
    if kind == "star":
        # the density term is the nonlinear source of the Newton solve; no linear source
        return np.zeros(x.shape[:-1])
    if kind == "gaussians":
        rows = np.asarray(problem["params"]).reshape(-1, 5)
        g = np.zeros(x.shape[:-1])
        for a, cx, cy, cz, s in rows:
            d2 = (X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2
            g += a * np.exp(-d2 / (2.0 * s * s))
        return g
    if kind == "polynomial_dirichlet":
        return np.zeros(x.shape[:-1])  # Dirichlet data only
    if kind == "layered_x":
        return np.zeros(x.shape[:-1])  # k du/dx = 1 on both sides of x0
    raise ValueError(kind)


def dirichlet_g(problem, x):
    return exact_u(problem, x)


def grad_u(problem, x):
    """grad u of the manufactured u, for the kinds that carry Neumann data."""
    kind = problem["kind"]
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    if kind == "sinsinsin":
        sx, sy, sz = np.sin(np.pi * X), np.sin(np.pi * Y), np.sin(np.pi * Z)
        cx, cy, cz = np.cos(np.pi * X), np.cos(np.pi * Y), np.cos(np.pi * Z)
        return np.pi * np.stack([cx * sy * sz, sx * cy * sz, sx * sy * cz], axis=-1)
    if kind in ("polynomial", "polynomial_dirichlet"):
        C = _poly_coeffs(problem)
        P = C.shape[0]
        gx, gy, gz = (np.zeros(x.shape[:-1]) for _ in range(3))
        for a in range(P):
            for b in range(P):
                for c in range(P):
                    if a >= 1:
                        gx += C[a, b, c] * a * X ** (a - 1) * Y ** b * Z ** c
                    if b >= 1:
                        gy += C[a, b, c] * b * X ** a * Y ** (b - 1) * Z ** c
                    if c >= 1:
                        gz += C[a, b, c] * c * X ** a * Y ** b * Z ** (c - 1)
        return np.stack([gx, gy, gz], axis=-1)
    raise ValueError("no Neumann data for problem kind %s" % kind)


def robin_u(problem, x):
    """u on a Robin face for the Robin data g_R = k n.grad u + gamma u (0 for the Gaussian
    sources, which carry homogeneous boundary data)."""
    if problem["kind"] == "gaussians":
        return np.zeros(x.shape[:-1])
    return exact_u(problem, x)


def neumann_g(problem, x, nhat, kx):
    """Neumann data (Eq. NeumannBC, as the flux k n.grad u of the form -div(k grad u) = g):
    g_N = k grad u . n with n the outward unit normal; 0 for "gaussians" (a source with
    homogeneous boundary data)."""
    if problem["kind"] == "gaussians":
        return np.zeros(x.shape[:-1])
    return kx * np.einsum("...d,...d->...", grad_u(problem, x), nhat)


def _poly_coeffs(problem):
    C = np.asarray(problem["params"], float)
    P = int(round(len(C) ** (1.0 / 3.0)))
    return C.reshape(P, P, P)


def nl_alpha_beta(nl, x):
    """alpha(x), beta(x) of the nonlinear source  -lap u = beta (1 + alpha u)^-7.

    ``puncture``: alpha = 1 / (1 + sum_I m_I / (2 r_I)), r_I = |x - c_I| (the puncture sum
    of Sec. III.D written as psi = (1 + alpha u) / alpha), and a smooth decaying
    beta = sum_I a_I exp(-r_I^2 / (2 s^2)) / (1 + |x|^2)^2; params = [s, rows (c, m, a)].
    ``nl_quadratic``: alpha constant, beta = (-lap u*) (1 + alpha u*)^7 for the quadratic
    u* of params[1:] (so that u* is an exact solution); params = [alpha, C (27)].
    """
    kind = nl["kind"]
    P = np.asarray(nl["params"], float)
    if kind == "puncture":
        s = P[0]
        rows = P[1:].reshape(-1, 5)
        psum = np.zeros(x.shape[:-1])
        beta = np.zeros(x.shape[:-1])
        for cx, cy, cz, m, a in rows:
            r2 = (x[..., 0] - cx) ** 2 + (x[..., 1] - cy) ** 2 + (x[..., 2] - cz) ** 2
            psum += m / (2.0 * np.sqrt(r2))
            beta += a * np.exp(-r2 / (2.0 * s * s))
        beta /= (1.0 + np.sum(x * x, axis=-1)) ** 2
        return 1.0 / (1.0 + psum), beta
    if kind == "nl_quadratic":
        alpha = P[0]
        poly = dict(kind="polynomial", params=P[1:])
        u = exact_u(poly, x)
        return np.full(x.shape[:-1], alpha), source_g(poly, x) * (1.0 + alpha * u) ** 7
    if kind == "star":
        # -lap psi = 2 pi rho psi^5 (Sec. III.B): alpha is unused, beta = 2 pi rho(x)
        rho0, r0 = P[:2]
        r = np.linalg.norm(x, axis=-1)
        return np.zeros(x.shape[:-1]), np.where(r <= r0, 2.0 * np.pi * rho0, 0.0)
    raise ValueError(kind)


def nl_terms(nl, alpha, beta, u):
    """Integrand factor of N(u) and the Jacobian's mass coefficient -dN/du at GL points:
    puncture-type sources beta (1 + alpha u)^-7 and 7 alpha beta (1 + alpha u)^-8; the star
    beta u^5 and -5 beta u^4."""
    if nl["kind"] == "star":
        return beta * u ** 5, -5.0 * beta * u ** 4
    s = 1.0 + alpha * u
    if np.any(s <= 0.0):
        raise FloatingPointError("1 + alpha u <= 0 at a quadrature point")
    return beta * s ** -7, 7.0 * alpha * beta * s ** -8
