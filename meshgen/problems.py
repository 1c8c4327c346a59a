"""Problem descriptors (ids + parameters) and seeded vectors.

A problem is the model equation  -div(k grad u) + c u = g  with Dirichlet data u = g_D
(the sign convention under which the paper's bilinear form is positive).  The
descriptor names the manufactured solution (or source) and the coefficient; each
consumer evaluates u, g, k itself:

* ``sinsinsin``  u = sin(pi x) sin(pi y) sin(pi z), k = 1, g = 3 pi^2 u.
* ``shell_harmonic``  u = 1/r + c x z / r^5 (harmonic), k = 1, g = 0; params = [c].
* ``radial_step``  k = k_in for |x| < r0 else k_out; u = |x|^2 / k + c_k with
  c_in = r0^2 (1/k_out - 1/k_in), c_out = 0 (continuous, flux-continuous); g = -6;
  params = [r0, k_in, k_out].
* ``polynomial``  u = sum_{a,b,c} C[a,b,c] x^a y^b z^c, k = 1, g = -lap u;
  params = C flattened with shape [P+1]^3 (P = params_shape[0] - 1).
* ``gaussians``  g = sum_i a_i exp(-|x - c_i|^2 / (2 s_i^2)), g_D = 0, k = 1, no exact u;
  params = rows (a, cx, cy, cz, s).
"""
import numpy as np

PROBLEM_IDS = {"sinsinsin": 0, "shell_harmonic": 1, "radial_step": 2, "polynomial": 3,
               "gaussians": 4}


def problem_config1():
    return dict(kind="sinsinsin", params=np.zeros(0))


def problem_config2(c=1.0):
    return dict(kind="shell_harmonic", params=np.array([c], float))


def problem_config3(r0=0.5, k_in=1.0, k_out=5.0):
    return dict(kind="radial_step", params=np.array([r0, k_in, k_out], float))


def polynomial_problem(degree, seed=0, total=False):
    """Random polynomial with per-axis degree <= degree (``total``: total degree <= degree)."""
    rng = np.random.default_rng(seed)
    C = rng.uniform(-1, 1, size=(degree + 1,) * 3)
    if total:
        a, b, c = np.meshgrid(*(np.arange(degree + 1),) * 3, indexing="ij")
        C[a + b + c > degree] = 0.0
    return dict(kind="polynomial", params=C.reshape(-1), shape=C.shape)


def gaussian_problem(n=8, lo=(-1, -1, -1), hi=(1, 1, 1), seed=0):
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    diam = float(np.linalg.norm(hi - lo))
    rows = []
    for _ in range(n):
        a = rng.uniform(-1, 1)
        c = rng.uniform(lo, hi)
        s = rng.uniform(0.05, 0.2) * diam
        rows.append([a, c[0], c[1], c[2], s])
    return dict(kind="gaussians", params=np.array(rows, float).reshape(-1))


def polynomial_dirichlet_problem(C):
    """Dirichlet data u = sum C[a,b,c] x^a y^b z^c with no volume source (g = 0)."""
    C = np.asarray(C, float)
    return dict(kind="polynomial_dirichlet", params=C.reshape(-1), shape=C.shape)


def puncture_problem(n_punctures=3, seed=0, r_ball=8.0, m_range=(0.3, 1.0), p_max=0.2, s=2.0):
    """Nonlinear source of the puncture-type problem  -lap u = beta (1 + alpha u)^-7.

    Seeded punctures: centres c_I uniform in the ball |x| < r_ball, masses m_I uniform in
    ``m_range``, momenta P_I with uniform direction and |P_I| uniform in [0, p_max].  Then
    alpha = 1 / (1 + sum_I m_I / (2 |x - c_I|)) and
    beta = sum_I |P_I|^2 exp(-|x - c_I|^2 / (2 s^2)) / (1 + |x|^2)^2 (a smooth decaying
    field standing in for the extrinsic-curvature term).
    params = [s, then rows (cx, cy, cz, m, a = |P|^2)].
    """
    rng = np.random.default_rng(seed)
    rows = []
    while len(rows) < n_punctures:
        c = rng.uniform(-r_ball, r_ball, 3)
        if np.linalg.norm(c) >= r_ball:
            continue
        m = rng.uniform(*m_range)
        d = rng.standard_normal(3)
        P = d / np.linalg.norm(d) * rng.uniform(0.0, p_max)
        rows.append([c[0], c[1], c[2], m, float(P @ P)])
    return dict(kind="puncture", params=np.concatenate([[s], np.array(rows).reshape(-1)]))


def quadratic_nonlinear_problem(alpha=0.5, seed=0):
    """Manufactured nonlinear problem with a quadratic exact solution.

    u* = 0.5 - 0.3 |x|^2 + (seeded linear terms, |b_i| <= 0.05); alpha constant; the source
    is chosen so that u* solves -lap u = beta (1 + alpha u)^-7, i.e.
    beta = (-lap u*) (1 + alpha u*)^7 with -lap u* = 1.8.
    params = [alpha, then the 27 coefficients C[a, b, c] of x^a y^b z^c (a, b, c <= 2)].
    Use with Dirichlet data u* (``polynomial_dirichlet_problem(C)``).
    """
    rng = np.random.default_rng(seed)
    C = np.zeros((3, 3, 3))
    C[0, 0, 0] = 0.5
    C[2, 0, 0] = C[0, 2, 0] = C[0, 0, 2] = -0.3
    b = rng.uniform(-0.05, 0.05, 3)
    C[1, 0, 0], C[0, 1, 0], C[0, 0, 1] = b
    return dict(kind="nl_quadratic", params=np.concatenate([[alpha], C.reshape(-1)])), C


def star_problem(rho0=0.001, r0=1.0):
    """Constant-density star (Sec. III.B): -lap psi = 2 pi rho psi^5 with rho = rho0 inside
    r <= r0 and 0 outside; Dirichlet data from the closed-form psi.  Returns the nonlinear
    source and the Dirichlet-data descriptors (both kind "star", params [rho0, r0])."""
    p = np.array([rho0, r0], float)
    return dict(kind="star", params=p.copy()), dict(kind="star", params=p.copy())


def dof_count(mesh):
    return int(np.sum((mesh["elem_p"].astype(np.int64) + 1) ** 3))


def random_vector(mesh, seed=0, dist="normal"):
    rng = np.random.default_rng(seed)
    n = dof_count(mesh)
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, n)
    return rng.standard_normal(n)
