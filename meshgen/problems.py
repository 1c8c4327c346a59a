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


def dof_count(mesh):
    return int(np.sum((mesh["elem_p"].astype(np.int64) + 1) ** 3))


def random_vector(mesh, seed=0, dist="normal"):
    rng = np.random.default_rng(seed)
    n = dof_count(mesh)
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, n)
    return rng.standard_normal(n)
