"""1-D rules: Legendre-Gauss-Lobatto collocation nodes, Gauss-Legendre quadrature, Lagrange polynomials.

Sec. II.A.3 (basis functions, Eq. Lagrange_Basis): N+1 LGL points per dimension,
Lagrange interpolating polynomials l_i.  Sec. II.A.5 (quadrature): integrals on GL
points, with polynomials interpolated from LGL to GL points.
"""
import numpy as np


def legendre(n, x):
    """P_n(x) and P_n'(x) by the three-term recurrence."""
    x = np.asarray(x, float)
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    # derivative: (1 - x^2) P_n' = n (P_{n-1} - x P_n); at |x| = 1 use n(n+1)/2 * x^(n+1)
    with np.errstate(divide="ignore", invalid="ignore"):
        dp = n * (p0 - x * p1) / (1.0 - x * x)
    end = np.isclose(np.abs(x), 1.0, rtol=0, atol=1e-15)
    dp = np.where(end, 0.5 * n * (n + 1) * np.sign(x) ** (n + 1), dp)
    return p1, dp


def gl(q):
    """q-point Gauss-Legendre nodes (ascending) and weights: roots of P_q, w = 2/((1-x^2) P_q'^2)."""
    x = -np.cos(np.pi * (np.arange(q) + 0.75) / (q + 0.5))
    for _ in range(100):
        p, dp = legendre(q, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    x = 0.5 * (x - x[::-1])  # exact symmetry
    if q % 2 == 1:
        x[q // 2] = 0.0
    _, dp = legendre(q, x)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    w = 0.5 * (w + w[::-1])
    return x, w


def lgl(n):
    """n-point (degree N = n-1) Legendre-Gauss-Lobatto nodes and weights.

    Nodes: -1, +1 and the roots of P_N'; weights 2 / (N (N+1) P_N(x)^2).
    """
    N = n - 1
    assert N >= 1
    x = -np.cos(np.pi * np.arange(n) / N)
    for _ in range(100):
        # Newton on (1 - x^2) P_N'(x) for the interior nodes: f = P_{N-1} - P_{N+1}
        pm, dpm = legendre(N - 1, x[1:-1])
        pp, dpp = legendre(N + 1, x[1:-1])
        f = pm - pp
        df = dpm - dpp
        dx = f / df
        x[1:-1] -= dx
        if dx.size == 0 or np.max(np.abs(dx)) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    x = 0.5 * (x - x[::-1])
    if n % 2 == 1:
        x[n // 2] = 0.0
    p, _ = legendre(N, x)
    w = 2.0 / (N * (N + 1) * p * p)
    w = 0.5 * (w + w[::-1])
    return x, w


def lagrange(nodes, x):
    """L[a, i] = l_i(x_a) by the product definition of the Lagrange polynomials."""
    nodes = np.asarray(nodes, float)
    x = np.atleast_1d(np.asarray(x, float))
    n = len(nodes)
    L = np.ones((len(x), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                L[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return L


def lagrange_deriv(nodes, x):
    """D[a, i] = l_i'(x_a): product rule applied to the product definition."""
    nodes = np.asarray(nodes, float)
    x = np.atleast_1d(np.asarray(x, float))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for j in range(n):
                if j != i and j != m:
                    term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            D[:, i] += term
    return D
