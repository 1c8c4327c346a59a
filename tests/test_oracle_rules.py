"""Pins for the oracle's 1-D rules (Sec. II.A.3 basis, Sec. II.A.5 quadrature)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import rules

GOLD = os.path.join(os.path.dirname(__file__), "golden", "quadrature_closed_forms.json")


def _ev(s):
    return eval(s, {"sqrt": math.sqrt})  # closed-form strings of the fixture


def test_closed_forms():
    gold = json.load(open(GOLD))
    for n, v in gold["lgl"].items():
        x, w = rules.lgl(int(n))
        np.testing.assert_allclose(x, [_ev(s) for s in v["nodes"]], atol=1e-15)
        np.testing.assert_allclose(w, [_ev(s) for s in v["weights"]], atol=1e-15)
    for q, v in gold["gl"].items():
        x, w = rules.gl(int(q))
        np.testing.assert_allclose(x, [_ev(s) for s in v["nodes"]], atol=1e-15)
        np.testing.assert_allclose(w, [_ev(s) for s in v["weights"]], atol=1e-15)


@pytest.mark.parametrize("n", range(2, 21))
def test_lgl_exactness_and_symmetry(n):
    # n-point LGL integrates monomials of degree <= 2n - 3 exactly; sum of weights is 2
    x, w = rules.lgl(n)
    assert abs(w.sum() - 2.0) < 1e-14
    np.testing.assert_allclose(x, -x[::-1], atol=0)
    np.testing.assert_allclose(w, w[::-1], atol=0)
    for k in range(2 * n - 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 5e-14
    # and not degree 2n - 2 (the rule is exactly that strong)
    k = 2 * n - 2
    if n <= 10:
        assert abs(np.dot(w, x ** k) - 2.0 / (k + 1)) > 1e-12


@pytest.mark.parametrize("q", range(1, 22))
def test_gl_exactness(q):
    x, w = rules.gl(q)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * q):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 5e-14
    k = 2 * q
    if q <= 10:
        assert abs(np.dot(w, x ** k) - 2.0 / (k + 1)) > 1e-12


@pytest.mark.parametrize("n", [2, 3, 5, 8, 12])
def test_lagrange_exact_on_polynomials(n):
    nodes, _ = rules.lgl(n)
    x = np.linspace(-1, 1, 17)
    L = rules.lagrange(nodes, x)
    D = rules.lagrange_deriv(nodes, x)
    np.testing.assert_allclose(rules.lagrange(nodes, nodes), np.eye(n), atol=1e-14)
    for k in range(n):  # degree <= n - 1 reproduced exactly, with its derivative
        np.testing.assert_allclose(L @ nodes ** k, x ** k, atol=1e-12)
        dk = k * x ** (k - 1) if k > 0 else 0 * x
        np.testing.assert_allclose(D @ nodes ** k, dk, atol=1e-10 * max(1, k * k))
    # a degree-n polynomial is not reproduced
    assert np.max(np.abs(L @ nodes ** n - x ** n)) > 1e-6


def test_legendre_derivative_matches_finite_difference():
    for n in (3, 7, 11):
        x = np.linspace(-0.9, 0.9, 9)
        h = 1e-6
        p_plus, _ = rules.legendre(n, x + h)
        p_minus, _ = rules.legendre(n, x - h)
        _, dp = rules.legendre(n, x)
        np.testing.assert_allclose(dp, (p_plus - p_minus) / (2 * h), rtol=1e-7, atol=1e-7)
