"""Pins for the oracle's simplex quadrature (Sec. 4.1: one n-simplex rule
mapped to all faces) against the closed-form Dirichlet integral
    int_{reference n-simplex} xi^alpha = prod(alpha_i!) / (|alpha| + n)!"""
import itertools
import math

import numpy as np
import pytest

from oracle.quadrature import gauss_jacobi01, simplex_rule


def dirichlet_integral(alpha):
    num = 1
    for a in alpha:
        num *= math.factorial(a)
    return num / math.factorial(sum(alpha) + len(alpha))


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("q", [1, 2, 3, 4, 6, 8])
def test_simplex_rule_exact_to_degree_2q_minus_1(n, q):
    lam, w = simplex_rule(n, q)
    assert lam.shape == (q ** n, n + 1)
    assert np.all(w > 0)
    assert np.all(lam > 0) and np.allclose(lam.sum(1), 1.0, atol=1e-15)
    xi = lam[:, 1:]
    for deg in range(0, 2 * q):
        for alpha in itertools.product(range(deg + 1), repeat=n):
            if sum(alpha) != deg:
                continue
            val = (w * np.prod(xi ** np.array(alpha), axis=1)).sum()
            assert abs(val - dirichlet_integral(alpha)) <= 2e-15 * max(1.0, dirichlet_integral(alpha)) * q ** n


@pytest.mark.parametrize("a", [0, 1, 2])
def test_gauss_jacobi_moments(a):
    # int_0^1 (1-s)^a s^k ds = a! k! / (a+k+1)!  (Beta function)
    q = 6
    s, w = gauss_jacobi01(q, a)
    for k in range(2 * q):
        exact = math.factorial(a) * math.factorial(k) / math.factorial(a + k + 1)
        assert abs((w * s ** k).sum() - exact) < 1e-15


def test_not_exact_beyond_degree():
    # a q-point Gauss rule cannot integrate degree 2q exactly (sanity of the pin)
    lam, w = simplex_rule(1, 3)
    xi = lam[:, 1]
    assert abs((w * xi ** 6).sum() - dirichlet_integral((6,))) > 1e-8
