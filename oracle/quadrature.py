"""Quadrature on n-simplices for the oracle (test infrastructure only).

The method only integrates over n-dimensional simplices: the spatial elements
(mapped to the space-like bottom and top facets of a tent) and the vertical
time-like faces (Sec. 2.4, closing remark; Sec. 4.1, Fig. 2).  One rule on the
reference n-simplex is generated once and mapped everywhere.

Rule: collapsed-coordinate (conical product) Gauss rule.  With q points per
direction it integrates every polynomial of total degree <= 2q - 1 exactly.
  xi_n     = s_n,                      weight (1 - s_n)^(n-1)  (Gauss-Jacobi)
  xi_{n-1} = s_{n-1} (1 - s_n),        weight (1 - s_{n-1})^(n-2)
  ...
  xi_1     = s_1 (1 - s_2) ... (1 - s_n)                        (Gauss-Legendre)
Point order: s_n slowest, s_1 fastest; 1D nodes ascending.  Barycentric
coordinates: lambda_0 = 1 - sum(xi), lambda_k = xi_k.  Weights sum to 1/n!.

The 1D Gauss rules come from the Golub-Welsch eigenvalue method applied to the
three-term recurrence of the Jacobi polynomials P^(a,0).
"""
from __future__ import annotations

import math

import numpy as np


def gauss_jacobi(q: int, a: float):
    """Nodes/weights on [-1, 1] for the weight (1 - x)^a (b = 0)."""
    b = 0.0
    alpha = np.empty(q)
    for i in range(q):
        s = 2 * i + a + b
        if i == 0:
            alpha[i] = (b - a) / (a + b + 2.0)
        else:
            alpha[i] = (b * b - a * a) / (s * (s + 2.0))
    beta = np.empty(max(q - 1, 0))
    for i in range(1, q):
        s = 2 * i + a + b
        beta[i - 1] = 4.0 * i * (i + a) * (i + b) * (i + a + b) / (s * s * (s + 1.0) * (s - 1.0))
    J = np.diag(alpha) + np.diag(np.sqrt(beta), 1) + np.diag(np.sqrt(beta), -1)
    nodes, vecs = np.linalg.eigh(J)
    mu0 = 2.0 ** (a + b + 1.0) * math.gamma(a + 1.0) * math.gamma(b + 1.0) / math.gamma(a + b + 2.0)
    w = mu0 * vecs[0, :] ** 2
    return nodes, w


def gauss_jacobi01(q: int, a: int):
    """Nodes/weights on [0, 1] for the weight (1 - s)^a."""
    x, w = gauss_jacobi(q, float(a))
    return 0.5 * (x + 1.0), w * 2.0 ** (-a - 1.0)


def simplex_rule(n: int, q: int):
    """Collapsed Gauss rule on the reference n-simplex.

    Returns (lam, w): lam (Q, n+1) barycentric coordinates, w (Q,) weights
    summing to 1/n!, with Q = q^n."""
    if n == 0:
        return np.ones((1, 1)), np.ones(1)
    rules = [gauss_jacobi01(q, d - 1) for d in range(1, n + 1)]  # rules[d-1] for s_d
    pts = []
    wts = []
    # s_n slowest ... s_1 fastest
    for idx in np.ndindex(*([q] * n)):
        # idx[0] is the index of s_n, idx[n-1] the index of s_1
        s = {}
        wt = 1.0
        for pos, i in enumerate(idx):
            d = n - pos
            s[d] = rules[d - 1][0][i]
            wt *= rules[d - 1][1][i]
        xi = np.empty(n)
        scale = 1.0
        for d in range(n, 0, -1):
            xi[d - 1] = s[d] * scale
            scale *= (1.0 - s[d])
        pts.append(xi)
        wts.append(wt)
    xi = np.array(pts)
    lam = np.concatenate([1.0 - xi.sum(axis=1, keepdims=True), xi], axis=1)
    return lam, np.array(wts)

