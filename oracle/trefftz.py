"""Exact-rational polynomial Trefftz basis of U^p (oracle; test infrastructure).

Follows Sec. 3 of the paper.  A space-time polynomial
    U(x, t) = sum_{|alpha| + k <= p} a_{k,alpha} x^alpha t^k
solves -Lap U + U_tt = 0 (wave speed 1) exactly when, for k >= 2,
    a_{k,alpha} = 1/(k(k-1)) sum_m (alpha_m + 1)(alpha_m + 2) a_{k-2, alpha + 2 e_m}
(eq. 3.1 with c = 1; Remark 3.1 maps to any c by a change of variables).
The recursion is seeded by a spatial basis for k = 0 and one for k = 1: a basis
function either has U(.,0) = x^beta, U_t(.,0) = 0 with |beta| <= p ("type 0"),
or U(.,0) = 0, U_t(.,0) = x^beta with |beta| <= p - 1 ("type 1").  Sec. 3
allows any polynomial basis of the spatial variables as seeds and Sec. 6.3
compares three: monomials x^beta (the default, found the best conditioned),
and the tensor products prod_m P_(beta_m)(x_m) of Legendre or
prod_m T_(beta_m)(x_m) of Chebyshev polynomials of the first kind, in the
scaled coordinates of Remark 3.1.  The seed of multi-index beta replaces x^beta
in the k = 0 (type 0) or k = 1 (type 1) row, and the recursion fills the rest;
every choice spans the same space.  The dimension is C(p+n, n) + C(p-1+n, n)
(Sec. 3).

Ordering: type 0 then type 1; inside a type by |beta| ascending, then beta in
descending lexicographic order.  Function 0 is the constant 1.

The first-order Trefftz fields are (v, sigma) = (dU/dt, -grad U) (Sec. 3,
the space W); the constant drops out, leaving N - 1 of them.

A polynomial is a dict {(k, alpha): Fraction} with alpha a tuple of length n.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from functools import lru_cache

import numpy as np


def multi_indices(n: int, deg: int):
    """All alpha in N^n with |alpha| = deg, in descending lexicographic order."""
    out = [a for a in itertools.product(range(deg + 1), repeat=n) if sum(a) == deg]
    out.sort(reverse=True)
    return out


def dim_U(n: int, p: int) -> int:
    from math import comb

    return comb(p + n, n) + (comb(p - 1 + n, n) if p >= 1 else 0)


SEED_KINDS = ("monomial", "legendre", "chebyshev")


def seed_polynomial_1d(kind: str, d: int):
    """Coefficients [c_0, ..., c_d] (Fractions) of the degree-d seed polynomial
    of one variable: x^d, the Legendre polynomial P_d by Bonnet's three-term
    recurrence (k+1) P_(k+1) = (2k+1) x P_k - k P_(k-1), or the Chebyshev
    polynomial T_d by T_(k+1) = 2x T_k - T_(k-1) (P_0 = T_0 = 1, P_1 = T_1 = x)."""
    if kind == "monomial":
        return [Fraction(0)] * d + [Fraction(1)]
    if kind not in SEED_KINDS:
        raise ValueError(f"unknown seed basis {kind!r}")
    prev, cur = [Fraction(1)], [Fraction(0), Fraction(1)]
    if d == 0:
        return prev
    for k in range(1, d):
        xcur = [Fraction(0)] + cur          # x * P_k
        nxt = [Fraction(0)] * (k + 2)
        for i, c in enumerate(xcur):
            nxt[i] += (Fraction(2 * k + 1, k + 1) if kind == "legendre" else Fraction(2)) * c
        for i, c in enumerate(prev):
            nxt[i] -= (Fraction(k, k + 1) if kind == "legendre" else Fraction(1)) * c
        prev, cur = cur, nxt
    return cur


def seed_polynomial(kind: str, beta):
    """The seed of multi-index beta as {alpha: Fraction}: the product over the
    variables of the one-variable seed polynomials of degrees beta_m."""
    poly = {(): Fraction(1)}
    for bm in beta:
        c1 = seed_polynomial_1d(kind, bm)
        poly = {a + (i,): ca * ci for a, ca in poly.items() for i, ci in enumerate(c1) if ci != 0}
    return {a: c for a, c in poly.items() if c != 0}


def _seeds(n: int, p: int):
    s = []
    for d in range(p + 1):
        for beta in multi_indices(n, d):
            s.append((0, beta))
    for d in range(p):
        for beta in multi_indices(n, d):
            s.append((1, beta))
    return s


@lru_cache(maxsize=None)
def trefftz_basis(n: int, p: int, seed: str = "monomial"):
    """List of dim_U(n, p) exact polynomials spanning U^p for c = 1, seeded
    by the spatial basis `seed` (one of SEED_KINDS)."""
    basis = []
    for typ, beta in _seeds(n, p):
        a = {}
        # seed: row k = typ holds the seed polynomial of beta, the other of
        # rows 0 and 1 is zero
        for alpha, c in seed_polynomial(seed, beta).items():
            a[(typ, alpha)] = c
        for k in range(2, p + 1):
            for d in range(0, p - k + 1):
                for alpha in multi_indices(n, d):
                    acc = Fraction(0)
                    for m in range(n):
                        up = list(alpha)
                        up[m] += 2
                        prev = a.get((k - 2, tuple(up)))
                        if prev:
                            acc += (alpha[m] + 1) * (alpha[m] + 2) * prev
                    if acc:
                        a[(k, alpha)] = acc / (k * (k - 1))
        basis.append({key: val for key, val in a.items() if val != 0})
    return tuple(basis)


def d_dt(poly):
    out = {}
    for (k, alpha), c in poly.items():
        if k >= 1:
            key = (k - 1, alpha)
            out[key] = out.get(key, 0) + k * c
    return {k: v for k, v in out.items() if v != 0}


def d_dx(poly, m):
    out = {}
    for (k, alpha), c in poly.items():
        if alpha[m] >= 1:
            al = list(alpha)
            al[m] -= 1
            key = (k, tuple(al))
            out[key] = out.get(key, 0) + alpha[m] * c
    return {k: v for k, v in out.items() if v != 0}


def first_order_fields(n: int, p: int, seed: str = "monomial"):
    """(v, sigma_1..sigma_n) = (dU/dt, -dU/dx_1, ..., -dU/dx_n) for each
    non-constant basis function of U^p (functions 1 .. N-1)."""
    out = []
    for b in trefftz_basis(n, p, seed)[1:]:
        comps = [d_dt(b)]
        for m in range(n):
            comps.append({k: -v for k, v in d_dx(b, m).items()})
        out.append(comps)
    return out


def eval_poly(poly, xh, th):
    """Evaluate an exact polynomial at float points: xh (Q, n), th (Q,)."""
    val = np.zeros(th.shape, dtype=np.float64)
    for (k, alpha), c in poly.items():
        term = np.full(th.shape, float(c))
        term = term * th ** k
        for m, am in enumerate(alpha):
            term = term * xh[:, m] ** am
        val = val + term
    return val
