"""Pins for the exact Trefftz basis (Sec. 3, eq. 3.1).

* Trefftz property, checked by applying the wave operator -Lap + d_tt to every
  basis polynomial in exact rational arithmetic (independent of the recursion).
* dimension: both printed forms of dim U^p (Sec. 3) and the L-shape DOF
  totals of Table 1, which are all multiples of dim U^3 in 2D = 16.
* linear independence (rank) and the seeds U(.,0), U_t(.,0).
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.trefftz import d_dt, d_dx, dim_U, first_order_fields, multi_indices, trefftz_basis

HERE = os.path.dirname(os.path.abspath(__file__))


def wave_operator(poly, n):
    out = {}
    for key, c in d_dt(d_dt(poly)).items():
        out[key] = out.get(key, 0) + c
    for m in range(n):
        for key, c in d_dx(d_dx(poly, m), m).items():
            out[key] = out.get(key, 0) - c
    return {k: v for k, v in out.items() if v != 0}


CASES = [(1, p) for p in range(1, 11)] + [(2, p) for p in range(1, 9)] + [(3, p) for p in range(1, 7)]


@pytest.mark.parametrize("n,p", CASES)
def test_basis_is_trefftz_exactly(n, p):
    for b in trefftz_basis(n, p):
        assert wave_operator(b, n) == {}


@pytest.mark.parametrize("n,p", CASES)
def test_dimension_both_printed_forms(n, p):
    N = len(trefftz_basis(n, p))
    assert N == math.comb(p + n, n) + math.comb(p - 1 + n, n)
    assert Fraction(2 * p + n, p) * math.comb(p - 1 + n, n) == N
    assert dim_U(n, p) == N
    # first-order space: the constant drops out
    assert len(first_order_fields(n, p)) == N - 1


@pytest.mark.parametrize("n,p", [(1, 6), (2, 4), (3, 3)])
def test_basis_linearly_independent(n, p):
    basis = trefftz_basis(n, p)
    keys = sorted({k for b in basis for k in b})
    M = np.array([[float(b.get(k, 0)) for k in keys] for b in basis])
    assert np.linalg.matrix_rank(M) == len(basis)


@pytest.mark.parametrize("n,p", [(1, 5), (2, 4), (3, 3)])
def test_seeds(n, p):
    basis = trefftz_basis(n, p)
    i = 0
    for typ, cap in ((0, p), (1, p - 1)):
        for d in range(cap + 1):
            for beta in multi_indices(n, d):
                b = basis[i]
                at0 = {a: c for (k, a), c in b.items() if k == 0}
                dt0 = {a: c for (k, a), c in b.items() if k == 1}
                if typ == 0:
                    assert at0 == {beta: 1} and dt0 == {}
                else:
                    assert at0 == {} and dt0 == {beta: 1}
                i += 1
    assert i == len(basis)


def test_worked_examples_1d():
    # x^3 + 3 x t^2 and x^2 t + t^3/3 solve u_tt = u_xx (checked by hand)
    basis = trefftz_basis(1, 3)
    assert basis[3] == {(0, (3,)): 1, (2, (1,)): 3}
    assert basis[6] == {(1, (2,)): 1, (3, (0,)): Fraction(1, 3)}


def test_table1_dofs_are_multiples_of_dim_U3_2d():
    vals = [int(l) for l in open(os.path.join(HERE, "golden", "table1_lshape_dofs.txt")) if l.strip() and not l.startswith("#")]
    assert len(vals) == 8
    N = dim_U(2, 3)
    assert N == 16
    assert all(v % N == 0 for v in vals)
    # the other candidate readings of the degree do not divide them all
    assert not all(v % dim_U(2, 4) == 0 for v in vals)
    assert not all(v % (dim_U(2, 4) - 1) == 0 for v in vals)
    assert not all(v % (3 * math.comb(3 + 2, 2)) == 0 for v in vals)
