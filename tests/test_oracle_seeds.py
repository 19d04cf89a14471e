"""Pins of the oracle's choice of seed basis (Sec. 3: any polynomial basis of
the spatial variables seeds the recursion of eq. 3.1; Sec. 6.3 compares
monomials, Legendre and Chebyshev polynomials).

Each check is against something other than the oracle's own formula:
textbook coefficients and orthogonality of the seed families, the Trefftz
property and the initial rows in exact arithmetic, linearity of the
recursion (a seeded function is the same combination of monomial-seeded
functions, an independent route), the invariance of the discrete solution
under a change of basis of the same space, and the paper's finding of
Sec. 6.3 on the 1+1D standing wave of Sec. 6."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.global_tdg import global_solve
from oracle.pitcher import pitch
from oracle.tdg import OracleTDG
from oracle.trefftz import (SEED_KINDS, d_dt, d_dx, dim_U, multi_indices, seed_polynomial,
                            seed_polynomial_1d, trefftz_basis)
from workloads import configs as C
from workloads import fields as F
from workloads import meshes as M

# textbook closed forms, coefficients of x^0 .. x^d
LEGENDRE = [
    [Fr(1)],
    [Fr(0), Fr(1)],
    [Fr(-1, 2), Fr(0), Fr(3, 2)],
    [Fr(0), Fr(-3, 2), Fr(0), Fr(5, 2)],
    [Fr(3, 8), Fr(0), Fr(-30, 8), Fr(0), Fr(35, 8)],
    [Fr(0), Fr(15, 8), Fr(0), Fr(-70, 8), Fr(0), Fr(63, 8)],
]
CHEBYSHEV = [
    [1], [0, 1], [-1, 0, 2], [0, -3, 0, 4], [1, 0, -8, 0, 8], [0, 5, 0, -20, 0, 16],
]


def test_seed_polynomials_match_textbook_forms():
    for d in range(6):
        assert seed_polynomial_1d("legendre", d) == LEGENDRE[d]
        assert seed_polynomial_1d("chebyshev", d) == [Fr(c) for c in CHEBYSHEV[d]]
        assert seed_polynomial_1d("monomial", d) == [Fr(0)] * d + [Fr(1)]
    with pytest.raises(ValueError):
        seed_polynomial_1d("hermite", 2)


def test_legendre_orthogonal_and_chebyshev_cosine_identity():
    # int_-1^1 P_a P_b dx = 2/(2a+1) delta_ab, exactly
    def integral(c):
        return sum(ci * Fr(2, i + 1) for i, ci in enumerate(c) if i % 2 == 0)

    for a in range(9):
        for b in range(9):
            pa, pb = seed_polynomial_1d("legendre", a), seed_polynomial_1d("legendre", b)
            prod = [Fr(0)] * (a + b + 1)
            for i, x in enumerate(pa):
                for j, y in enumerate(pb):
                    prod[i + j] += x * y
            assert integral(prod) == (Fr(2, 2 * a + 1) if a == b else 0)
    # T_d(cos th) = cos(d th)
    th = np.linspace(0.0, np.pi, 37)
    for d in range(11):
        c = [float(x) for x in seed_polynomial_1d("chebyshev", d)]
        val = sum(ci * np.cos(th) ** i for i, ci in enumerate(c))
        assert np.abs(val - np.cos(d * th)).max() < 1e-12


def test_tensor_product_seed():
    s = seed_polynomial("legendre", (2, 1))
    # P_2(x) P_1(y) = (3/2 x^2 - 1/2) y
    assert s == {(2, 1): Fr(3, 2), (0, 1): Fr(-1, 2)}
    assert seed_polynomial("chebyshev", (0, 0, 3)) == {(0, 0, 3): Fr(4), (0, 0, 1): Fr(-3)}


@pytest.mark.parametrize("n,p", [(1, 6), (2, 4), (3, 3)])
@pytest.mark.parametrize("seed", ["legendre", "chebyshev"])
def test_seeded_functions_are_trefftz_with_the_seed_as_data(n, p, seed):
    basis = trefftz_basis(n, p, seed)
    assert len(basis) == dim_U(n, p)
    seeds = [(0, b) for d in range(p + 1) for b in multi_indices(n, d)] + \
            [(1, b) for d in range(p) for b in multi_indices(n, d)]
    for U, (typ, beta) in zip(basis, seeds):
        # U_tt - Lap U = 0 exactly
        res = dict(d_dt(d_dt(U)))
        for m in range(n):
            for k, v in d_dx(d_dx(U, m), m).items():
                res[k] = res.get(k, 0) - v
        assert all(v == 0 for v in res.values())
        # rows t^0 and t^1: the seed in row `typ`, zero in the other
        row = {typ: seed_polynomial(seed, beta), 1 - typ: {}}
        for k in (0, 1):
            got = {a: v for (kk, a), v in U.items() if kk == k}
            assert got == row[k]
        assert max(k + sum(a) for (k, a) in U) == typ + sum(beta)


@pytest.mark.parametrize("n,p", [(1, 7), (2, 5), (3, 3)])
@pytest.mark.parametrize("seed", ["legendre", "chebyshev"])
def test_seeded_function_is_the_combination_of_monomial_seeded_ones(n, p, seed):
    # the recursion is linear in its data: the function seeded by
    # b_beta = sum_gamma s_gamma x^gamma is sum_gamma s_gamma U_(typ, gamma)
    mono = trefftz_basis(n, p, "monomial")
    seeded = trefftz_basis(n, p, seed)
    seeds = [(0, b) for d in range(p + 1) for b in multi_indices(n, d)] + \
            [(1, b) for d in range(p) for b in multi_indices(n, d)]
    pos = {s: i for i, s in enumerate(seeds)}
    for i, (typ, beta) in enumerate(seeds):
        acc = {}
        for gamma, w in seed_polynomial(seed, beta).items():
            for k, v in mono[pos[(typ, gamma)]].items():
                acc[k] = acc.get(k, 0) + w * v
        assert {k: v for k, v in acc.items() if v != 0} == seeded[i]


def _tent_run(pr, f, seed, recover="mean"):
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=pr.p, q=pr.p, alpha=pr.alpha, beta=pr.beta,
                  gD=lambda x, t: f.v(x, t), recover=recover, seed=seed)
    X = o.quad_points()
    o.set_initial(f.v(X, 0.0), f.sigma(X, 0.0), f.U(X, 0.0))
    o.run()
    return o


@pytest.mark.parametrize("dim", ["1d", "2d", "3d"])
def test_solution_does_not_depend_on_the_seed_basis(dim):
    # the seeds span the same space, so every seed gives the same discrete
    # solution up to round-off (v, sigma and the recovered U)
    if dim == "1d":
        pr = C.cfg1_standing_1d(n_elems=8, p=4)
        recs = ("mean", "all")
    elif dim == "2d":
        pr = C.cfg2_plane_2d(m=4, p=3)
        pr.T = 0.3
        recs = ("mean",)
    else:
        pr = C.cfg5_cube_3d(m=1, p=2, variant="b")
        pr.T = 0.1
        recs = ("mean",)
    f = pr.data
    for rec in recs:
        ref = _tent_run(pr, f, "monomial", rec)
        for seed in ("legendre", "chebyshev"):
            o = _tent_run(pr, f, seed, rec)
            for a, b in ((o.v, ref.v), (o.sig, ref.sig), (o.U, ref.U)):
                assert np.abs(a - b).max() <= 1e-11 * max(1.0, np.abs(b).max())


def test_seed_invariance_with_interfaces_neumann_faces_and_the_paper_recovery():
    # two speeds (interface faces of Sec. 4.2), Neumann faces on y = 1 (eq. 4.1)
    # and the recovery of U with every test function (Sec. 5)
    from oracle.topology import Topology

    pr = C.cfg4_interface_2d(m=9, p=3)
    pr.T = 0.3
    f = pr.data
    topo = Topology(pr.coords, pr.elems, pr.c)
    kinds = []
    for e, k in topo.boundary_facets():
        cen = pr.coords[[v for j, v in enumerate(pr.elems[e]) if j != k]].mean(axis=0)
        kinds.append(1 if cen[1] > 1 - 1e-9 else 0)
    assert 0 < sum(kinds) < len(kinds)

    def gN(x, t):
        return np.where(np.abs(x[:, 1] - 1.0) < 1e-12, f.sigma(x, t)[:, 1], 0.0)

    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    out = []
    for seed in SEED_KINDS:
        o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=pr.p, q=pr.p, gD=lambda x, t: f.v(x, t), gN=gN,
                      bface_kind=kinds, recover="all", seed=seed)
        X = o.quad_points()
        o.set_initial(f.v(X, 0.0), f.sigma(X, 0.0), f.U(X, 0.0))
        o.run()
        out.append((o.v, o.sig, o.U))
    for got in out[1:]:
        for a, b in zip(got, out[0]):
            assert np.abs(a - b).max() <= 1e-11 * max(1.0, np.abs(b).max())


def _global_1d(p, seed, ne=8):
    coords, elems = M.interval_mesh(ne)
    c = np.ones(len(elems))
    f = F.PaperStandingWave(1)
    tents, lp = pitch(coords, elems, c, 1.0, 0.5)
    o = OracleTDG(coords, elems, c, tents, lp, p=p, q=p, seed=seed)
    X = o.quad_points()
    info = {}
    vT, sT, _ = global_solve(coords, elems, c, tents, p, p, f.v(X, 0.0), f.sigma(X, 0.0),
                             gD=lambda x, t: f.v(x, t), seed=seed, info=info)
    o.v, o.sig = vT, sT
    e_abs, _ = o.error(f.v(X, 1.0), f.sigma(X, 1.0))
    return e_abs, np.linalg.cond(info["A"].toarray())


def test_sec63_monomial_seeds_condition_best():
    # Sec. 6.3 on the 1+1D standing wave of Sec. 6 (8 elements, T = 1, global
    # system eq. 2.5): the three seeds give the same error at low degree, the
    # global matrix is better conditioned with monomial seeds than with
    # Legendre or Chebyshev ones, and at the highest degree the others lose
    # accuracy to round-off
    for p in (4, 6, 8):
        res = {s: _global_1d(p, s) for s in SEED_KINDS}
        em, cm = res["monomial"]
        el, cl = res["legendre"]
        ec, cc = res["chebyshev"]
        assert cm < cl < cc
        if p <= 6:
            assert abs(el - em) <= 1e-6 * em and abs(ec - em) <= 1e-6 * em
    em, cm = _global_1d(10, "monomial")
    ec, cc = _global_1d(10, "chebyshev")
    assert cc > 30 * cm
    assert ec > 3 * em
