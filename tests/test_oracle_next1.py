"""Pins of the oracle's Neumann faces (eq. 4.1, T^N), of the paper's recovery
of U with the extra terms for every test function (Sec. 5, read on the tent's
bottom facets) and of the U error (Sec. 6.6):

* polynomial reproduction: data from a Trefftz polynomial of degree <= p
  (plane-wave polynomials, independent of eq. 3.1) with g_N = sigma.n of the
  exact field on the Neumann facets and g_D = v on the others is reproduced to
  round-off, U included, with either recovery;
* global equivalence: the face-by-face assembly of the whole tent mesh
  (eq. 2.5 with F^N faces, and with the recovery terms of Sec. 5 added for
  every test function or for the constant only) solved at once equals the
  tent-by-tent solution;
* the per-tent energy balance with Neumann faces (dissipation beta (sigma.n)^2,
  data term g_N (beta sigma.n - v)) holds to round-off;
* the U error of a zero solution against the standing wave in closed form.
"""
import numpy as np
import pytest

from oracle.global_tdg import global_solve
from oracle.pitcher import pitch
from oracle.tdg import OracleTDG
from oracle.topology import Topology
from workloads import configs as C
from workloads import fields as F


def _kinds(coords, elems, c, rule):
    """Kind per boundary facet (Topology.boundary_facets order): Neumann where
    rule(facet centroid) holds."""
    topo = Topology(coords, elems, c)
    out = []
    for e, k in topo.boundary_facets():
        vs = [v for j, v in enumerate(topo.elems[e]) if j != k]
        out.append(1 if rule(topo.coords[vs].mean(axis=0)) else 0)
    return np.array(out)


def _gN(field, n):
    """sigma.n of the field on the faces of the unit square / cube / interval
    (outward normal from the side the point lies on)."""
    def g(x, t):
        s = field.sigma(x, t)
        out = np.zeros(len(x))
        for d in range(n):
            lo = np.abs(x[:, d]) < 1e-12
            hi = np.abs(x[:, d] - 1.0) < 1e-12
            out[lo] -= s[lo, d]
            out[hi] += s[hi, d]
        return out
    return g


CASES = {
    "1d_p3": lambda: (C.cfg1_standing_1d(n_elems=6, p=3), F.PolynomialPlaneWaves(1, 3, 2, seed=5),
                      lambda x: x[0] < 0.5),
    "2d_p3": lambda: (C.cfg2_plane_2d(m=5, p=3), F.PolynomialPlaneWaves(2, 3, 4, seed=6),
                      lambda x: x[0] < 1e-9 or x[1] < 1e-9),
    "2d_p4_two_speeds": lambda: (C.cfg4_interface_2d(m=7, p=2), None, lambda x: x[1] > 1 - 1e-9),
    "3d_p2": lambda: (C.cfg5_cube_3d(m=2, p=2, variant="b", regions=1), F.PolynomialPlaneWaves(3, 2, 4, seed=7, c=1.5),
                      lambda x: x[2] < 1e-9 or x[0] > 1 - 1e-9),
}


def _solve(pr, f, kinds, recover, p=None):
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=p or pr.p, q=pr.qpts, alpha=pr.alpha, beta=pr.beta,
                  gD=lambda x, t: f.v(x, t), gN=_gN(f, pr.n), bface_kind=kinds, recover=recover)
    X = o.quad_points()
    o.set_initial(f.v(X, 0.0), f.sigma(X, 0.0), f.U(X, 0.0))
    return o, tents


@pytest.mark.parametrize("recover", ["mean", "all"])
@pytest.mark.parametrize("name", ["1d_p3", "2d_p3", "3d_p2"])
def test_neumann_polynomial_reproduction(name, recover):
    pr, f, rule = CASES[name]()
    pr.T = min(pr.T, 0.4)
    kinds = _kinds(pr.coords, pr.elems, pr.c, rule)
    assert 0 < kinds.sum() < len(kinds)
    o, _ = _solve(pr, f, kinds, recover)
    o.run()
    X = o.quad_points()
    e_abs, e_rel = o.error(f.v(X, pr.T), f.sigma(X, pr.T))
    u_abs, u_rel = o.error_U(f.U(X, pr.T))
    assert e_rel < 1e-11, e_rel
    assert u_rel < 1e-11, u_rel


def test_neumann_data_matter():
    """Sanity of the pin: wrong Neumann data (sign flipped) is not reproduced."""
    pr, f, rule = CASES["2d_p3"]()
    pr.T = 0.4
    kinds = _kinds(pr.coords, pr.elems, pr.c, rule)
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    g = _gN(f, 2)
    o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=pr.p, q=pr.qpts, gD=lambda x, t: f.v(x, t),
                  gN=lambda x, t: -g(x, t), bface_kind=kinds)
    X = o.quad_points()
    o.set_initial(f.v(X, 0.0), f.sigma(X, 0.0), f.U(X, 0.0))
    o.run()
    assert o.error(f.v(X, pr.T), f.sigma(X, pr.T))[1] > 1e-4


@pytest.mark.parametrize("recover", ["mean", "all"])
@pytest.mark.parametrize("name", ["1d_p3", "2d_p3", "2d_p4_two_speeds"])
def test_global_equivalence_with_neumann_and_recovery(name, recover):
    pr, f, rule = CASES[name]()
    pr.T = min(pr.T, 0.3)
    f = f or pr.data
    kinds = _kinds(pr.coords, pr.elems, pr.c, rule)
    o, tents = _solve(pr, f, kinds, recover)
    o.run()
    X = o.quad_points()
    vT, sT, _, UT = global_solve(pr.coords, pr.elems, pr.c, tents, pr.p, pr.qpts, f.v(X, 0.0), f.sigma(X, 0.0),
                                 alpha=pr.alpha, beta=pr.beta, gD=lambda x, t: f.v(x, t), gN=_gN(f, pr.n),
                                 bface_kind=kinds, U0=f.U(X, 0.0), recover=recover)
    assert np.abs(vT - o.v).max() <= 1e-10 * np.abs(o.v).max()
    assert np.abs(sT - o.sig).max() <= 1e-10 * np.abs(o.sig).max()
    assert np.abs(UT - o.U).max() <= 1e-10 * np.abs(o.U).max()


def test_recoveries_differ_only_off_polynomials():
    """The two recoveries give the same (v, sigma) on Trefftz polynomial data
    (both exact) and different ones on non-polynomial data (the paper's form
    also moves the first-order rows)."""
    pr = C.cfg1_standing_1d(n_elems=8, p=3)
    pr.T = 0.5
    f = pr.data
    om, _ = _solve(pr, f, None, "mean")
    oa, _ = _solve(pr, f, None, "all")
    om.run()
    oa.run()
    d = np.abs(om.v - oa.v).max() / np.abs(om.v).max()
    assert 1e-10 < d < 1e-2, d


@pytest.mark.parametrize("name", ["2d_p3", "2d_p4_two_speeds"])
def test_energy_balance_with_neumann_faces(name):
    pr, f, rule = CASES[name]()
    pr.T = min(pr.T, 0.3)
    f = f or pr.data
    kinds = _kinds(pr.coords, pr.elems, pr.c, rule)
    o, _ = _solve(pr, f, kinds, "mean")
    d = o.run(want_diag=True)
    bal = max(abs(x["E_top"] - (x["E_bot_in"] - x["D_T"] + x["G_bnd"])) / abs(x["E_bot_in"]) for x in d)
    assert bal < 1e-12, bal
    assert all(x["D_T"] >= -1e-15 for x in d)


def test_u_error_closed_form():
    # zero U against U = sin(pi x) cos(pi t): ||U||^2 = cos^2(pi t) / 2 on [0, 1]
    pr = C.cfg1_standing_1d(n_elems=16)
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=3, q=10)
    X = o.quad_points()
    t = 0.3
    d, rel = o.error_U(pr.data.U(X, t))
    assert abs(d - abs(np.cos(np.pi * t)) / np.sqrt(2.0)) < 1e-13
    assert rel == pytest.approx(1.0)
